"""Python binding of libhgp.so (include/hgp.h): argument marshalling only.

Every computation runs in the library's HIP kernels on the GPU.  Device
buffers are torch tensors (``data_ptr()``) and streams are torch streams
(``cuda_stream``); torch provides memory and streams, nothing else.  When the
library is missing this module raises instead of falling back to anything.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# HGP_LIB names another build of the library (the autotuner times variant builds this way)
LIB_PATH = os.environ.get("HGP_LIB") or os.path.join(_HERE, "libhgp.so")

STATUS = {0: "HGP_OK", -1: "HGP_E_INVALID", -2: "HGP_E_UNSUPPORTED_L", -3: "HGP_E_OOM", -4: "HGP_E_DEVICE",
          -5: "HGP_E_STATE"}
STATUS_OOM = -3
HGP_NORMALIZE = 1
HGP_FP64 = 0
HGP_MIXED = 1
MIXED_THETA_DEFAULT = 1e-10     # HGP_MIXED_THETA_DEFAULT in include/hgp.h

# exported symbol -> (restype, argtypes)
_vp, _i32, _i64, _d, _sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
SIGNATURES = {
    "hgp_version": (_i32, []),
    "hgp_max_l": (_i32, []),
    "hgp_basis_create": (ctypes.c_int, [_i32, _vp, _vp, _vp, _vp, _vp, _i32, ctypes.POINTER(_vp)]),
    "hgp_basis_nbf": (ctypes.c_int, [_vp, ctypes.POINTER(_i32), _vp]),
    "hgp_basis_destroy": (ctypes.c_int, [_vp]),
    "hgp_plan_create": (ctypes.c_int, [_vp, _d, _i32, _sz, _vp, ctypes.POINTER(_vp)]),
    "hgp_plan_create_mixed": (ctypes.c_int, [_vp, _d, _d, _sz, _vp, ctypes.POINTER(_vp)]),
    "hgp_plan_create_multi": (ctypes.c_int, [_vp, _i32, _d, _d, _sz, _vp, ctypes.POINTER(_vp)]),
    "hgp_jk_multi": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "hgp_batch_create": (ctypes.c_int, [_vp, _i32, _vp, _vp, _vp, ctypes.POINTER(_vp)]),
    "hgp_batch_run": (ctypes.c_int, [_vp, _vp]),
    "hgp_batch_destroy": (ctypes.c_int, [_vp]),
    "hgp_plan_class_precision": (ctypes.c_int, [_vp, _i32, ctypes.POINTER(_i32)]),
    "hgp_plan_destroy": (ctypes.c_int, [_vp]),
    "hgp_plan_stats": (ctypes.c_int, [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_i64)]),
    "hgp_plan_prim_stats": (ctypes.c_int, [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64)]),
    "hgp_plan_stream_stats": (ctypes.c_int, [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_i64)]),
    "hgp_plan_num_classes": (_i32, [_vp]),
    "hgp_plan_class_info": (ctypes.c_int, [_vp, _i32, _vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64),
                                           ctypes.POINTER(_d), ctypes.POINTER(_d), ctypes.POINTER(_i32)]),
    "hgp_plan_schwarz": (ctypes.c_int, [_vp, _vp]),
    "hgp_plan_set_timing": (ctypes.c_int, [_vp, _i32]),
    "hgp_plan_class_timing": (ctypes.c_int, [_vp, _i32, _i32, ctypes.POINTER(_i64), ctypes.POINTER(_d)]),
    "hgp_jk": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "hgp_eri_shell_quartets": (ctypes.c_int, [_vp, _i64, _vp, _vp, _vp, _vp]),
    "hgp_eri_deriv_shell_quartets": (ctypes.c_int, [_vp, _i64, _vp, _vp, _vp, _vp]),
    "hgp_deriv_max_l": (_i32, []),
    "hgp_eri_prim_quartets": (ctypes.c_int, [_i32, _i32, _i32, _i32, _i64, _vp, _vp, _vp, _i32, _vp]),
    "hgp_eri_prim_quartets_noalloc": (ctypes.c_int, [_i32, _i32, _i32, _i32, _i64, _vp, _vp, _vp, _i32, _vp]),
    "hgp_eri_prim_quartets_noalloc_max": (_i64, [_i32, _i32, _i32, _i32]),
    "hgp_class_form": (ctypes.c_int, [_i32, _i32, _i32, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
    "hgp_last_error": (ctypes.c_char_p, []),
}

_lib = None


class HGPError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def lib():
    """Load libhgp.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2605_10312_amd.build`")
        # torch ships its own HIP runtime.  Loading torch first makes the
        # library bind to that same runtime; loaded the other way round, the
        # process ends up with two runtimes and the library's sees no device.
        import torch  # noqa: F401
        h = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(h, name)
            fn.restype = res
            fn.argtypes = args
        _lib = h
    return _lib


def _check(rc):
    if rc != 0:
        raise HGPError(rc, lib().hgp_last_error().decode())


def _stream_ptr(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


def _dptr(t, dtype=None):
    """Device pointer of a contiguous CUDA tensor (None -> NULL)."""
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"expected dtype {dtype}, got {t.dtype}")
    return ctypes.c_void_p(t.data_ptr())


def _host(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


class Basis:
    """hgp_basis: shells l[n], nprim[n], centres [n,3] (bohr), exponents and
    coefficients (flat, shell by shell); raw coefficients normalised by the
    library (normalize=True, HGP_NORMALIZE) or used as given."""

    def __init__(self, l, nprim, centers, exps, coefs, normalize: bool = True):
        self._keep = [_host(l, np.int32), _host(nprim, np.int32), _host(centers, np.float64),
                      _host(exps, np.float64), _host(coefs, np.float64)]
        ptrs = [a.ctypes.data_as(ctypes.c_void_p) for a in self._keep]
        h = ctypes.c_void_p()
        _check(lib().hgp_basis_create(int(self._keep[0].shape[0]), *ptrs, HGP_NORMALIZE if normalize else 0,
                                      ctypes.byref(h)))
        self.handle = h
        n = ctypes.c_int32()
        self.shell_offsets = np.zeros(self._keep[0].shape[0] + 1, np.int32)
        _check(lib().hgp_basis_nbf(h, ctypes.byref(n), self.shell_offsets.ctypes.data_as(ctypes.c_void_p)))
        self.nbf = int(n.value)
        self.l = self._keep[0]

    @classmethod
    def from_workload(cls, b):
        return cls(b.l, b.nprim, b.centers, b.exps, b.coefs)

    def close(self):
        if getattr(self, "handle", None):
            lib().hgp_basis_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """hgp_plan: pairs, Schwarz factors and screened class quartet lists."""

    def __init__(self, basis: Basis, tau: float = 1e-12, hbm_budget: int = 0, stream=None, theta: float = 0.0):
        """theta > tau: mixed precision, quartets with tau <= Q_ab Q_cd < theta
        of register-tier classes use FP32 VRR and primitive contraction; HRR, Boys
        and J/K stay FP64 (hgp_plan_create_mixed)."""
        self.basis = basis
        h = ctypes.c_void_p()
        _check(lib().hgp_plan_create_mixed(basis.handle, float(tau), float(theta), int(hbm_budget),
                                           ctypes.c_void_p(_stream_ptr(stream)), ctypes.byref(h)))
        self.handle = h

    def stats(self):
        k, t, b = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().hgp_plan_stats(self.handle, ctypes.byref(k), ctypes.byref(t), ctypes.byref(b)))
        pk, pt = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().hgp_plan_prim_stats(self.handle, ctypes.byref(pk), ctypes.byref(pt)))
        qs, ch, cap = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().hgp_plan_stream_stats(self.handle, ctypes.byref(qs), ctypes.byref(ch), ctypes.byref(cap)))
        return {"quartets_kept": k.value, "quartets_total": t.value, "device_bytes": b.value,
                "prim_pairs_kept": pk.value, "prim_pairs_total": pt.value, "quartets_streamed": qs.value,
                "stream_chunks": ch.value, "chunk_capacity": cap.value}

    def classes(self):
        out = []
        for c in range(lib().hgp_plan_num_classes(self.handle)):
            ls = np.zeros(4, np.int32)
            nq, npq, vf, pf = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
            tier = ctypes.c_int32()
            _check(lib().hgp_plan_class_info(self.handle, c, ls.ctypes.data_as(ctypes.c_void_p), ctypes.byref(nq),
                                             ctypes.byref(npq), ctypes.byref(vf), ctypes.byref(pf), ctypes.byref(tier)))
            bits = ctypes.c_int32()
            _check(lib().hgp_plan_class_precision(self.handle, c, ctypes.byref(bits)))
            out.append({"ls": tuple(int(x) for x in ls), "quartets": nq.value, "prim_quartets": npq.value,
                        "vrr_flops": vf.value, "phase2_flops": pf.value, "tier": tier.value, "bits": bits.value})
        return out

    def schwarz(self):
        """Schwarz factors by shell pair, [nshell, nshell]."""
        n = int(self.basis.l.shape[0]) if self.basis is not None else sum(int(b.l.shape[0]) for b in self.bases)
        q = np.zeros((n, n))
        _check(lib().hgp_plan_schwarz(self.handle, q.ctypes.data_as(ctypes.c_void_p)))
        return q

    def set_timing(self, enable: bool):
        _check(lib().hgp_plan_set_timing(self.handle, 1 if enable else 0))

    def class_timing(self):
        """Per class: {ls, tier, kernels: [(launches, total_ms) for kernel 0, 1]},
        waiting for the recorded events.  Kernel 0 is the register tier's
        kernel or a staged class's Phase-1 kernel, kernel 1 a staged class's
        Phase-2 + digestion kernel."""
        out = []
        for c, info in enumerate(self.classes()):
            ks = []
            for k in (0, 1):
                n, ms = ctypes.c_int64(), ctypes.c_double()
                _check(lib().hgp_plan_class_timing(self.handle, c, k, ctypes.byref(n), ctypes.byref(ms)))
                ks.append((n.value, ms.value))
            out.append({"ls": info["ls"], "tier": info["tier"], "kernels": ks})
        return out

    @classmethod
    def multi(cls, bases, tau: float = 1e-12, theta: float = 0.0, hbm_budget: int = 0, stream=None):
        """One plan over several independent systems (hgp_plan_create_multi):
        each class runs as one launch over the quartets of every system."""
        self = cls.__new__(cls)
        self.basis = None
        self.bases = list(bases)
        arr = (ctypes.c_void_p * len(self.bases))(*[b.handle.value for b in self.bases])
        h = ctypes.c_void_p()
        _check(lib().hgp_plan_create_multi(arr, len(self.bases), float(tau), float(theta), int(hbm_budget),
                                           ctypes.c_void_p(_stream_ptr(stream)), ctypes.byref(h)))
        self.handle = h
        return self

    def jk(self, D, J=None, K=None, stream=None):
        """Enqueue J/K for device density D into device J and/or K (overwritten)."""
        import torch
        _check(lib().hgp_jk(self.handle, _dptr(D, torch.float64), _dptr(J, torch.float64), _dptr(K, torch.float64),
                            ctypes.c_void_p(_stream_ptr(stream))))

    def jk_multi(self, Ds, Js=None, Ks=None, stream=None):
        """J/K of every system of a multi-system plan: lists of device tensors
        (Js or Ks None to skip)."""
        import torch
        n = len(Ds)
        arr = lambda xs: (ctypes.c_void_p * n)(*[_dptr(x, torch.float64) for x in xs])
        _check(lib().hgp_jk_multi(self.handle, arr(Ds), None if Js is None else arr(Js),
                                  None if Ks is None else arr(Ks), ctypes.c_void_p(_stream_ptr(stream))))

    def close(self):
        if getattr(self, "handle", None):
            lib().hgp_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def eri_shell_quartets(basis: Basis, quartets, offsets, out, stream=None, deriv=False):
    """Spherical blocks of the listed shell quartets into device tensor `out`.
    quartets [nq, 4] (int32) and offsets [nq] (int64, elements) are device
    tensors, or host arrays that are copied to the device first.  deriv: the
    first derivatives instead, 12 blocks [position][axis] a quartet
    (hgp_eri_deriv_shell_quartets)."""
    import torch
    made = []

    def dev(a, np_dt, t_dt):
        if isinstance(a, torch.Tensor) and a.is_cuda:
            if a.dtype != t_dt:
                raise ValueError(f"expected dtype {t_dt}, got {a.dtype}")
            return a.contiguous()
        t = torch.from_numpy(_host(a, np_dt)).to("cuda")      # a blocking copy
        made.append(t)
        return t
    q = dev(quartets, np.int32, torch.int32).reshape(-1, 4)
    off = dev(offsets, np.int64, torch.int64).reshape(-1)
    if off.shape[0] != q.shape[0]:
        raise ValueError("one offset per quartet")
    sp = _stream_ptr(stream)
    fn = lib().hgp_eri_deriv_shell_quartets if deriv else lib().hgp_eri_shell_quartets
    _check(fn(basis.handle, int(q.shape[0]), _dptr(q), _dptr(off), _dptr(out, torch.float64), ctypes.c_void_p(sp)))
    if made and sp != torch.cuda.current_stream().cuda_stream:
        torch.cuda.synchronize()     # the copies are freed on return: let the other stream finish reading them


class Batch:
    """hgp_batch: the J/K builds of several plans captured as one HIP graph
    (one branch per system).  D, J, K: lists of device tensors per plan (J or
    K entries may be None); run() replays the graph on the stream."""

    def __init__(self, plans, D, J, K):
        import torch
        n = len(plans)
        self._keep = (list(plans), list(D), list(J), list(K))
        arr = lambda xs: (ctypes.c_void_p * n)(*[None if x is None else _dptr(x, torch.float64) for x in xs])
        self._arrays = (ctypes.c_void_p * n)(*[p.handle.value for p in plans]), arr(D), arr(J), arr(K)
        h = ctypes.c_void_p()
        _check(lib().hgp_batch_create(self._arrays[0], n, self._arrays[1], self._arrays[2], self._arrays[3],
                                      ctypes.byref(h)))
        self.handle = h

    def run(self, stream=None):
        _check(lib().hgp_batch_run(self.handle, ctypes.c_void_p(_stream_ptr(stream))))

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().hgp_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def eri_prim_quartets(ls, centers, exps, out, stream=None, precision=None):
    """n normalised primitive quartets of class ls: device centres [n,4,3],
    exponents [n,4] and output [n, nsph...].  precision HGP_FP64 (default)
    or HGP_MIXED."""
    import torch
    n = int(centers.shape[0])
    prec = HGP_FP64 if precision is None else int(precision)
    _check(lib().hgp_eri_prim_quartets(*[int(x) for x in ls], n, _dptr(centers, torch.float64),
                                       _dptr(exps, torch.float64), _dptr(out, torch.float64), prec,
                                       ctypes.c_void_p(_stream_ptr(stream))))


def eri_prim_quartets_noalloc(ls, centers, exps, out, stream=None):
    """eri_prim_quartets through the entry point that allocates nothing (the
    library's fixed per-device buffer; see hgp_eri_prim_quartets_noalloc)."""
    import torch
    n = int(centers.shape[0])
    _check(lib().hgp_eri_prim_quartets_noalloc(*[int(x) for x in ls], n, _dptr(centers, torch.float64),
                                               _dptr(exps, torch.float64), _dptr(out, torch.float64), HGP_FP64,
                                               ctypes.c_void_p(_stream_ptr(stream))))


def class_form(ls):
    """(tier, has_fp32) of class ls in this library."""
    tier, f32 = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().hgp_class_form(*[int(x) for x in ls], ctypes.byref(tier), ctypes.byref(f32)))
    return int(tier.value), bool(f32.value)


def class_has_fp32(ls) -> bool:
    return class_form(ls)[1]


def eri_prim_quartets_noalloc_max(ls) -> int:
    return int(lib().hgp_eri_prim_quartets_noalloc_max(*[int(x) for x in ls]))


def max_l() -> int:
    return int(lib().hgp_max_l())


def deriv_max_l() -> int:
    return int(lib().hgp_deriv_max_l())
