"""CPU oracle for contracted ERIs and J/K -- test infrastructure only.

Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package.  The HIP library never calls it
and shares no code with it (the two share only the seeded input generators in
``workloads``, which hold none of the method's arithmetic).

The arithmetic lives in ``oracle.c`` (plain C, FP64, OpenMP), built twice: a
double build (``liboracle.so``) and a long-double build (``liboracle_ld.so``)
used to estimate the double build's own rounding error.  This module only
marshals numpy arrays into those calls.

Pins (tests/test_oracle_*.py) tie it to things other than itself: mpmath's
confluent hypergeometric form and erf for the Boys function, the closed-form
(ss|ss), Gauss-Hermite/Rys-variable quadrature of the Coulomb operator for
low-l primitive integrals, sphere-sampled real spherical harmonics for the
shell transformation, and the invariances of the exact integrals.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIBS = {"double": os.path.join(_HERE, "liboracle.so"), "long double": os.path.join(_HERE, "liboracle_ld.so")}


def build(force: bool = True) -> None:
    """Compile both builds of the oracle with gcc (OpenMP)."""
    for kind, out in _LIBS.items():
        if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(_SRC):
            continue
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=gnu11", "-Wall", "-o", out + ".tmp", _SRC, "-lm"]
        if kind == "long double":
            cmd.insert(1, "-DORACLE_LD")
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)


_cache: dict = {}


def _lib(precision: str = "double"):
    if precision not in _cache:
        path = _LIBS[precision]
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
            build(force=False)
        lib = ctypes.CDLL(path)
        pfx = "oracle_ld_" if precision == "long double" else "oracle_"
        _cache[precision] = (lib, pfx)
    return _cache[precision]


def _fn(name: str, precision: str):
    lib, pfx = _lib(precision)
    f = getattr(lib, pfx + name)
    f.restype = ctypes.c_int
    return f


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with status {rc}")


def _basis_args(basis):
    l = np.ascontiguousarray(basis.l, dtype=np.int32)
    npr = np.ascontiguousarray(basis.nprim, dtype=np.int32)
    cen = np.ascontiguousarray(basis.centers, dtype=np.float64)
    ex = np.ascontiguousarray(basis.exps, dtype=np.float64)
    co = np.ascontiguousarray(basis.coefs, dtype=np.float64)
    keep = (l, npr, cen, ex, co)
    return keep, [ctypes.c_int(int(l.shape[0])), _p(l), _p(npr), _p(cen), _p(ex), _p(co)]


def nsph(l: int) -> int:
    return 2 * l + 1


def ncart(l: int) -> int:
    return (l + 1) * (l + 2) // 2


def boys(mmax: int, T: float, precision: str = "double") -> np.ndarray:
    out = np.zeros(mmax + 1)
    _check(_fn("boys", precision)(ctypes.c_int(mmax), ctypes.c_double(T), _p(out)), "boys")
    return out


def sph_matrix(l: int, precision: str = "double") -> np.ndarray:
    out = np.zeros((nsph(l), ncart(l)))
    _check(_fn("sph_matrix", precision)(ctypes.c_int(l), _p(out)), "sph_matrix")
    return out


def norm_coefs(l: int, exps, coefs, precision: str = "double") -> np.ndarray:
    ex = np.ascontiguousarray(exps, np.float64)
    co = np.ascontiguousarray(coefs, np.float64)
    out = np.zeros_like(ex)
    _check(_fn("norm_coefs", precision)(ctypes.c_int(l), ctypes.c_int(len(ex)), _p(ex), _p(co), _p(out)), "norm_coefs")
    return out


def prim_cart_eri(ls, centers, alphas, precision: str = "double") -> np.ndarray:
    """Unnormalised primitive Cartesian block (unit coefficients)."""
    cen = np.ascontiguousarray(centers, np.float64).reshape(12)
    al = np.ascontiguousarray(alphas, np.float64).reshape(4)
    out = np.zeros([ncart(x) for x in ls])
    rc = _fn("prim_cart_eri", precision)(*[ctypes.c_int(int(x)) for x in ls], _p(cen), _p(al), _p(out))
    _check(rc, "prim_cart_eri")
    return out


def eri_shell_quartet(basis, i, j, k, l, precision: str = "double") -> np.ndarray:
    keep, args = _basis_args(basis)
    shape = [nsph(int(basis.l[s])) for s in (i, j, k, l)]
    out = np.zeros(shape)
    rc = _fn("eri_shell_quartet", precision)(*args, *[ctypes.c_int(int(s)) for s in (i, j, k, l)], _p(out))
    _check(rc, "eri_shell_quartet")
    return out


def eri_deriv_shell_quartet(basis, i, j, k, l, precision: str = "double") -> np.ndarray:
    """First derivatives of the spherical block (ij|kl) with respect to the
    centres of shells i, j, k, l: array [4 centres, 3 axes, ni, nj, nk, nl]."""
    keep, args = _basis_args(basis)
    shape = [4, 3] + [nsph(int(basis.l[s])) for s in (i, j, k, l)]
    out = np.zeros(shape)
    rc = _fn("eri_deriv_shell_quartet", precision)(*args, *[ctypes.c_int(int(s)) for s in (i, j, k, l)], _p(out))
    _check(rc, "eri_deriv_shell_quartet")
    return out


def eri_prim_quartets(ls, centers, exps, precision: str = "double") -> np.ndarray:
    """centers [n,4,3] bohr, exps [n,4]; normalised primitives; spherical blocks [n, ...]."""
    cen = np.ascontiguousarray(centers, np.float64)
    ex = np.ascontiguousarray(exps, np.float64)
    n = cen.shape[0]
    out = np.zeros([n] + [nsph(int(x)) for x in ls])
    rc = _fn("eri_prim_quartets", precision)(*[ctypes.c_int(int(x)) for x in ls], ctypes.c_int64(n),
                                              _p(cen), _p(ex), _p(out))
    _check(rc, "eri_prim_quartets")
    return out


def schwarz(basis, precision: str = "double") -> np.ndarray:
    keep, args = _basis_args(basis)
    out = np.zeros((basis.nshell, basis.nshell))
    _check(_fn("schwarz", precision)(*args, _p(out)), "schwarz")
    return out


def jk(basis, D, tau: float = 0.0, precision: str = "double"):
    keep, args = _basis_args(basis)
    N = basis.nbf
    Dm = np.ascontiguousarray(D, np.float64)
    assert Dm.shape == (N, N)
    J = np.zeros((N, N))
    K = np.zeros((N, N))
    rc = _fn("jk", precision)(*args, _p(Dm), ctypes.c_double(tau), _p(J), _p(K))
    _check(rc, "jk")
    return J, K


def jk_blocks(basis, D, pairs, tau: float = 0.0, precision: str = "double"):
    """Direct J/K blocks for shell pairs [(P,Q), ...]: returns lists of arrays."""
    keep, args = _basis_args(basis)
    pr = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
    sizes = [nsph(int(basis.l[p])) * nsph(int(basis.l[q])) for p, q in pr]
    Jo = np.zeros(sum(sizes))
    Ko = np.zeros(sum(sizes))
    Dm = np.ascontiguousarray(D, np.float64)
    rc = _fn("jk_blocks", precision)(*args, _p(Dm), ctypes.c_double(tau), ctypes.c_int(len(pr)), _p(pr),
                                     _p(Jo), _p(Ko))
    _check(rc, "jk_blocks")
    Js, Ks, off = [], [], 0
    for (p, q), s in zip(pr, sizes):
        shp = (nsph(int(basis.l[p])), nsph(int(basis.l[q])))
        Js.append(Jo[off:off + s].reshape(shp))
        Ks.append(Ko[off:off + s].reshape(shp))
        off += s
    return Js, Ks


def eri_tensor(basis, precision: str = "double") -> np.ndarray:
    keep, args = _basis_args(basis)
    N = basis.nbf
    out = np.zeros((N, N, N, N))
    _check(_fn("eri_tensor", precision)(*args, _p(out)), "eri_tensor")
    return out


def eri_quartet_list(basis, quartets, precision: str = "double"):
    """Evaluate the listed shell quartets; returns (integrals evaluated, checksum)."""
    keep, args = _basis_args(basis)
    q = np.ascontiguousarray(np.asarray(quartets, dtype=np.int32).reshape(-1, 4))
    cnt = ctypes.c_int64()
    chk = ctypes.c_double()
    rc = _fn("eri_quartet_list", precision)(*args, ctypes.c_int64(q.shape[0]), _p(q), ctypes.byref(cnt),
                                             ctypes.byref(chk))
    _check(rc, "eri_quartet_list")
    return cnt.value, chk.value


def num_threads(precision: str = "double") -> int:
    return int(_fn("num_threads", precision)())
