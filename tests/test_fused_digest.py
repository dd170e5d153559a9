"""The J/K kernels' one-pass digestion (FusedDigest in gen/emit_staged.py),
compiled for the host with g++ and run on random integrals and a random
density.  It must add to J' and K' exactly the six contractions of the
8-fold symmetric Scatter (Alg. 2), written out here with numpy, for both
slice orders the kernels use: ket functions (lam, sig) as slices in the row
form, bra functions (mu, nu) in the chunk form.  The six-pass digestion it
replaces is checked against the same sums.  One lane: the wave's segmented
sums reduce to the lane's own value."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from paper_2605_10312_amd.gen.emit_staged import FusedDigest, slot_digestion

HOST_PRELUDE = r"""
#include <cmath>
#include <cstdint>
using std::fma;
struct HostPair { int x, y; };
struct HostShell { int sh_a; };
struct HostArgs { bool want_j, want_k; double *J, *K; };
static inline int hgp_seg_start(long long) { return 0; }
static inline bool hgp_seg_tail(long long) { return true; }
static inline double hgp_seg_sum(double v, int) { return v; }
static inline void atomicAdd(double *p, double v) { *p += v; }
#define HGP_STAGE(x) (void)(x)
"""


def _source(sizes, form):
    na, nb, nc, nd = sizes
    L = [HOST_PRELUDE,
         'extern "C" void digest(const double *I, const double *D, int N, int fa, int fb, int fc, int fd,',
         '                       double sj, double sk, int want_j, int want_k, double *J, double *K)',
         "{",
         "    HostArgs a{want_j != 0, want_k != 0, J, K};",
         "    HostPair pq{3, 5};",
         "    HostShell pk{2};",
         "    uint32_t li = 0;"]
    idx = lambda mu, nu, lam, sig: f"I[{((mu * nb + nu) * nc + lam) * nd + sig}]"
    if form == "slots":
        L += slot_digestion(na, nb, nc, nd, idx)
    else:
        outer, inner = (2, 3) if form == "row" else (0, 1)
        fd_ = FusedDigest(sizes, outer, inner)
        L += fd_.prologue()
        for p in range(sizes[outer]):
            L += fd_.outer_begin(p)
            for q in range(sizes[inner]):
                if form == "row":
                    val = lambda r, s, p=p, q=q: idx(r, s, p, q)
                else:
                    val = lambda r, s, p=p, q=q: idx(p, q, r, s)
                L += fd_.slice(p, q, val)
            L += fd_.outer_end(p)
        L += fd_.epilogue()
    L.append("}")
    return "\n".join(L) + "\n"


def _reference(I, D, f, sj, sk, N):
    fa, fb, fc, fd = f
    na, nb, nc, nd = I.shape
    J = np.zeros((N, N))
    K = np.zeros((N, N))
    A, B, C, E = (slice(fa, fa + na), slice(fb, fb + nb), slice(fc, fc + nc), slice(fd, fd + nd))
    J[A, B] += sj * np.einsum("mnls,ls->mn", I, D[C, E])
    J[C, E] += sj * np.einsum("mnls,mn->ls", I, D[A, B])
    K[A, C] += sk * np.einsum("mnls,ns->ml", I, D[B, E])
    K[B, C] += sk * np.einsum("mnls,ms->nl", I, D[A, E])
    K[A, E] += sk * np.einsum("mnls,nl->ms", I, D[B, C])
    K[B, E] += sk * np.einsum("mnls,ml->ns", I, D[A, C])
    return J, K


@pytest.mark.parametrize("sizes", [(5, 5, 5, 5), (5, 3, 5, 3), (5, 5, 5, 1), (7, 1, 3, 3), (1, 1, 1, 1)])
@pytest.mark.parametrize("form", ["row", "chunk", "slots"])
def test_digestion_matches_the_six_contractions(tmp_path, sizes, form):
    src = tmp_path / "dg.cpp"
    src.write_text(_source(sizes, form))
    lib = tmp_path / "libdg.so"
    subprocess.run(["g++", "-O1", "-shared", "-fPIC", "-o", str(lib), str(src)], check=True)
    dg = ctypes.CDLL(str(lib))
    rng = np.random.default_rng(sum(sizes) * 7 + len(form))
    N = 40
    I = rng.standard_normal(sizes)
    D = rng.standard_normal((N, N))
    D = D + D.T
    f = (1, 9, 17, 30)                       # the four shells' first functions
    p = lambda x: x.ctypes.data_as(ctypes.c_void_p)
    for want_j, want_k in ((1, 1), (1, 0), (0, 1)):
        J = np.zeros((N, N))
        K = np.zeros((N, N))
        sj, sk = (0.75 if want_j else 0.0), (0.375 if want_k else 0.0)
        dg.digest(p(I), p(D), ctypes.c_int(N), *[ctypes.c_int(x) for x in f], ctypes.c_double(sj),
                  ctypes.c_double(sk), ctypes.c_int(want_j), ctypes.c_int(want_k), p(J), p(K))
        Jr, Kr = _reference(I, D, f, sj, sk, N)
        assert np.abs(J - Jr).max() <= 1e-12 and np.abs(K - Kr).max() <= 1e-12, (want_j, want_k)
