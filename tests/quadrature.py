"""Brute-force reference integrals used to pin the oracle (test helper).

Nothing here follows the HGP recurrences.  The Coulomb operator is written as
1/r12 = (2/sqrt(pi)) int_0^inf exp(-u^2 r12^2) du; for each u the six-
dimensional integral of Cartesian Gaussians factorises over x, y, z into
two-dimensional Gaussian-times-polynomial integrals, which tensor
Gauss-Hermite quadrature (after a Cholesky change of variables) evaluates
exactly.  The u-integral is done with Gauss-Legendre nodes after the change of
variables u = s t / sqrt(1 - t^2), under which the integrand is smooth on
[0, 1]; the interval is split near the peak of exp(-T t^2).
"""
import math

import numpy as np

_GH_X, _GH_W = np.polynomial.hermite.hermgauss(10)     # exact to degree 19 per variable
_GL_X, _GL_W = np.polynomial.legendre.leggauss(160)


def _cart_list(l):
    return [(x, y, l - x - y) for x in range(l, -1, -1) for y in range(l - x, -1, -1)]


def _axis_table(u, ex, cen, lmax):
    """T[i,j,k,l,u] = int int (x1-A)^i (x1-B)^j (x2-C)^k (x2-D)^l
    exp(-a(x1-A)^2 - b(x1-B)^2 - c(x2-C)^2 - d(x2-D)^2 - u^2 (x1-x2)^2) dx1 dx2
    for one Cartesian axis (cen: the four centre coordinates on this axis)."""
    a, b, c, d = ex
    A, B, C, D = cen
    p, q = a + b, c + d
    P, Q = (a * A + b * B) / p, (c * C + d * D) / q
    const0 = -a * b / p * (A - B) ** 2 - c * d / q * (C - D) ** 2
    u2 = u ** 2
    m11, m22, m12 = p + u2, q + u2, -u2
    det = m11 * m22 - m12 * m12
    h1, h2 = p * P, q * Q
    mu1 = (m22 * h1 - m12 * h2) / det
    mu2 = (m11 * h2 - m12 * h1) / det
    const = h1 * mu1 + h2 * mu2 - p * P * P - q * Q * Q + const0
    l11 = np.sqrt(m11)
    l21 = m12 / l11
    l22 = np.sqrt(m22 - l21 * l21)
    y1 = _GH_X[None, :, None]
    y2 = _GH_X[None, None, :]
    # x - mu = L^{-T} y with L the lower Cholesky factor of M
    x2 = mu2[:, None, None] + y2 / l22[:, None, None]
    x1 = mu1[:, None, None] + (y1 - l21[:, None, None] * (x2 - mu2[:, None, None])) / l11[:, None, None]
    w = (_GH_W[:, None] * _GH_W[None, :])[None]
    pref = np.exp(const) / (l11 * l22)
    la, lb, lc, ld = lmax
    pa = np.stack([(x1 - A) ** i for i in range(la + 1)])
    pb = np.stack([(x1 - B) ** i for i in range(lb + 1)])
    pc = np.stack([(x2 - C) ** i for i in range(lc + 1)])
    pd = np.stack([(x2 - D) ** i for i in range(ld + 1)])
    t = np.einsum("iuxy,juxy,kuxy,luxy,uxy->ijklu", pa, pb, pc, pd, np.broadcast_to(w, x1.shape), optimize=True)
    return t * pref[None, None, None, None, :]


def prim_cart_eri(ls, centers, alphas):
    """Unnormalised primitive Cartesian block (ab|cd), unit coefficients,
    Cartesian order x-descending then y-descending within each shell."""
    centers = np.asarray(centers, float).reshape(4, 3)
    alphas = np.asarray(alphas, float).reshape(4)
    a, b, c, d = alphas
    p, q = a + b, c + d
    s = math.sqrt(p * q / (p + q))
    P = (a * centers[0] + b * centers[1]) / p
    Q = (c * centers[2] + d * centers[3]) / q
    T = s * s * float(np.sum((P - Q) ** 2))
    # u = s t / sqrt(1 - t^2): split t at the width of exp(-T t^2)
    t0 = min(0.999, 6.0 / math.sqrt(T)) if T > 36 else 0.999
    nodes, weights = [], []
    for lo, hi in ((0.0, t0), (t0, 1.0)):
        nodes.append(0.5 * (hi - lo) * _GL_X + 0.5 * (hi + lo))
        weights.append(0.5 * (hi - lo) * _GL_W)
    t = np.concatenate(nodes)
    wt = np.concatenate(weights)
    u = s * t / np.sqrt(1 - t * t)
    jac = s / (1 - t * t) ** 1.5
    tabs = [_axis_table(u, alphas, centers[:, ax], ls) for ax in range(3)]
    cl = [_cart_list(l) for l in ls]
    out = np.zeros([len(c_) for c_ in cl])
    for ia, ca in enumerate(cl[0]):
        for ib, cb in enumerate(cl[1]):
            for ic, cc in enumerate(cl[2]):
                for id_, cd in enumerate(cl[3]):
                    f = np.ones_like(u)
                    for ax in range(3):
                        f = f * tabs[ax][ca[ax], cb[ax], cc[ax], cd[ax]]
                    out[ia, ib, ic, id_] = 2.0 / math.sqrt(math.pi) * np.sum(f * jac * wt)
    return out


def gauss_moment(n, beta):
    """int x^n exp(-beta x^2) dx over the real line, by Gauss-Hermite."""
    return beta ** (-(n + 1) / 2.0) * float(np.sum(_GH_W * _GH_X ** n))
