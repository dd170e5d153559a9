"""Cartesian -> pure spherical shell transformation T^(l) (Sec. III-B,
Eq. cart2sph), derived exactly with sympy.

Row m of T^(l) holds the Cartesian coefficients of the real solid harmonic of
degree l and order m: r^l P_l^|m|(cos theta) times cos(|m| phi) for m >= 0 or
sin(|m| phi) for m < 0, written as a homogeneous polynomial
Re/Im[(x + i y)^|m|] * r^(l-|m|) * (d^|m| P_l / dt^|m|)(z / r).  Each row is
scaled to unit norm for Gaussian primitives that all carry the factor
normalising x^l exp(-a r^2), and its sign is chosen so that the leading
monomial (x^|m| z^(l-|m|) for m >= 0, x^(|m|-1) y z^(l-|m|) for m < 0) has a
positive coefficient.  s and p shells are left untransformed.
"""
from __future__ import annotations

from functools import lru_cache

import sympy as sp

from .cart import comps, index_in_shell

_x, _y, _z, _t = sp.symbols("x y z t", real=True)


def _dfact(n: int) -> int:
    r = 1
    while n > 1:
        r *= n
        n -= 2
    return r


def _solid_harmonic(l: int, m: int):
    am = abs(m)
    dp = sp.Poly(sp.diff(sp.legendre(l, _t), _t, am), _t)
    radial = 0
    for (k,), c in dp.terms():
        radial += c * _z ** k * (_x ** 2 + _y ** 2 + _z ** 2) ** ((l - am - k) // 2)
    xy = sp.expand((_x + sp.I * _y) ** am)
    ang = sp.re(xy) if m >= 0 else sp.im(xy)
    return sp.Poly(sp.expand(ang * radial), _x, _y, _z)


def _metric(l, c1, c2):
    num = 1
    for a in range(3):
        s = c1[a] + c2[a]
        if s % 2:
            return sp.Integer(0)
        num *= _dfact(s - 1)
    return sp.Rational(num, _dfact(2 * l - 1))


@lru_cache(maxsize=None)
def tmatrix_exact(l: int):
    """T^(l) as a tuple of rows of sympy numbers, (2l+1) x ncart(l)."""
    cs = comps(l)
    if l <= 1:
        return tuple(tuple(sp.Integer(1 if i == j else 0) for j in range(len(cs))) for i in range(len(cs)))
    rows = []
    for m in range(-l, l + 1):
        poly = _solid_harmonic(l, m)
        row = [sp.Integer(0)] * len(cs)
        for mon, c in poly.terms():
            row[index_in_shell(mon)] += c
        nn = sum(row[i] * row[j] * _metric(l, cs[i], cs[j]) for i in range(len(cs)) for j in range(len(cs)))
        scale = 1 / sp.sqrt(sp.nsimplify(nn))
        row = [sp.nsimplify(v * scale) for v in row]
        am = abs(m)
        lead = (am, 0, l - am) if m >= 0 else (am - 1, 1, l - am)
        if row[index_in_shell(lead)] < 0:
            row = [-v for v in row]
        rows.append(tuple(row))
    return tuple(rows)


@lru_cache(maxsize=None)
def tmatrix(l: int):
    """T^(l) as floats: tuple of rows, each a tuple of (cart index, coefficient)
    over the nonzero entries only."""
    out = []
    for row in tmatrix_exact(l):
        out.append(tuple((j, float(sp.N(v, 30))) for j, v in enumerate(row) if v != 0))
    return tuple(out)


def tmatrix_dense(l: int):
    import numpy as np

    cs = comps(l)
    n = 1 if l <= 1 else 0
    rows = tmatrix(l)
    a = np.zeros((len(rows), len(cs)))
    for i, r in enumerate(rows):
        for j, v in r:
            a[i, j] = v
    return a
