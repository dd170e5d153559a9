"""Cartesian and spherical component bookkeeping for the kernel generator.

Cartesian order within a shell of angular momentum l: x power descending,
then y power descending (xx, xy, xz, yy, yz, zz for l = 2).  Pure spherical
order: s and p are kept as is (p as x, y, z); l >= 2 as m = -l .. l.
"""
from __future__ import annotations

from functools import lru_cache


@lru_cache(maxsize=None)
def comps(l: int):
    """Cartesian exponent triples of one shell, in the library's order."""
    return tuple((x, y, l - x - y) for x in range(l, -1, -1) for y in range(l - x, -1, -1))


def ncart(l: int) -> int:
    return (l + 1) * (l + 2) // 2


def nsph(l: int) -> int:
    return 2 * l + 1


def index_in_shell(c) -> int:
    """Position of exponent triple c inside its shell."""
    y, z = c[1], c[2]
    s = y + z
    return s * (s + 1) // 2 + z


def levels(lo: int, hi: int):
    """All triples with lo <= |c| <= hi, level by level."""
    out = []
    for l in range(lo, hi + 1):
        out.extend(comps(l))
    return tuple(out)


def add(c, axis, by=1):
    d = list(c)
    d[axis] += by
    return tuple(d)


def canonical_classes(lmax: int):
    """Canonical quartet classes (la lb|lc ld): la >= lb, lc >= ld and
    (la, lb) >= (lc, ld) in the pair order used by the library (pairs
    ordered by (la, lb) lexicographically).  21 for l <= 2, 55 for l <= 3,
    120 for l <= 4 (Sec. IV's count of unique angular-momentum tuples)."""
    pairs = [(a, b) for a in range(lmax + 1) for b in range(a + 1)]
    out = []
    for i, p in enumerate(pairs):
        for q in pairs[: i + 1]:
            out.append((p[0], p[1], q[0], q[1]))
    return out


def pair_classes(lmax: int):
    return [(a, b) for a in range(lmax + 1) for b in range(a + 1)]
