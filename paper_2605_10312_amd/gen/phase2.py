"""Phase 2: horizontal recurrence with stepwise Cartesian -> spherical fusion
(Sec. II-A, Eq. hrr; Sec. III-B, Eqs. bra-sph .. stepwise-sph).

Starting from the contracted accumulators H[e][f] (la <= |e| <= la+lb,
lc <= |f| <= lc+ld), the ops produced here are, in order:

  for every ket component f:   bra HRR  (a b+1_i| = (a+1_i b| + AB_i (a b|
                               T^(la) on a, then T^(lb) on b   (mask 1000, 1100)
  for every spherical (m, n):  ket HRR  (mn|c d+1_i) = (mn|c+1_i d) + CD_i (mn|c d)
                               T^(lc) on c, then T^(ld) on d   (mask 1110, 1111)

so the Cartesian tensor is never materialised: each index is projected as
soon as its recurrence is finished.  s and p shells are not transformed.

Ops are SSA: (dst, "hrr", hi, lo, coef) meaning dst = hi + coef * lo, and
(dst, "lin", [(c, src), ...]) meaning dst = sum c * src.  Sources may be
input names (the H accumulators) or earlier destinations.
"""
from __future__ import annotations

from .cart import add, comps, levels
from .sph import tmatrix


class Phase2:
    def __init__(self, la, lb, lc, ld, hname, ab=("ABx", "ABy", "ABz"), cd=("CDx", "CDy", "CDz"),
                 prefix="x", spherical=True):
        """hname(e, f) -> name of the contracted accumulator [e0|f0]."""
        self.ls = (la, lb, lc, ld)
        self.ops = []
        self.n = 0
        self.prefix = prefix
        self.flops = 0
        self.spherical = spherical
        na = len(tmatrix(la)) if spherical else len(comps(la))
        nb = len(tmatrix(lb)) if spherical else len(comps(lb))
        # ---- bra side, one ket component f at a time
        s2 = {}
        self.bra_stages = []      # per f: (f, first op, end op)
        for f in levels(lc, lc + ld):
            first = len(self.ops)
            memo = {}

            def X(a, b):
                if sum(b) == 0:
                    return hname(a, f)
                if (a, b) in memo:
                    return memo[(a, b)]
                i = max(k for k in range(3) if b[k] > 0)
                b1 = add(b, i, -1)
                hi = X(add(a, i, +1), b1)
                lo = X(a, b1)
                memo[(a, b)] = self._hrr(hi, lo, ab[i])
                return memo[(a, b)]

            xb = {(a, b): X(a, b) for a in comps(la) for b in comps(lb)}
            s1 = {}
            for ib, b in enumerate(comps(lb)):
                for mu, row in enumerate(self._rows(la)):
                    s1[(mu, ib)] = self._lin([(c, xb[(comps(la)[j], b)]) for j, c in row])
            for mu in range(na):
                for nu, row in enumerate(self._rows(lb)):
                    s2[(mu, nu, f)] = self._lin([(c, s1[(mu, j)]) for j, c in row])
            self.bra_stages.append((f, first, len(self.ops)))
        self.s2 = s2
        # ---- ket side, one spherical bra pair (m, n) at a time
        self.out = {}
        self.ket_stages = []      # per (m, n): (m, n, first op, end op)
        for mu in range(na):
            for nu in range(nb):
                first = len(self.ops)
                memo = {}

                def Y(c, d):
                    if sum(d) == 0:
                        return s2[(mu, nu, c)]
                    if (c, d) in memo:
                        return memo[(c, d)]
                    i = max(k for k in range(3) if d[k] > 0)
                    d1 = add(d, i, -1)
                    hi = Y(add(c, i, +1), d1)
                    lo = Y(c, d1)
                    memo[(c, d)] = self._hrr(hi, lo, cd[i])
                    return memo[(c, d)]

                yc = {(c, d): Y(c, d) for c in comps(lc) for d in comps(ld)}
                z = {}
                for idd, d in enumerate(comps(ld)):
                    for lam, row in enumerate(self._rows(lc)):
                        z[(lam, idd)] = self._lin([(c, yc[(comps(lc)[j], d)]) for j, c in row])
                for lam in range(len(self._rows(lc))):
                    for sig, row in enumerate(self._rows(ld)):
                        self.out[(mu, nu, lam, sig)] = self._lin([(c, z[(lam, j)]) for j, c in row])
                self.ket_stages.append((mu, nu, first, len(self.ops)))
        self.na, self.nb = na, nb
        self.nc = len(self._rows(lc))
        self.nd = len(self._rows(ld))

    def _rows(self, l):
        if self.spherical:
            return tmatrix(l)
        return tuple(((j, 1.0),) for j in range(len(comps(l))))

    def _new(self):
        name = f"{self.prefix}{self.n}"
        self.n += 1
        return name

    def _hrr(self, hi, lo, coef):
        d = self._new()
        self.ops.append((d, "hrr", hi, lo, coef))
        self.flops += 2
        return d

    def _lin(self, terms):
        if len(terms) == 1 and terms[0][0] == 1.0:
            return terms[0][1]                      # identity row: no op
        d = self._new()
        self.ops.append((d, "lin", tuple(terms)))
        self.flops += 2 * len(terms) - 1
        return d
