"""Contracted-ERI counts for throughput figures: unique (8-fold) spherical
function quartets of the shell quartets a Schwarz screen keeps.  Host
arithmetic on the plan's own screening factors (hgp_plan_schwarz), none of
the method's; the kernels compute whole shell-quartet blocks, whose
redundant elements (coincident shells or shell pairs) are not counted."""
from __future__ import annotations

import numpy as np


def pair_functions(l_a, l_b, same):
    """Unique spherical function pairs of a shell pair (i >= j)."""
    na, nb = 2 * np.asarray(l_a) + 1, 2 * np.asarray(l_b) + 1
    return np.where(same, na * (na + 1) // 2, na * nb)


def unique_eris(Q, l, tau):
    """(unique function quartets, kept shell quartets) of one system: shell
    pairs p = (i >= j) with factor Q[i, j], unordered pairs of pairs {p, r}
    kept where Q_p Q_r >= tau (the plan's test, in the same floating point);
    a quartet holds F_p F_r function quartets, F_p (F_p + 1) / 2 when p = r.
    For a multi-system plan, call it per system on its block of Q."""
    l = np.asarray(l)
    i, j = np.tril_indices(len(l))
    q = np.asarray(Q)[i, j]
    F = pair_functions(l[i], l[j], i == j).astype(np.float64)
    if tau <= 0.0:                               # no screen: every quartet
        n = float(np.sum(F))
        return int(round((n * n - np.sum(F * F)) / 2 + np.sum(F * (F + 1) / 2))), len(q) * (len(q) + 1) // 2
    keep = q > 0.0                               # a factor of 0 never passes tau > 0
    q, F = q[keep], F[keep]
    order = np.argsort(q)
    qs, Fs = q[order], F[order]
    # first sorted index r with q_p * qs[r] >= tau (exact products: step the guess from tau / q_p)
    idx = np.searchsorted(qs, tau / q)
    for _ in range(4):
        lo = (idx > 0) & (q * qs[np.maximum(idx - 1, 0)] >= tau)
        idx = np.where(lo, idx - 1, idx)
        hi = (idx < len(qs)) & (q * qs[np.minimum(idx, len(qs) - 1)] < tau)
        idx = np.where(hi, idx + 1, idx)
    suffix_F = np.concatenate([np.cumsum(Fs[::-1])[::-1], [0.0]])
    ordered = float(np.sum(F * suffix_F[idx]))
    ordered_n = float(np.sum(len(qs) - idx))
    diag = q * q >= tau
    eris = (ordered - np.sum(F[diag] ** 2)) / 2 + np.sum(F[diag] * (F[diag] + 1) / 2)
    nquart = (ordered_n - np.count_nonzero(diag)) / 2 + np.count_nonzero(diag)
    return int(round(eris)), int(round(nquart))
