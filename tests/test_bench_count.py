"""The throughput figures' ERI count (paper_2605_10312_amd/counts.py): unique (8-fold) spherical function quartets of the
shell quartets a Schwarz screen keeps, against brute force over every pair of
shell pairs of small bases (coincident shells and coincident pairs
included)."""
import itertools

import numpy as np
import pytest

from paper_2605_10312_amd import counts
import oracle
import workloads


def brute(Q, l, tau):
    ns = len(l)
    pairs = [(i, j) for i in range(ns) for j in range(i + 1)]
    eris = kept = 0
    for p, r in itertools.combinations_with_replacement(range(len(pairs)), 2):
        (i, j), (k, m) = pairs[p], pairs[r]
        if not Q[i, j] * Q[k, m] >= tau:
            continue
        kept += 1
        # enumerate the function quartets and keep one of each 8-fold image set
        fi = [(a, b) for a in range(2 * l[i] + 1) for b in range(2 * l[j] + 1) if i != j or a >= b]
        fk = [(a, b) for a in range(2 * l[k] + 1) for b in range(2 * l[m] + 1) if k != m or a >= b]
        if p == r:
            eris += len(fi) * (len(fi) + 1) // 2
        else:
            eris += len(fi) * len(fk)
    return eris, kept


@pytest.mark.parametrize("seed,tau", [(31, 1e-12), (32, 1e-6), (33, 1e-3), (34, 0.0)])
def test_unique_eri_count_matches_brute_force(seed, tau):
    bw = workloads.random_small_basis(seed=seed, natom=3, lmax=2, maxprim=2, box=4.0)
    Q = oracle.schwarz(bw)
    l = np.asarray(bw.l)
    assert counts.unique_eris(Q, l, tau) == brute(Q, l, tau)
