"""Writes fullsize_jk_blocks.json: J and K blocks of the 30-atom 3s2p1d
benchmark molecule (N = 420, Schwarz tau = 1e-12) computed by the CPU oracle
only -- each block straight from the definition of J and K, summed over every
ordered shell pair with the same screening rule -- in double and in long
double (the double build's own rounding error).  The 64 blocks cover every
ordered pair of shell angular momenta (s, p, d) on the two sides, diagonal
blocks, blocks of shells on one atom and blocks of distant shells.

    python tests/golden/make_fullsize_blocks.py      (about 30 min on 8 cores)
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle      # noqa: E402
import workloads   # noqa: E402

TAU = 1e-12
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fullsize_jk_blocks.json")


def choose_pairs(bw, n=64, seed=4242):
    rng = np.random.default_rng(seed)
    by_l = {l: np.where(bw.l == l)[0] for l in (0, 1, 2)}
    dist = np.linalg.norm(bw.centers[:, None, :] - bw.centers[None, :, :], axis=2)
    pairs = []
    combos = [(a, b) for a in (0, 1, 2) for b in (0, 1, 2)]
    k = 0
    while len(pairs) < n:
        la, lb = combos[k % len(combos)]
        kind = (k // len(combos)) % 4      # 0 any, 1 same atom, 2 far apart, 3 diagonal when la == lb
        k += 1
        P = int(rng.choice(by_l[la]))
        cand = by_l[lb]
        if kind == 1:
            cand = [s for s in cand if bw.atom[s] == bw.atom[P]] or list(cand)
        elif kind == 2:
            cand = [s for s in cand if dist[P, s] > 8.0] or list(cand)
        Q = P if (kind == 3 and la == lb) else int(rng.choice(cand))
        if (P, Q) not in pairs:
            pairs.append((P, Q))
    return pairs


def main():
    bw, D = workloads.molecule_3s2p1d()
    pairs = choose_pairs(bw)
    t = time.time()
    J, K = oracle.jk_blocks(bw, D, pairs, tau=TAU)
    print(f"double: {time.time() - t:.0f} s", flush=True)
    t = time.time()
    Jl, Kl = oracle.jk_blocks(bw, D, pairs, tau=TAU, precision="long double")
    print(f"long double: {time.time() - t:.0f} s", flush=True)
    data = {"workload": "mol30_3s2p1d (seed 1002), Schwarz tau 1e-12", "tau": TAU, "pairs": pairs,
            "l": [[int(bw.l[p]), int(bw.l[q])] for p, q in pairs],
            "J": [b.ravel().tolist() for b in J], "K": [b.ravel().tolist() for b in K],
            "J_ld": [b.ravel().tolist() for b in Jl], "K_ld": [b.ravel().tolist() for b in Kl]}
    with open(OUT, "w") as fh:
        json.dump(data, fh)
    print(f"wrote {OUT}: {len(pairs)} blocks")


if __name__ == "__main__":
    main()
