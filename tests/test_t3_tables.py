"""The HBM-scratch tier's op tables, run on the CPU.

The generator turns a class into a slot-packed VRR program and a Phase-2
program (gen/emit_t3.py); a GPU kernel only interprets them.  Here a plain
numpy interpreter of the same op semantics runs the tables on a few random
normalised primitive quartets and the result is compared with the oracle,
so slot reuse, operand encoding and the transform coefficients are checked
without a GPU.  The Boys values come from scipy's 1F1, independent of both
the oracle and the GPU path."""
import numpy as np
import pytest
from scipy.special import hyp1f1

import oracle
import workloads
from paper_2605_10312_amd.gen import emit_t3


def _norm(a, l):
    df = 1.0
    for k in range(2 * l - 1, 1, -2):
        df *= k
    return (2 * a / np.pi) ** 0.75 * (4 * a) ** (0.5 * l) / np.sqrt(df)


def run_tables(t, ls, centers, exps):
    n = centers.shape[0]
    A, B, C, D = (centers[:, k, :].T for k in range(4))          # [3, n]
    a, b, c, d = (exps[:, k] for k in range(4))
    zeta, eta = a + b, c + d
    P = (a * A + b * B) / zeta
    Q = (c * C + d * D) / eta
    Kab = _norm(a, ls[0]) * _norm(b, ls[1]) * np.exp(-a * b / zeta * np.sum((A - B) ** 2, 0)) * np.sqrt(2) * np.pi ** 1.25 / zeta
    Kcd = _norm(c, ls[2]) * _norm(d, ls[3]) * np.exp(-c * d / eta * np.sum((C - D) ** 2, 0)) * np.sqrt(2) * np.pi ** 1.25 / eta
    ze = zeta + eta
    rz, re, o2ze = eta / ze, zeta / ze, 0.5 / ze
    PQ = P - Q
    T = zeta * rz * np.sum(PQ ** 2, 0)
    base = Kab * Kcd / np.sqrt(ze)
    sb = np.zeros((t.nslots, n))
    for m in range(t.L + 1):
        sb[m] = base * hyp1f1(m + 0.5, m + 1.5, -T) / (2 * m + 1)
    PA, QC, WP, WQ = P - A, Q - C, -rz * PQ, re * PQ
    o2z, o2e = 0.5 / zeta, 0.5 / eta
    AB, CD = A - B, C - D
    ops = np.array(t.ops, dtype=np.int64).reshape(-1, 8)
    coefs = np.array(t.coefs)
    none = emit_t3.NONE
    for k, w in enumerate(ops):
        code, axis = w[0] & 15, (w[0] >> 4) & 3
        dst = w[1]
        if code == emit_t3.OP_ACC:
            sb[dst] += sb[w[2]]
        elif code in (emit_t3.OP_VRR_BRA, emit_t3.OP_VRR_KET):
            ks, kc = (w[0] >> 6) & 31, (w[0] >> 11) & 31
            X, Y, o2, r = (PA, WP, o2z, rz) if code == emit_t3.OP_VRR_BRA else (QC, WQ, o2e, re)
            v = X[axis] * sb[w[2]] + Y[axis] * sb[w[3]]
            if ks:
                v = v + ks * o2 * (sb[w[4]] - r * sb[w[5]])
            if kc:
                v = v + kc * o2ze * sb[w[6]]
            sb[dst] = v
        elif code in (emit_t3.OP_HRR_BRA, emit_t3.OP_HRR_KET):
            dv = AB if code == emit_t3.OP_HRR_BRA else CD
            sb[dst] = sb[w[2]] + dv[axis] * sb[w[3]]
        else:
            v = sb[dst].copy() if code == emit_t3.OP_LIN_ACC else np.zeros(n)
            for s, ci in zip(w[2:5], w[5:8]):
                if s != none:
                    v = v + coefs[ci] * sb[s]
            sb[dst] = v
    out = sb[np.array(t.outslots)].T
    return out.reshape([n] + [2 * l + 1 for l in ls])


@pytest.mark.parametrize("ls,n", [((0, 0, 0, 0), 4), ((1, 0, 1, 0), 4), ((2, 1, 1, 0), 4), ((2, 2, 2, 2), 4),
                                  ((3, 2, 1, 0), 3), ((3, 3, 3, 3), 3), ((4, 3, 2, 1), 2)])
def test_t3_tables_match_oracle(ls, n):
    t = emit_t3.build_tables(*ls)
    # compact quartets (1 A box, moderate exponents) so that the integrals are of order one
    cen, ex = workloads.prim_quartets(max(ls), n, seed=77, box=1.0, exp_range=(0.2, 2.0))
    got = run_tables(t, ls, cen, ex)
    ref = oracle.eri_prim_quartets(ls, cen, ex)
    ref_ld = oracle.eri_prim_quartets(ls, cen, ex, precision="long double")
    err = np.abs(got - ref_ld).max()
    e_orc = np.abs(ref - ref_ld).max()
    print(f"{ls}: {t.nslots} slots, {t.n_vrr} + {t.n_p2} ops, max |I| {np.abs(ref_ld).max():.2e}, "
          f"max |tables - oracle_ld| {err:.2e} (oracle {e_orc:.2e})")
    assert err <= 1e-12 + 8 * e_orc


def test_t3_slot_packing():
    """Slot reuse keeps the buffer near the liveness bound: accumulators plus
    the VRR frontier, far below one slot per VRR node."""
    t = emit_t3.build_tables(3, 3, 3, 3)
    from paper_2605_10312_amd.gen import vrr
    g = vrr.VRRGraph(3, 3, 3, 3)
    assert t.nslots < t.acc0 + t.n_hrr + len(g.nodes) // 4
    assert t.n_vrr == sum(1 for nd in g.nodes if nd.kind != "base") + t.n_hrr
