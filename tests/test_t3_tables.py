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


def run_tables(t, ls, centers, exps, ops=None, K=None, zero=None, weights=False, shape=None):
    """Run tables t on the quartets; ops/K/zero: the wave-cooperative form
    (its own words, groups of K ops, absent operands naming slot zero).
    weights: fill slots L+1..L+3 with 2a, 2b, 2c of each primitive quartet
    (the derivative tables' ACC_W weights).  shape: of one quartet's outputs."""
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
    sb = np.zeros((t.nslots + 2, n))
    for m in range(t.L + 1):
        sb[m] = base * hyp1f1(m + 0.5, m + 1.5, -T) / (2 * m + 1)
    if weights:
        sb[t.L + 1], sb[t.L + 2], sb[t.L + 3] = 2 * a, 2 * b, 2 * c
    PA, QC, WP, WQ = P - A, Q - C, -rz * PQ, re * PQ
    o2z, o2e = 0.5 / zeta, 0.5 / eta
    AB, CD = A - B, C - D
    ops = np.array(t.ops if ops is None else ops, dtype=np.int64).reshape(-1, 8)
    coefs = np.array(t.coefs)
    none = emit_t3.NONE if zero is None else zero
    K = emit_t3.BUNDLE if K is None else K
    assert len(ops) % K == 0 and t.n_vrr % K == 0

    def val(s):
        assert s < t.nslots or s == none
        return sb[s] if s != none else sb[0] * 0.0

    # a group reads all its operands before it writes anything, as on the GPU
    for g0 in range(0, len(ops), K):
        grp = [w for w in ops[g0:g0 + K] if w[0] != 0]
        codes = {w[0] & 15 for w in grp}
        kinds = {0 if c in (1, 2) else 3 if c in (3, 8) else c if c < 6 else 6 for c in codes}
        assert len(kinds - {4, 5} | ({4} if codes & {4, 5} else set())) == 1
        reads = [[val(s) for s in w[2:7]] + [sb[w[1]].copy()] for w in grp]
        for w, r in zip(grp, reads):
            code, axis = w[0] & 15, (w[0] >> 4) & 3
            dst = w[1]
            assert dst < t.nslots
            if code == emit_t3.OP_ACC:
                sb[dst] = r[5] + r[0]
            elif code == emit_t3.OP_ACC_W:
                sb[dst] = r[5] + r[1] * r[0]
            elif code in (emit_t3.OP_VRR_BRA, emit_t3.OP_VRR_KET):
                ks, kc = (w[0] >> 6) & 31, (w[0] >> 11) & 31
                X, Y, o2, rr = (PA, WP, o2z, rz) if code == emit_t3.OP_VRR_BRA else (QC, WQ, o2e, re)
                v = X[axis] * r[0] + Y[axis] * r[1]
                if ks:
                    v = v + ks * o2 * (r[2] - rr * r[3])
                if kc:
                    v = v + kc * o2ze * r[4]
                sb[dst] = v
            elif code in (emit_t3.OP_HRR_BRA, emit_t3.OP_HRR_KET):
                dv = AB if code == emit_t3.OP_HRR_BRA else CD
                sb[dst] = r[0] + dv[axis] * r[1]
            else:
                v = r[5] if code == emit_t3.OP_LIN_ACC else np.zeros(n)
                for s, x, ci in zip(w[2:5], r[0:3], w[5:8]):
                    if s != none:
                        v = v + coefs[ci] * x
                sb[dst] = v
    out = sb[np.array(t.outslots)].T
    return out.reshape([n] + (list(shape) if shape else [2 * l + 1 for l in ls]))


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


@pytest.mark.parametrize("ls,n", [((1, 0, 1, 0), 4), ((2, 2, 1, 1), 3), ((3, 2, 1, 0), 3), ((3, 3, 2, 1), 2),
                                  ((4, 1, 3, 0), 2)])
def test_wave_tables_match_oracle(ls, n):
    """The wave-cooperative form: 128-op groups, absent operands naming the
    zero slot, padding ops writing the sink slot and reading only zeros."""
    w = emit_t3.build_wave_tables(*ls)
    t = w.t
    assert w.zero == t.nslots and w.sink == t.nslots + 1
    words = np.array(w.ops, dtype=np.int64).reshape(-1, 8)
    assert len(words) == t.n_vrr + t.n_p2 and len(words) % emit_t3.WAVE == 0
    pad = words[words[:, 0] == 0]
    assert np.all(pad[:, 1] == w.sink) and np.all(pad[:, 2:5] == w.zero)
    assert not np.any(words[words[:, 0] != 0][:, 1] >= t.nslots)           # real ops never write Z or the sink
    assert not np.any(words[:, 2:5] == emit_t3.NONE)
    for g0 in range(0, len(words), emit_t3.WAVE):                            # one op class per group, lane 0 real
        assert words[g0, 0] != 0
    cen, ex = workloads.prim_quartets(max(ls), n, seed=78, box=1.0, exp_range=(0.2, 2.0))
    got = run_tables(t, ls, cen, ex, ops=w.ops, K=emit_t3.WAVE, zero=w.zero)
    ref_ld = oracle.eri_prim_quartets(ls, cen, ex, precision="long double")
    e_orc = np.abs(oracle.eri_prim_quartets(ls, cen, ex) - ref_ld).max()
    err = np.abs(got - ref_ld).max()
    print(f"{ls}: {t.nslots} slots, LDS {w.lds_bytes} B, max |tables - oracle_ld| {err:.2e} (oracle {e_orc:.2e})")
    assert err <= 1e-12 + 8 * e_orc


def test_wave_routing():
    """Every class that leaves the register and staged tiers fits the LDS
    variant (160 KB per workgroup) except (gg|gg)."""
    assert emit_t3.wave_fits(3, 3, 3, 3)
    assert emit_t3.wave_fits(4, 3, 3, 2)
    assert emit_t3.wave_fits(4, 4, 4, 3)
    src, meta = emit_t3.emit_class_t3(4, 4, 4, 4)      # too large: slots in the scratch buffer
    assert meta.tier == 2 and meta.max_batch == emit_t3.GSLOT_MAX_BATCH
    w = emit_t3.build_wave_tables(4, 4, 4, 4)
    assert meta.scratch_slots == w.t.nslots + 2
    assert "t3w_launch_jk(t3_4444" in src and ", 1, &t3_4444_lane};" in src and "T3Class t3_4444_lane = " in src


def test_t3_slot_packing():
    """Slot reuse keeps the buffer near the liveness bound: accumulators plus
    the VRR frontier, far below one slot per VRR node."""
    t = emit_t3.build_tables(3, 3, 3, 3)
    from paper_2605_10312_amd.gen import vrr
    g = vrr.VRRGraph(3, 3, 3, 3)
    assert t.nslots < t.acc0 + t.n_hrr + len(g.nodes) // 4
    K = emit_t3.BUNDLE
    assert t.n_vrr % K == 0 and t.n_p2 % K == 0
    assert t.n_vrr >= sum(1 for nd in g.nodes if nd.kind != "base") + t.n_hrr
    assert t.n_real_ops >= 0.9 * (t.n_vrr + t.n_p2)       # groups stay nearly full
