"""The row tier's program (gen/emit_row.py), run on the CPU.

The row tier splits Phase 1 into chunks of whole bra rows (ket stage fused
after the primitive loop) or tiles of one row, and runs the bra stage per
ket function in a second kernel, all through a slot buffer.  Here a numpy
interpreter executes exactly that program -- each chunk's VRR subgraph in its
emission order, the ket-stage ops of the swapped Phase 2, the slot
assignments, the bra-stage ops -- on a few normalised primitive quartets,
and the integrals are compared with the oracle.  So chunk coverage, the slot
layout and the ket-first stepwise transform are checked before any GPU run.
The Boys values come from scipy's 1F1, independent of both sides."""
import numpy as np
import pytest
from scipy.special import hyp1f1

import oracle
import workloads
from paper_2605_10312_amd.gen import emit_row


def _norm(a, l):
    df = 1.0
    for k in range(2 * l - 1, 1, -2):
        df *= k
    return (2 * a / np.pi) ** 0.75 * (4 * a) ** (0.5 * l) / np.sqrt(df)


def run_row_plan(plan, centers, exps, wave=False):
    """wave: kernel 2 as the integrals-out kernels run it (the tiled rows' ket
    stage and the bra stage each as one op list shared by every row or ket
    function); otherwise as the J/K kernel runs it."""
    ls = plan.ls
    g = plan.g
    A, B, C, D = (centers[:, k, :].T for k in range(4))
    a, b, c, d = (exps[:, k] for k in range(4))
    zeta, eta = a + b, c + d
    P, Q = (a * A + b * B) / zeta, (c * C + d * D) / eta
    Kab = _norm(a, ls[0]) * _norm(b, ls[1]) * np.exp(-a * b / zeta * np.sum((A - B) ** 2, 0)) * np.sqrt(2) * np.pi ** 1.25 / zeta
    Kcd = _norm(c, ls[2]) * _norm(d, ls[3]) * np.exp(-c * d / eta * np.sum((C - D) ** 2, 0)) * np.sqrt(2) * np.pi ** 1.25 / eta
    ze = zeta + eta
    rz, re, o2ze = eta / ze, zeta / ze, 0.5 / ze
    PQ = P - Q
    T = zeta * rz * np.sum(PQ ** 2, 0)
    base = Kab * Kcd / np.sqrt(ze)
    F = [hyp1f1(m + 0.5, m + 1.5, -T) / (2 * m + 1) for m in range(g.L + 1)]
    PA, QC, WP, WQ = P - A, Q - C, -rz * PQ, re * PQ
    o2z, o2e = 0.5 / zeta, 0.5 / eta
    env = {"ABx": (A - B)[0], "ABy": (A - B)[1], "ABz": (A - B)[2],
           "CDx": (C - D)[0], "CDy": (C - D)[1], "CDz": (C - D)[2]}
    n = centers.shape[0]
    sb = np.full((plan.nslots, n), np.nan)
    written = np.zeros(plan.nslots, bool)

    def run_ops(ops, vals):
        for op in ops:
            if op[1] == "hrr":
                dst, _, hi, lo, coef = op
                vals[dst] = vals[hi] + env[coef] * vals[lo]
            else:
                dst, _, terms = op
                vals[dst] = sum(cf * vals[s] for cf, s in terms)

    def store(slot, v):
        assert not written[slot], slot
        written[slot] = True
        sb[slot] = v

    eidx = {e: i for i, e in enumerate(plan.E)}
    kstage = {f2: (a0, a1) for (f2, a0, a1) in plan.kp2.bra_stages}
    covered = []
    for ch in plan.chunks:
        v = {}
        for u in ch.order:                   # the emitted order: parents always first
            nd = g.nodes[u]
            if nd.kind == "base":
                v[u] = base * F[nd.key[2]]
                continue
            p1, p2, p3, p4, p5 = nd.parents
            X, W, o2, rr = (PA, WP, o2z, rz) if nd.kind == "bra" else (QC, WQ, o2e, re)
            x = X[nd.axis] * v[p1] + W[nd.axis] * v[p2]
            if nd.k_same:
                x = x + nd.k_same * o2 * (v[p3] - rr * v[p4])
            if nd.k_cross:
                x = x + nd.k_cross * o2ze * v[p5]
            v[u] = x
        acc = {f"h{g.target_ids.index(t)}": v[t] for t in ch.targets}
        covered.extend(ch.targets)
        if ch.kind == "rows":
            for e in ch.rows:
                a0, a1 = kstage[e]
                vals = dict(acc)
                run_ops(plan.kp2.ops[a0:a1], vals)
                for lam in range(plan.nc):
                    for sig in range(plan.nd):
                        store(plan.zslot(eidx[e], lam, sig), vals[plan.kp2.s2[(lam, sig, e)]])
        else:
            tr = plan.tile_rows.index(ch.rows[0])
            for t in ch.targets:
                f = g.nodes[t].key[1]
                store(plan.hslot(tr, plan.F.index(f)), acc[f"h{g.target_ids.index(t)}"])
    assert sorted(covered) == sorted(g.target_ids)       # every target in exactly one chunk
    if wave:
        tops, tins, touts = plan.wave_ket()
        for tr, e in enumerate(plan.tile_rows):
            vals = {nm: sb[plan.hslot(tr, plan.F.index(f))] for f, nm in tins.items()}
            run_ops(tops, vals)
            for (lam, sig), nm in touts.items():
                store(plan.zslot(eidx[e], lam, sig), vals[nm])
        assert written[:plan.nslots_ints].all()
        wops, wins, wouts = plan.wave_bra()
        out = np.full((n, plan.na, plan.nb, plan.nc, plan.nd), np.nan)
        for lam in range(plan.nc):
            for sig in range(plan.nd):
                vals = {nm: sb[plan.zslot(eidx[e], lam, sig)] for e, nm in wins.items()}
                run_ops(wops, vals)
                for (mu, nu), nm in wouts.items():
                    out[:, mu, nu, lam, sig] = vals[nm]
        assert not np.isnan(out).any()
        return out
    # kernel 2: the tiled rows' ket stage, then the bra stage per ket function,
    # group by group as emitted (each group reads its inputs from the buffer)
    for tr, e in enumerate(plan.tile_rows):
        for ops, ins, outs in plan.k2_ket(e):
            vals = {nm: sb[plan.hslot(tr, plan.F.index(f))] for f, nm in ins.items()}
            run_ops(ops, vals)
            for (lam, sig), nm in outs.items():
                store(plan.zslot(eidx[e], lam, sig), vals[nm])
    assert written[:plan.nslots_ints].all()
    out = np.full((n, plan.na, plan.nb, plan.nc, plan.nd), np.nan)
    for lam in range(plan.nc):
        for sig in range(plan.nd):
            for ops, ins, outs in plan.k2_bra(lam, sig):
                vals = {nm: sb[plan.zslot(eidx[e], lam, sig)] for e, nm in ins.items()}
                run_ops(ops, vals)
                for (mu, nu), nm in outs.items():
                    assert np.isnan(out[0, mu, nu, lam, sig])
                    out[:, mu, nu, lam, sig] = vals[nm]
    assert not np.isnan(out).any()
    return out


@pytest.mark.parametrize("ls,budget", [((2, 2, 2, 2), 240), ((3, 2, 2, 1), 240), ((2, 1, 3, 3), 240),
                                       ((3, 3, 2, 2), 160), ((4, 3, 1, 0), 240), ((3, 3, 3, 3), 240),
                                       ((4, 2, 3, 1), 200)])
def test_row_plan_matches_oracle(ls, budget):
    plan = emit_row.plan_rows(*ls, budget=budget)
    for ch in plan.chunks:                                  # every chunk fits the register line by the model
        assert len(ch.targets) + ch.peak_live + 40 <= budget or (ch.kind == "tile" and len(ch.targets) == 1)
    cen, ex = workloads.prim_quartets(max(ls), 3, seed=91, box=1.5, exp_range=(0.3, 3.0))
    got = run_row_plan(plan, cen, ex)
    gw = run_row_plan(plan, cen, ex, wave=True)            # the integrals-out form of kernel 2
    ref = oracle.eri_prim_quartets(ls, cen, ex)
    ref_ld = oracle.eri_prim_quartets(ls, cen, ex, precision="long double")
    e_orc = np.abs(ref - ref_ld).max()
    err = np.abs(got - ref_ld).max()
    rows = sum(1 for c in plan.chunks if c.kind == "rows")
    print(f"{ls}: {len(plan.chunks)} chunks ({rows} of rows, {len(plan.tile_rows)} rows tiled), "
          f"recompute x{emit_row.recompute_factor(plan):.2f}, {plan.nslots} slots, err {err:.2e} (oracle {e_orc:.2e})")
    assert err <= 1e-12 + 8 * e_orc
    assert np.abs(gw - ref_ld).max() <= 1e-12 + 8 * e_orc


def test_row_plan_grouped_stages():
    """Stages with more inputs than kernel 2 holds at once run in groups of
    second-index functions; forced here on a small class."""
    plan = emit_row.plan_rows(3, 2, 2, 2, budget=240)
    plan.bra_groups, plan.ket_groups = 3, 2
    plan.tile_rows = []
    assert len(plan.k2_bra(0, 0)) == 3
    cen, ex = workloads.prim_quartets(3, 3, seed=5, box=1.5, exp_range=(0.3, 3.0))
    got = run_row_plan(plan, cen, ex)
    ref_ld = oracle.eri_prim_quartets((3, 2, 2, 2), cen, ex, precision="long double")
    assert np.abs(got - ref_ld).max() <= 1e-12
    # a tiled row's ket stage in groups as well
    plan = emit_row.plan_rows(3, 3, 3, 3, budget=200)
    plan.bra_groups, plan.ket_groups = 2, 3
    cen, ex = workloads.prim_quartets(3, 2, seed=6, box=1.5, exp_range=(0.3, 3.0))
    got = run_row_plan(plan, cen, ex)
    ref_ld = oracle.eri_prim_quartets((3, 3, 3, 3), cen, ex, precision="long double")
    assert np.abs(got - ref_ld).max() <= 1e-12


def test_row_plan_tiles_a_row_that_does_not_fit():
    # a tight budget forces tiles; the tiles of a row partition its targets
    plan = emit_row.plan_rows(3, 3, 3, 3, budget=200)
    assert plan.tile_rows
    for e in plan.tile_rows:
        tiles = [c for c in plan.chunks if c.kind == "tile" and c.rows == [e]]
        assert len(tiles) >= 2
        ids = sorted(t for c in tiles for t in c.targets)
        assert len(ids) == len(set(ids)) == len(plan.F)


def test_row_emitter_source():
    src, meta = emit_row.emit_class_row(2, 2, 2, 1)
    assert meta.tier == 1 and meta.form == "row" and meta.chunks >= 1
    assert "void eri_2221(EriArgs a)" in src and "void launch_p1_2221(" in src and "launch_eri_2221" in src
    assert "void jk_2221(JKArgs a)" in meta.extra_sources["jk"] and "launch_jk_2221" in meta.extra_sources["jk"]
    parts = {k: v for k, v in meta.extra_sources.items() if k.startswith("p")}
    assert len(parts) == meta.parts and all(f"void p1_2221p{k}(P1Args a)" in parts[f"p{k}"] for k in range(meta.parts))
    assert sum(p.count("case ") for p in parts.values()) == meta.chunks
    # the FP32 Phase 1 of mixed precision: the same chunks, float VRR and accumulators, FP64 ket stage
    p32 = {k: v for k, v in meta.extra_sources.items() if k.startswith("q")}
    assert meta.p1_32 and len(p32) == meta.parts
    assert all(f"void p1f_2221p{k}(P1Args a)" in p32[f"q{k}"] and "float Bf[" in p32[f"q{k}"] and
               "= (double)h0f" in p32[f"q{k}"] for k in range(meta.parts))
    assert "void launch_p1f_2221(" in src
    src, meta = emit_row.emit_class_row(3, 3, 3, 3, budget=200)   # many chunks: several Phase-1 parts
    assert meta.parts == -(-meta.chunks // emit_row.P1_PART_CHUNKS) > 1
    assert all(f"launch_p1_3333p{k}(a, s);" in src for k in range(meta.parts))
    # integrals out: one wave per quartet; the tiled rows' ket stage runs in it, into LDS
    assert meta.eri_wave and not meta.eri_tiles and "jj < 49 &&" in src and "__shared__ double zt[P * " in src
    assert "eri_3333<1>" in src and "eri_3333<2>" not in src           # 49 ket functions: one quartet a wave
    src21, _ = emit_row.emit_class_row(2, 2, 2, 1)
    assert "eri_2221<4>" in src21 and "eri_2221<1>" in src21           # 15: four quartets a wave (Schwarz mode: one)
    from paper_2605_10312_amd.gen import emit
    table = emit.emit_table([meta])
    assert ", 1, nullptr, launch_p1f_3333, nullptr}" in table
    assert all("hgp_store_runs<" in meta.extra_sources[f"p{k}"] for k in range(meta.parts))
