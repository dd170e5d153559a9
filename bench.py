#!/usr/bin/env python3
"""Benchmark: one J/K build per step on one MI355X.

Workload: a 30-atom synthetic molecule with 3s2p1d shells per atom (1-6
primitives per shell, exponents log-uniform [0.05, 5e3] bohr^-2, spherical d;
N = 420 functions, 180 shells), Schwarz threshold 1e-12, FP64 throughout.
A step is one hgp_jk call (J and K together) on a plan built once before the
timed region, as in the density updates of an SCF run.  The plan build (pair
data, Schwarz factors, screened class lists) is reported as setup_s.

Prints ONE JSON line.  `value` is contracted ERIs per second: the number of
unique contracted spherical integrals the kept quartets hold, per second of
J/K build.  `roofline` refers to the class kernel with the largest share of
the step, timed with HIP events recorded on the stream it runs on;
`cpu_baseline` times the CPU oracle (integrals only, all host threads) on a
random sample of the same screened unique quartets.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

METRIC = "J/K build time & contracted ERIs/s at stated err vs FP64; served p50/p99"
FP64_VALU_PEAK_TFLOPS = 78.6    # 256 CU x 128 FP64 FLOP/clk x 2.4 GHz
TAU = 1e-12


def nsph(l):
    return 2 * l + 1


def overhead_flops(L):
    """Per primitive quartet, outside the VRR graph: pair combination (25),
    Boys Taylor step (21) and downward recurrence (2 per order)."""
    return 46 + 2 * L


def phase_flops(c):
    """(Phase-1 FLOPs, Phase-2 + digestion FLOPs) of one class per J/K build:
    per primitive quartet the unchunked VRR graph plus the pair/Boys overhead,
    per contracted quartet the HRR + transforms plus 12 per integral."""
    la, lb, lc, ld = c["ls"]
    nint = nsph(la) * nsph(lb) * nsph(lc) * nsph(ld)
    per_prim = c["vrr_flops"] + overhead_flops(la + lb + lc + ld)
    per_quartet = c["phase2_flops"] + 12 * nint
    return c["prim_quartets"] * per_prim, c["quartets"] * per_quartet


def algorithmic_flops(c):
    return sum(phase_flops(c))


TRAFFIC_SUMMARY = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                               "jk_mol30_3s2p1d_hbm_traffic.md")


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, calibrated on a plain copy kernel), or
    None when the summary has no row for it or the kernel's sources changed
    since the counters were taken."""
    from paper_2605_10312_amd import build as hb
    if not os.path.exists(TRAFFIC_SUMMARY):
        return None
    tag = kernel.split("_", 1)[1]
    for line in open(TRAFFIC_SUMMARY):
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) == 5 and cells[0] == kernel:
            try:
                fetch, write = float(cells[2]), float(cells[3])
            except ValueError:
                return None
            if cells[4] != hb.class_source_hash(tag):
                return None
            return int(round((fetch + write) * 2 ** 20))
    return None


from paper_2605_10312_amd.counts import pair_functions, unique_eris      # noqa: E402  (host counting only)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(bw, target_s, seed=7):
    """Oracle ERIs/s (unique function quartets, as the GPU line counts them) on
    random screened unique quartets of the same workload."""
    import oracle

    rng = np.random.default_rng(seed)
    Q = oracle.schwarz(bw)
    ns = bw.nshell
    iu = np.tril_indices(ns)
    npair = len(iu[0])

    def draw(n):
        out = []
        while len(out) < n:
            p = rng.integers(0, npair, 4 * n)
            r = rng.integers(0, npair, 4 * n)
            p, r = np.maximum(p, r), np.minimum(p, r)
            keep = Q[iu[0][p], iu[1][p]] * Q[iu[0][r], iu[1][r]] >= TAU
            for a, c in zip(p[keep], r[keep]):
                out.append((iu[0][a], iu[1][a], iu[0][c], iu[1][c]))
        return np.array(out[:n], np.int32)

    probe = draw(200)
    t = time.perf_counter()
    oracle.eri_quartet_list(bw, probe)
    dt = time.perf_counter() - t
    n = int(max(200, min(2_000_000, 200 * target_s / max(dt, 1e-3))))
    sample = draw(n)
    t = time.perf_counter()
    oracle.eri_quartet_list(bw, sample)
    dt = time.perf_counter() - t
    L = np.asarray(bw.l)
    a, b_, c, d = (sample[:, k] for k in range(4))
    Fb = pair_functions(L[a], L[b_], a == b_)
    Fk = pair_functions(L[c], L[d], c == d)
    same = (a == c) & (b_ == d)
    cnt = float(np.sum(np.where(same, Fb * (Fb + 1) // 2, Fb * Fk)))
    return {"value": cnt / dt, "unit": "contracted ERIs/s", "cores": oracle.num_threads(), "cpu_model": cpu_model(),
            "kind": "oracle",
            "sample": f"{n} uniformly drawn screened unique shell quartets of the same workload, "
                      f"integrals only (no J/K digestion), {dt:.1f} s; ERIs counted as unique function quartets"}


def kernel_resources():
    """The compiler's resource report of the loaded library (VGPR, AGPR,
    private scratch, LDS, occupancy per kernel), written beside it by the build."""
    import paper_2605_10312_amd as hgp
    from paper_2605_10312_amd import build as hb
    path = hb.resources_path(hgp.LIB_PATH)
    if not os.path.exists(path):
        return {}
    return {k.split("#")[0]: {x: v.get(x) for x in ("vgpr", "agpr", "scratch", "lds", "occupancy")}
            for k, v in json.load(open(path)).items()}


GOLDEN_BLOCKS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden", "fullsize_jk_blocks.json")


def block_errors(bw, J, K):
    """J/K against the oracle on the 64 stored blocks of this workload (every
    ordered pair of shell angular momenta; written by the oracle alone, in
    double and long double): max abs and RMS over their entries, relative
    Frobenius norm, and the FP64 oracle's own error against long double."""
    gold = json.load(open(GOLDEN_BLOCKS))
    off = bw.shell_offsets()
    mj = mk = eo = sq = nj = nk = 0.0
    cnt = 0
    for k, (p, r) in enumerate(gold["pairs"]):
        shp = (off[p + 1] - off[p], off[r + 1] - off[r])
        sl = (slice(off[p], off[p + 1]), slice(off[r], off[r + 1]))
        jb, kb = np.reshape(gold["J"][k], shp), np.reshape(gold["K"][k], shp)
        dj, dk = J[sl] - jb, K[sl] - kb
        mj, mk = max(mj, float(np.abs(dj).max())), max(mk, float(np.abs(dk).max()))
        sq += float(np.sum(dj ** 2) + np.sum(dk ** 2))
        nj += float(np.sum(jb ** 2))
        nk += float(np.sum(kb ** 2))
        cnt += 2 * dj.size
        eo = max(eo, float(np.abs(jb - np.reshape(gold["J_ld"][k], shp)).max()),
                 float(np.abs(kb - np.reshape(gold["K_ld"][k], shp)).max()))
    return {"blocks": len(gold["pairs"]), "entries": cnt, "J_max_abs": mj, "K_max_abs": mk,
            "rms": (sq / max(cnt, 1)) ** 0.5, "rel_frobenius": (sq / max(nj + nk, 1e-300)) ** 0.5,
            "oracle_fp64_vs_long_double_max_abs": eo, "reference": "CPU oracle, J/K blocks from their definition"}


MICRO_N = 100_000


def microbench_runs(steps, warmup, check=64, ls_list=((2, 2, 2, 2), (3, 3, 3, 3), (4, 4, 4, 4)), precision="fp64"):
    """High-l class microbench: 1e5 independent normalised primitive quartets
    per class, (dd|dd), (ff|ff), (gg|gg), centres in a 6 A box, exponents
    log-uniform [0.1, 100]; inputs and outputs device-resident.  Per class:
    primitive-quartet spherical integrals per second, the generator's FLOP
    count per quartet against the FP64 VALU peak, and the error against the
    CPU oracle on `check` sampled quartets (max abs, RMS, max relative over
    |I| > 1e-10, and the FP64 oracle's own error against long double).
    precision "mixed": the library's HGP_MIXED form (FP32 VRR and contraction
    for the classes that have it; the row records which ran)."""
    import torch
    import oracle
    import paper_2605_10312_amd as hgp
    import workloads
    from paper_2605_10312_amd.gen import phase2 as p2mod, vrr as vrrmod

    out = []
    for ls in ls_list:
        l = ls[0]
        cen, ex = workloads.prim_quartets(l, MICRO_N)
        ct = torch.tensor(cen, device="cuda")
        et = torch.tensor(ex, device="cuda")
        n_sph = int(np.prod([2 * x + 1 for x in ls]))
        res = torch.empty((MICRO_N, n_sph), dtype=torch.float64, device="cuda")
        prec = hgp.HGP_MIXED if precision == "mixed" else hgp.HGP_FP64
        for _ in range(warmup):
            hgp.eri_prim_quartets(ls, ct, et, res, precision=prec)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(steps):
            hgp.eri_prim_quartets(ls, ct, et, res, precision=prec)
        ev1.record()
        torch.cuda.synchronize()
        dt = ev0.elapsed_time(ev1) * 1e-3 / steps
        g = vrrmod.VRRGraph(*ls)
        tg = {tt: f"h{k}" for k, tt in enumerate(g.targets)}
        p2 = p2mod.Phase2(*ls, hname=lambda e, f: tg[(e, f)])
        flop = g.flops() + overhead_flops(sum(ls)) + p2.flops
        err = None
        if check:
            idx = np.random.default_rng(11).choice(MICRO_N, check, replace=False)
            got = res[torch.tensor(idx, device="cuda")].cpu().numpy()
            ref = oracle.eri_prim_quartets(ls, cen[idx], ex[idx]).reshape(check, -1)
            ref_ld = oracle.eri_prim_quartets(ls, cen[idx], ex[idx], precision="long double").reshape(check, -1)
            d = got - ref
            big = np.abs(ref) > 1e-10
            err = {"quartets_checked": int(check), "max_abs": float(np.abs(d).max()),
                   "rms": float(np.sqrt(np.mean(d ** 2))),
                   "max_rel": float((np.abs(d[big]) / np.abs(ref[big])).max()) if big.any() else 0.0,
                   "oracle_fp64_vs_long_double_max_abs": float(np.abs(ref - ref_ld).max()),
                   "max_abs_vs_long_double": float(np.abs(got - ref_ld).max())}
        tag = "".join(str(x) for x in ls)
        nm = "".join("spdfg"[x] for x in ls)
        out.append({"class": f"({nm[:2]}|{nm[2:]})", "tag": tag, "quartets": MICRO_N, "ms_per_step": round(dt * 1e3, 4),
                    "eris_per_s": MICRO_N * n_sph / dt, "flop_per_quartet": flop,
                    "tflops": round(MICRO_N * flop / dt / 1e12, 3),
                    "frac": round(MICRO_N * flop / dt / 1e12 / FP64_VALU_PEAK_TFLOPS, 4), "err": err,
                    "precision": precision, "fp32_form": bool(precision == "mixed" and hgp.class_has_fp32(ls))})
        del res, ct, et
        torch.cuda.empty_cache()
    return out


def microbench(args):
    """One JSON line per high-l class (see microbench_runs)."""
    for r in microbench_runs(args.steps, args.warmup, check=0 if args.no_check else 64, precision=args.precision):
        l = int(r["tag"][0])
        mixed = r["fp32_form"]
        line = {"metric": "primitive-quartet spherical ERIs/s (high-l class microbench)", "value": r["eris_per_s"],
                "unit": "ERIs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                "dtype": "f32/f64 mixed" if mixed else "f64", "data": "synthetic",
                "config": {"workload": f"microbench_{r['tag']}: {MICRO_N} primitive quartets {r['class']}, 6 A box, "
                                       "exponents log-uniform [0.1, 100], " +
                                       ("FP32 VRR and contraction, FP64 Boys/HRR" if mixed else "FP64"),
                           "flop_per_quartet": r["flop_per_quartet"]},
                "roofline": {"bound": "alu", "achieved": r["tflops"], "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                             "frac": r["frac"], "traffic": None},
                "err": r["err"]}
        print(json.dumps(line), flush=True)


def batch(args):
    """Batched uneven systems: many molecules of different size, each with
    its own plan and density, built one after another on one stream and then
    as one captured HIP graph (hgp_batch).  One JSON line: contracted ERIs/s
    over the whole batch for the graph replay, with the sequential time
    beside it."""
    import torch
    import paper_2605_10312_amd as hgp
    import workloads

    n, natom, nprim = args.batch_n, (5, args.batch_max_atoms), (1, args.batch_max_prim)
    systems = workloads.batch_systems(seed=1004, n=n, natom=natom, lmax=3, nprim=nprim)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bases, plans, Ds, Js, Ks = [], [], [], [], []
    eris = 0
    for k, (bw, D) in enumerate(systems):
        if k % 16 == 0:
            print(f"batch: planning system {k}/{n} (N={bw.nbf})", file=sys.stderr, flush=True)
        b = hgp.Basis.from_workload(bw)
        p = hgp.Plan(b, tau=TAU)
        bases.append(b)
        plans.append(p)
        eris += unique_eris(p.schwarz(), np.asarray(bw.l), TAU)[0]     # unique function quartets, as the J/K line
        Dt = torch.tensor(D, dtype=torch.float64, device="cuda")
        Ds.append(Dt)
        Js.append(torch.empty_like(Dt))
        Ks.append(torch.empty_like(Dt))
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    graph = hgp.Batch(plans, Ds, Js, Ks)
    capture_s = time.perf_counter() - t0

    def seq():
        for p, D, J, K in zip(plans, Ds, Js, Ks):
            p.jk(D, J, K)

    def timed(fn, what):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            fn()
            torch.cuda.synchronize()
            print(f"batch: {what} step done", file=sys.stderr, flush=True)
        return (time.perf_counter() - t) / args.steps

    seq_s = timed(seq, "sequential")
    ref = [(J.clone(), K.clone()) for J, K in zip(Js, Ks)]
    graph_s = timed(graph.run, "graph")
    diff = max(max(float((J - r[0]).abs().max()), float((K - r[1]).abs().max())) for J, K, r in zip(Js, Ks, ref))
    # one multi-system plan: each class as one launch over every system's quartets
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    union = hgp.Plan.multi(bases, tau=TAU)
    torch.cuda.synchronize()
    union_setup_s = time.perf_counter() - t0
    union_s = timed(lambda: union.jk_multi(Ds, Js, Ks), "multi-system plan")
    diff_union = max(max(float((J - r[0]).abs().max()), float((K - r[1]).abs().max()))
                     for J, K, r in zip(Js, Ks, ref))
    union_stats = union.stats()
    union.close()
    nbf = [int(bw.nbf) for bw, _ in systems]
    line = {"metric": METRIC, "value": eris / graph_s, "unit": "contracted ERIs/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(graph_s * 1e3, 4),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"batch{n}_4s3p2d1f: {n} synthetic molecules of U{{{natom[0]}..{natom[1]}}} atoms, "
                                   f"4s3p2d1f per atom, U{{{nprim[0]}..{nprim[1]}}} primitives per shell, "
                                   "Schwarz tau=1e-12, J+K in FP64, one HIP graph per step",
                       "systems": n, "nbf_min": min(nbf), "nbf_max": max(nbf), "nbf_sum": sum(nbf),
                       "eris_per_step": int(eris)},
            "sequential_ms": round(seq_s * 1e3, 4), "graph_ms": round(graph_s * 1e3, 4),
            "graph_speedup": round(seq_s / graph_s, 3), "setup_s": round(setup_s, 3),
            "capture_s": round(capture_s, 4), "max_abs_graph_vs_sequential": diff,
            "multi_plan_ms": round(union_s * 1e3, 4), "multi_plan_speedup": round(seq_s / union_s, 3),
            "multi_plan_setup_s": round(union_setup_s, 3), "max_abs_multi_vs_sequential": diff_union,
            "multi_plan_quartets_kept": union_stats["quartets_kept"]}
    print(json.dumps(line), flush=True)
    graph.close()
    for o in plans + bases:
        o.close()


def serving(args):
    """Serving: Poisson arrivals of new systems, each with closed-loop
    density updates through one plan, admitted under an HBM budget and run
    concurrently on several streams.  One JSON line: contracted ERIs/s over
    the window, with offered/achieved rates and p50/p99 latencies."""
    import torch
    import paper_2605_10312_amd as hgp
    import workloads
    from paper_2605_10312_amd import serve

    n, nupd = args.serve_requests, args.serve_updates
    natom = (2, args.serve_max_atoms)
    theta = hgp.MIXED_THETA_DEFAULT if args.precision == "mixed" else 0.0
    systems = workloads.batch_systems(seed=1005, n=n, natom=natom, lmax=4, nprim=(1, 3))
    arrivals = serve.poisson_arrivals(args.serve_rate, n, seed=1005)
    reqs = []
    for i, (bw, D) in enumerate(systems):
        dens = [D] + [workloads.psd_density(bw.nbf, 5000 + 100 * i + k) for k in range(1, nupd)]
        reqs.append(serve.Request(i, float(arrivals[i]), bw, dens, tau=TAU, theta=theta))
    check = set(range(0, n, max(1, n // 4)))       # requests whose last update is checked against FP64 alone
    keep = lambda rid, k: rid in check and k == nupd - 1
    budget = int(args.serve_budget_gb * (1 << 30))
    if args.serve_mode == "iteration":
        ex = serve.GpuMultiExecutor(keep=keep)
        srv = serve.IterationServer(ex, hbm_budget=budget, max_active=args.serve_active)
    else:
        ex = serve.GpuExecutor(slots=args.serve_slots, keep=keep)
        srv = serve.Server(ex, hbm_budget=budget, max_active=args.serve_active, slots=args.serve_slots)
    # warm-up: one small request end to end (library load, table uploads)
    wex = serve.GpuExecutor(slots=1)
    serve.Server(wex, hbm_budget=1 << 34).run([serve.Request(-1, 0.0, reqs[0].basis, reqs[0].densities[:2],
                                                             TAU, theta)])
    torch.cuda.synchronize()
    print(f"serve: {n} requests x {nupd} updates, offered {args.serve_rate}/s", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    recs, ups = srv.run(reqs)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ex.close()
    wex.close()
    summ = serve.summarize(recs, ups, elapsed)
    if args.serve_mode == "iteration":
        summ["plan_rebuilds"] = srv.rebuilds
    eris = ex.eris_done if args.serve_mode == "iteration" else sum(ex.eris[u.rid] for u in ups)
    err = 0.0
    for rid in sorted(check):
        r = reqs[rid]
        b = hgp.Basis.from_workload(r.basis)
        p = hgp.Plan(b, tau=TAU)
        Dt = torch.tensor(r.densities[-1], device="cuda")
        J, K = torch.empty_like(Dt), torch.empty_like(Dt)
        p.jk(Dt, J, K)
        torch.cuda.synchronize()
        Js, Ks = ex.results[(rid, nupd - 1)]
        err = max(err, float(np.abs(J.cpu().numpy() - Js).max()), float(np.abs(K.cpu().numpy() - Ks).max()))
        p.close()
        b.close()
    nbf = [int(r.basis.nbf) for r in reqs]
    line = {"metric": METRIC, "value": eris / elapsed, "unit": "contracted ERIs/s", "n_gpus": 1, "steps": 1,
            "warmup": 1, "ms_per_step": round(elapsed * 1e3, 3), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64" if theta == 0 else "f32/f64 mixed", "data": "synthetic",
            "config": {"workload": f"serve{n}_5s4p3d2f1g: {n} requests, Poisson arrivals at {args.serve_rate}/s, "
                                   f"each a new synthetic molecule of U{{{natom[0]}..{natom[1]}}} atoms (5s4p3d2f1g, "
                                   f"U{{1..3}} primitives per shell) with {nupd} closed-loop density updates "
                                   f"through one plan; HBM budget {args.serve_budget_gb:g} GB, at most "
                                   f"{args.serve_active} active, "
                                   + ("iteration-level batching over one multi-system plan, "
                                      if args.serve_mode == "iteration" else f"{args.serve_slots} streams, ")
                                   + "Schwarz tau=1e-12, "
                                   + ("FP64" if theta == 0 else f"mixed (theta {theta:g})"),
                       "nbf_min": min(nbf), "nbf_max": max(nbf), "eris_total": int(eris)},
            "serve": {k: (round(v, 4) if isinstance(v, float) else v) for k, v in summ.items()},
            "peak_active": srv.peak_active, "peak_plan_bytes": getattr(srv, "peak_bytes", None),
            "max_abs_vs_fp64_alone": err}
    print(json.dumps(line), flush=True)


def plan_sizes(args):
    """Plans at the full sizes of the batched and served workloads' largest
    members: a 60-atom 4s3p2d1f molecule with U{1..8} primitives per shell
    (N = 1800) and a 120-atom 5s4p3d2f1g molecule with U{1..3} (N = 6600),
    grown as the 30-atom workload, tau = 1e-12.  One JSON line per system:
    plan time, quartets kept and streamed, device bytes, and the build's
    algorithmic FLOPs (per class: primitive quartets x VRR FLOPs + quartets x
    Phase-2 FLOPs).  With --plan-jk the 60-atom member's J/K build is also
    run once and timed."""
    import torch
    import paper_2605_10312_amd as hgp
    import workloads

    members = [("batched 60-atom member", 1004, 60, 3, (1, 8)), ("served 120-atom member", 1005, 120, 4, (1, 3))]
    for name, seed, natom, lmax, nprim in members:
        bw = workloads.batch_systems(seed=seed, n=1, natom=(natom, natom), lmax=lmax, nprim=nprim,
                                     with_density=False)[0][0]
        print(f"plan-sizes: {name}: N = {bw.nbf}, {bw.nshell} shells; planning", file=sys.stderr, flush=True)
        b = hgp.Basis.from_workload(bw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan = hgp.Plan(b, tau=TAU)
        torch.cuda.synchronize()
        t_plan = time.perf_counter() - t0
        st = plan.stats()
        cls = plan.classes()
        flop = sum(c["prim_quartets"] * c["vrr_flops"] + c["quartets"] * c["phase2_flops"] for c in cls)
        eris = unique_eris(plan.schwarz(), np.asarray(bw.l), TAU)[0]
        line = {"workload": f"plan_{name.split()[0]}_{natom}atoms", "nbf": int(bw.nbf), "shells": int(bw.nshell),
                "plan_s": round(t_plan, 2), **st, "eris_per_build": int(eris), "build_tflop": round(flop / 1e12, 1),
                "free_device_bytes": int(torch.cuda.mem_get_info()[0])}
        if args.plan_jk and lmax == 3:
            D = torch.tensor(workloads.psd_density(bw.nbf, seed + 1000), device="cuda")
            J, K = torch.empty_like(D), torch.empty_like(D)
            print(f"plan-sizes: {name}: one J/K build ({flop / 1e12:.0f} TFLOP)", file=sys.stderr, flush=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan.jk(D, J, K)
            torch.cuda.synchronize()
            line["jk_s"] = round(time.perf_counter() - t0, 2)
            line["jk_tflops"] = round(flop / 1e12 / line["jk_s"], 2)
            del D, J, K
        print(json.dumps(line), flush=True)
        plan.close()
        b.close()
        torch.cuda.empty_cache()


def sample_quartets(hgp, bw, b, want, seed=2005):
    """`want` uniformly drawn unique shell quartets (i >= j, k >= l, ij >= kl)
    of basis bw that the library's own Schwarz screen keeps (factors of a
    plan at tau 1e-12)."""
    plan = hgp.Plan(b, tau=TAU)
    Q = plan.schwarz()
    plan.close()
    ns = bw.nshell
    rng = np.random.default_rng(seed)
    picked = []
    while len(picked) < want:
        q = rng.integers(0, ns, (4 * want, 4))
        i, j, k, l = q.T
        keep = (i >= j) & (k >= l) & (i * (i + 1) // 2 + j >= k * (k + 1) // 2 + l) & (Q[i, j] * Q[k, l] >= TAU)
        picked.extend(map(tuple, q[keep][: want - len(picked)]))
    return np.array(picked, np.int32)


def sq_bench(args):
    """Contracted integrals (hgp_eri_shell_quartets) of the same 400 000-quartet
    sample as the derivative run, quartet and offset arrays on the device.
    One JSON line: contracted ERIs/s (whole n_sph^4 blocks, as the call
    writes them) and the error of sampled quartets against the long-double
    oracle."""
    import torch
    import oracle
    import paper_2605_10312_amd as hgp
    import workloads

    bw, _ = workloads.molecule_3s2p1d()
    b = hgp.Basis.from_workload(bw)
    quartets = sample_quartets(hgp, bw, b, args.deriv_quartets)
    L = np.asarray(bw.l)
    sizes = np.prod(2 * L[quartets] + 1, axis=1).astype(np.int64)
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    qd, od = torch.tensor(quartets, device="cuda"), torch.tensor(offs, device="cuda")
    out = torch.empty(int(sizes.sum()), dtype=torch.float64, device="cuda")
    for _ in range(args.warmup):
        hgp.eri_shell_quartets(b, qd, od, out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        hgp.eri_shell_quartets(b, qd, od, out)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    o = out.cpu().numpy()
    rng = np.random.default_rng(7)
    errs = []
    for i in rng.choice(len(quartets), 16, replace=False):
        ref = oracle.eri_shell_quartet(bw, *quartets[i], precision="long double")
        own = np.abs(oracle.eri_shell_quartet(bw, *quartets[i]) - ref).max()
        errs.append((np.abs(o[offs[i]:offs[i] + sizes[i]].reshape(ref.shape) - ref).max(), own))
    b.close()
    line = {"metric": "contracted ERIs/s (shell quartets given on the device)", "value": float(sizes.sum()) / dt,
            "unit": "contracted ERIs/s (whole blocks)", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(dt * 1e3, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"sq_mol30_3s2p1d: {len(quartets)} uniformly drawn screened unique shell quartets "
                                   "of the 30-atom 3s2p1d molecule (tau 1e-12), integrals, FP64",
                       "quartets": int(len(quartets))},
            "err": {"quartets_checked": len(errs), "max_abs_vs_long_double": float(max(e[0] for e in errs)),
                    "oracle_fp64_vs_long_double_max_abs": float(max(e[1] for e in errs))}}
    print(json.dumps(line), flush=True)


def deriv_bench(args):
    print(json.dumps(deriv_run(args.deriv_quartets, args.steps, args.warmup, args.cpu_seconds, 8)), flush=True)


def deriv_run(want, steps, warmup, cpu_seconds, n_check):
    """First-derivative integrals (hgp_eri_deriv_shell_quartets) of a uniform
    sample of the 30-atom 3s2p1d workload's screened unique shell quartets,
    quartet and offset arrays on the device.  One JSON line: derivative
    integrals per second (12 n_sph^4 per quartet), the algorithmic FLOP rate
    of the derivative program (per class: primitive quartets x per-primitive
    FLOPs + quartets x Phase-2 FLOPs of gen/emit_deriv.py; the staged form's
    recomputation is not counted) against the FP64 peak, the error of
    sampled quartets against the long-double oracle, and the oracle timed on
    the host cores."""
    import torch
    import oracle
    import paper_2605_10312_amd as hgp
    import workloads

    bw, _ = workloads.molecule_3s2p1d()
    b = hgp.Basis.from_workload(bw)
    quartets = sample_quartets(hgp, bw, b, want)
    sizes = np.array([12 * int(np.prod([2 * bw.l[s] + 1 for s in q])) for q in quartets], np.int64)
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    qd = torch.tensor(quartets, device="cuda")
    od = torch.tensor(offs, device="cuda")
    out = torch.empty(int(sizes.sum()), dtype=torch.float64, device="cuda")
    for _ in range(warmup):
        hgp.eri_shell_quartets(b, qd, od, out, deriv=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        hgp.eri_shell_quartets(b, qd, od, out, deriv=True)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    # algorithmic FLOPs of the tables
    info = {d["tag"]: d for d in json.load(open(os.path.join(os.path.dirname(os.path.abspath(hgp.__file__)),
                                                               "_gen", "deriv.json")))}
    nprim = np.asarray(bw.nprim)
    flop = 0.0
    for q in quartets:
        ls = [int(bw.l[s]) for s in q]
        a_, b_ = sorted(ls[:2], reverse=True)
        c_, d_ = sorted(ls[2:], reverse=True)
        if (a_ * (a_ + 1) // 2 + b_) < (c_ * (c_ + 1) // 2 + d_):
            a_, b_, c_, d_ = c_, d_, a_, b_
        t = info[f"{a_}{b_}{c_}{d_}"]
        flop += float(np.prod(nprim[list(q)])) * t["vrr_flops"] + t["p2_flops"]
    got = out.cpu().numpy()
    rng = np.random.default_rng(2006)
    chk = rng.choice(len(quartets), n_check, replace=False)
    errs = []
    for i in chk:
        ref = oracle.eri_deriv_shell_quartet(bw, *quartets[i], precision="long double")
        own = np.abs(oracle.eri_deriv_shell_quartet(bw, *quartets[i]) - ref).max()
        g = got[offs[i]:offs[i] + sizes[i]].reshape(ref.shape)
        errs.append((np.abs(g - ref).max(), np.abs(ref).max(), own))
    # the oracle on the host cores: the same derivative blocks of a bounded sample
    t0 = time.perf_counter()
    n_cpu = 0
    ints_cpu = 0
    while time.perf_counter() - t0 < cpu_seconds / 3 and n_cpu < len(quartets):
        oracle.eri_deriv_shell_quartet(bw, *quartets[n_cpu])
        ints_cpu += int(sizes[n_cpu])
        n_cpu += 1
    cpu_rate = ints_cpu / (time.perf_counter() - t0) if n_cpu else None
    value = float(sizes.sum()) / dt
    line = {"metric": "first-derivative contracted integrals/s", "value": value, "unit": "derivative integrals/s",
            "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": round(dt * 1e3, 3),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"deriv_mol30_3s2p1d: {len(quartets)} uniformly drawn screened unique shell "
                                   "quartets of the 30-atom 3s2p1d molecule (tau 1e-12), d/dR of all four centres, "
                                   "12 blocks each, FP64",
                       "quartets": int(len(quartets))},
            "roofline": {"bound": "alu", "kernel": "all derivative kernels (dreg_*, dp1_*, t3w_deriv_kernel)",
                         "achieved": round(flop / dt / 1e12, 3),
                         "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(flop / dt / 1e12 / FP64_VALU_PEAK_TFLOPS, 4), "traffic": None},
            "cpu_baseline": None if not n_cpu else {
                "value": cpu_rate, "unit": "derivative integrals/s", "cores": oracle.num_threads(), "kind": "oracle",
                "sample": f"the first {n_cpu} quartets of the same sample, one at a time (oracle_eri_deriv_shell_quartet)"},
            "err": None if not errs else {
                "quartets_checked": len(chk), "max_abs_vs_long_double": float(max(e[0] for e in errs)),
                "oracle_fp64_vs_long_double_max_abs": float(max(e[2] for e in errs)),
                "max_abs_derivative": float(max(e[1] for e in errs))}}
    b.close()
    return line


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-high-l", action="store_true", help="skip the high-l class microbench in the default run")
    ap.add_argument("--no-deriv", action="store_true", help="skip the first-derivative run in the default run")
    ap.add_argument("--precision", choices=("fp64", "mixed"), default="fp64",
                    help="mixed: quartets with Q_ab Q_cd < theta use FP32 VRR and contraction (register tier; HRR, Boys, J/K FP64)")
    ap.add_argument("--theta", type=float, default=None, help="mixed-precision threshold (default: the library's)")
    ap.add_argument("--workload", choices=("mol30", "microbench", "batch", "serve", "plan-sizes", "deriv", "sq"),
                    default="mol30",
                    help="mol30: the J/K build (one JSON line); microbench: the high-l primitive-quartet classes; "
                         "batch: many uneven systems in one HIP graph; serve: continuous batching of requests; "
                         "plan-sizes: plans of the batched and served workloads' largest members; "
                         "deriv: first-derivative integrals of sampled quartets of the 30-atom workload")
    ap.add_argument("--deriv-quartets", type=int, default=400000, help="deriv: quartets in the sample")
    ap.add_argument("--plan-jk", action="store_true", help="plan-sizes: also run the 60-atom member's J/K once")
    ap.add_argument("--serve-requests", type=int, default=64)
    ap.add_argument("--serve-updates", type=int, default=10)
    ap.add_argument("--serve-rate", type=float, default=200.0, help="offered requests per second")
    ap.add_argument("--serve-max-atoms", type=int, default=6)
    ap.add_argument("--serve-budget-gb", type=float, default=64.0)
    ap.add_argument("--serve-active", type=int, default=16)
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--serve-mode", choices=("continuous", "iteration"), default="iteration",
                    help="continuous: each request's updates on its own stream; iteration: every step one "
                         "multi-system plan over the active requests")
    ap.add_argument("--batch-n", type=int, default=64, help="batch: number of systems")
    ap.add_argument("--batch-max-atoms", type=int, default=15, help="batch: atoms per system U{5..this}")
    ap.add_argument("--batch-max-prim", type=int, default=3, help="batch: primitives per shell U{1..this}")
    ap.add_argument("--serial", action="store_true",
                    help="run the timed J/K builds with every class on one stream (for kernel profiles whose "
                         "per-kernel durations must match the event-timed ones)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run one plain device copy kernel (y = 1.0 * x, MIB MiB of FP64 each way), "
                         "a known-size reference for hardware byte counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    if args.workload == "microbench":
        microbench(args)
        return
    if args.workload == "batch":
        batch(args)
        return
    if args.workload == "serve":
        serving(args)
        return
    if args.workload == "plan-sizes":
        plan_sizes(args)
        return
    if args.workload == "sq":
        sq_bench(args)
        return
    if args.workload == "deriv":
        deriv_bench(args)
        return

    import torch
    import paper_2605_10312_amd as hgp
    import workloads

    if args.copy_calibration > 0:
        x = torch.ones(args.copy_calibration << 17, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        torch.mul(x, 1.0, out=y)
        torch.cuda.synchronize()
        del x, y

    bw, D = workloads.molecule_3s2p1d()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    basis = hgp.Basis.from_workload(bw)
    theta = 0.0
    if args.precision == "mixed":
        theta = hgp.MIXED_THETA_DEFAULT if args.theta is None else args.theta
    plan = hgp.Plan(basis, tau=TAU, theta=theta)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    classes = plan.classes()
    stats = plan.stats()
    # unique (8-fold) spherical function quartets of the kept shell quartets, from
    # the plan's own Schwarz factors; the kernels compute whole blocks
    blocks = sum(c["quartets"] * np.prod([nsph(x) for x in c["ls"]]) for c in classes)
    eris, nkept = unique_eris(plan.schwarz(), np.asarray(bw.l), TAU)
    if nkept != stats["quartets_kept"]:
        print(f"warning: the ERI count's screen keeps {nkept} shell quartets, the plan {stats['quartets_kept']}",
              file=sys.stderr, flush=True)

    Dt = torch.tensor(D, dtype=torch.float64, device="cuda")
    J = torch.empty_like(Dt)
    K = torch.empty_like(Dt)
    plan.set_timing(args.serial)         # --serial: every class on one stream, warm-up included
    for _ in range(args.warmup):
        plan.jk(Dt, J, K)
    torch.cuda.synchronize()
    # timed steps: the plan runs its scratch-free class lists concurrently on
    # several streams (with --serial, all on one stream, as while timing kernels)
    plan.set_timing(args.serial)         # also resets the per-class counters
    t = time.perf_counter()
    for _ in range(args.steps):
        plan.jk(Dt, J, K)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t
    ms_per_step = 1e3 * elapsed / args.steps
    # per-kernel durations: HIP events around each class kernel, which makes the
    # plan run every class on the one stream so that no kernel's interval is
    # stretched by another's (the timed steps above were concurrent unless --serial)
    if not args.serial:
        plan.set_timing(True)
        for _ in range(args.steps):
            plan.jk(Dt, J, K)
        torch.cuda.synchronize()
    timing = plan.class_timing()

    # one entry per kernel: register tier jk_<class>; staged tier p1_<class> (Phase 1)
    # and jk_<class> (Phase 2 + digestion); average duration per launch from HIP events
    per_kernel = []
    for c, t in zip(classes, timing):
        tag = "".join(str(x) for x in c["ls"])
        f1, f2 = phase_flops(c)
        if t["tier"] == 0:
            parts = [(f"jk{'32' if c['bits'] == 32 else ''}_{tag}", f1 + f2, t["kernels"][0])]
        elif t["tier"] == 2:
            parts = [(f"t3_jk_{tag}", f1 + f2, t["kernels"][0])]
        else:
            parts = [(f"p1_{tag}", f1, t["kernels"][0]), (f"jk_{tag}", f2, t["kernels"][1])]
        for name, fl, (n, ms) in parts:
            launches_per_step = max(n, 1) / args.steps
            avg = ms / max(n, 1)
            per_kernel.append({"kernel": name, "tier": t["tier"], "quartets": c["quartets"],
                               "prim_quartets": c["prim_quartets"], "avg_ms": round(avg, 4),
                               "ms_per_step": round(ms / args.steps, 4),
                               "gflop_per_launch": round(fl / launches_per_step / 1e9, 3),
                               "tflops": round(fl / launches_per_step / (avg * 1e-3) / 1e12, 3) if avg > 0 else None})
    per_kernel.sort(key=lambda x: -x["ms_per_step"])
    res = kernel_resources()
    for x in per_kernel:
        x.update(res.get(x["kernel"], {}))
    dom = per_kernel[0]
    achieved = dom["tflops"]
    roofline = {"bound": "alu", "kernel": dom["kernel"], "achieved": achieved, "peak": FP64_VALU_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / FP64_VALU_PEAK_TFLOPS, 4),
                "traffic": measured_traffic(dom["kernel"]),
                "avg_launch_ms": dom["avg_ms"], "gflop_per_launch": dom["gflop_per_launch"]}
    total_kernel_ms = sum(x["ms_per_step"] for x in per_kernel)
    total_flops = sum(algorithmic_flops(c) for c in classes)

    err_fp64 = None
    if args.precision == "mixed":
        # the same build in plain FP64, untimed: the mixed result's deviation from it
        p64 = hgp.Plan(basis, tau=TAU)
        J64 = torch.empty_like(Dt)
        K64 = torch.empty_like(Dt)
        p64.jk(Dt, J64, K64)
        torch.cuda.synchronize()
        err_fp64 = {"J_max_abs": float((J - J64).abs().max()), "K_max_abs": float((K - K64).abs().max()),
                    "fp32_quartet_share": round(sum(c["quartets"] for c in classes if c["bits"] == 32) /
                                                max(1, sum(c["quartets"] for c in classes)), 4), "theta": theta}
        p64.close()

    # J/K of the configuration that was timed (concurrent class lists unless
    # --serial): the per-kernel timing pass above ran every class on one stream
    plan.set_timing(False)
    plan.jk(Dt, J, K)
    torch.cuda.synchronize()
    err = None if args.no_check else block_errors(bw, J.cpu().numpy(), K.cpu().numpy())

    cpu = None if args.no_cpu_baseline else cpu_baseline(bw, args.cpu_seconds)
    # the high-l classes, which this workload (l <= 2) does not reach
    high_l = None if args.no_high_l else microbench_runs(2, 1, check=0 if args.no_check else 32)
    # first-derivative integrals of a sample of the same molecule's quartets
    deriv = None
    if not args.no_deriv:
        d = deriv_run(args.deriv_quartets, 3, 1, 0.0, 0 if args.no_check else 4)
        deriv = {k: d[k] for k in ("metric", "value", "unit", "ms_per_step", "dtype", "config", "roofline", "err")}

    line = {
        "metric": METRIC,
        "value": eris / (ms_per_step * 1e-3),
        "unit": "contracted ERIs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32/f64 mixed",
        "data": "synthetic",
        "config": {"workload": "mol30_3s2p1d: 30-atom synthetic molecule, 3s2p1d per atom (1-6 primitives), "
                               "N=420, Schwarz tau=1e-12, J+K " +
                               ("in FP64" if args.precision == "fp64" else
                                f"mixed (FP32 VRR and contraction below Schwarz bound {theta:g}, register tier; FP64 Boys, HRR and J/K)"),
                   "nbf": int(bw.nbf), "shells": int(bw.nshell), "tau": TAU,
                   "quartets_kept": stats["quartets_kept"], "quartets_total": stats["quartets_total"],
                   "prim_pairs_kept": stats["prim_pairs_kept"], "prim_pairs_total": stats["prim_pairs_total"],
                   "eris_per_step": int(eris), "eri_block_elements_per_step": int(blocks),
                   "eri_count_quartets": int(nkept),
                   "eris_counted_as": "unique (8-fold) spherical function quartets of the kept shell quartets"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "jk_build_ms": round(ms_per_step, 4),
        "setup_s": round(setup_s, 3),
        "step_tflops": round(total_flops / (ms_per_step * 1e-3) / 1e12, 3),
        "kernel_ms_sum": round(total_kernel_ms, 4),
        "class_streams": "one" if args.serial else "concurrent (caller's stream + 3 side streams)",
        "err": err,
        "err_vs_fp64": err_fp64,
        "kernels": per_kernel,
        "high_l_microbench": high_l,
        "first_derivatives": deriv,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
