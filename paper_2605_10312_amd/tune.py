"""Autotuner for the per-class kernel choices on gfx950.

The router's register model picks each class's tier and staged chunk cap
from its VRR graph.  It cannot see occupancy effects or how the compiler
schedules the digestion, so the choices are checked on the hardware.

    python -m paper_2605_10312_amd.tune build             (CPU: variant libraries)
    python -m paper_2605_10312_amd.tune measure --out F   (GPU: time every variant)
    python -m paper_2605_10312_amd.tune select F          (CPU: write the tuning table)
    python -m paper_2605_10312_amd.tune refine --variants V.. --out F
                                                          (GPU: time variants beside the current
                                                           library; adopt clear per-class wins)

`build` generates one complete library per variant into _variants/.  A
variant is a set of generator options applied to every class (waves per
SIMD, digestion style, staged cap).  `measure` runs each library in a child
process on the 30-atom 3s2p1d workload.  The child times every class kernel
with HIP events and reports milliseconds per J/K build.  `select` keeps, for
each class, the fastest variant and writes its options to tuning/gfx950.json.
The router reads that file in the next ordinary build.
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
VARIANTS_DIR = os.path.join(HERE, "_variants")
TABLE = os.path.join(HERE, "tuning", "gfx950.json")

# generator options per variant; keys the tier does not use are ignored
VARIANTS = {
    "seg": {"digest": "loads_first", "reduce": "segmented"},
    "seg_il": {"digest": "interleaved", "reduce": "segmented"},
    "seg_pf": {"digest": "loads_first", "reduce": "segmented", "loop": "prefetch"},
    "seg_w2": {"digest": "loads_first", "reduce": "segmented", "waves": 2},
    "b64": {"digest": "loads_first", "reduce": "segmented", "block": 64},
    "b64_il": {"digest": "interleaved", "reduce": "segmented", "block": 64},
    "b64_pf": {"digest": "loads_first", "reduce": "segmented", "block": 64, "loop": "prefetch"},
    "b64_w2": {"digest": "loads_first", "reduce": "segmented", "block": 64, "waves": 2},
    "b128": {"digest": "loads_first", "reduce": "segmented", "block": 128},
    "cap64": {"digest": "loads_first", "reduce": "segmented", "cap": 64},
    "cap48": {"digest": "loads_first", "reduce": "segmented", "cap": 48},
    "staged": {"digest": "loads_first", "reduce": "segmented", "tier": 1},
    "plain": {"digest": "interleaved", "reduce": "none"},
    "row_b180": {"digest": "loads_first", "reduce": "segmented", "budget": 180},
    "row_b200": {"digest": "loads_first", "reduce": "segmented", "budget": 200},
}
# timing workloads: the 30-atom 3s2p1d molecule (l <= 2 classes) and a
# 15-atom 4s3p2d1f molecule of the batched-systems recipe (l <= 3 classes)
WORKLOADS = ("mol30", "f15")
# Measured and dropped: 6 or 8 waves per SIMD forced on every l <= 2 class
# (block 64, with and without prefetch) spills and ran 1.04-15x slower than
# the tuned choice on every class.


def build_variants(names, lmax):
    from . import build as b
    os.makedirs(VARIANTS_DIR, exist_ok=True)
    for name in names:
        t = time.time()
        gen = os.path.join(b.ROOT, "_build", "gen_" + name)
        out = os.path.join(VARIANTS_DIR, f"libhgp_{name}.so")
        b.build(lmax, verbose=False, out=out, gen_dir=gen, defaults=VARIANTS[name], table={}, allow_scratch=True)
        print(f"built variant {name} -> {out} in {time.time() - t:.1f}s", flush=True)


def time_library(steps, warmup, workload="mol30"):
    """Child process: per-class milliseconds per J/K build with the library named by HGP_LIB."""
    import torch
    import paper_2605_10312_amd as hgp
    import workloads

    if workload == "f15":
        bw, D = workloads.batch_systems(seed=1006, n=1, natom=(15, 15), lmax=3, nprim=(1, 3))[0]
    else:
        bw, D = workloads.molecule_3s2p1d()
    basis = hgp.Basis.from_workload(bw)
    plan = hgp.Plan(basis, tau=1e-12)
    Dt = torch.tensor(D, dtype=torch.float64, device="cuda")
    J = torch.empty_like(Dt)
    K = torch.empty_like(Dt)
    for _ in range(warmup):
        plan.jk(Dt, J, K)
    torch.cuda.synchronize()
    plan.set_timing(True)
    t = time.perf_counter()
    for _ in range(steps):
        plan.jk(Dt, J, K)
    torch.cuda.synchronize()
    total = (time.perf_counter() - t) * 1e3 / steps
    res = {}
    for c, tm in zip(plan.classes(), plan.class_timing()):
        tag = "".join(str(x) for x in c["ls"])
        res[tag] = {"tier": tm["tier"], "ms": sum(ms for _, ms in tm["kernels"]) / steps}
    plan.close()
    basis.close()
    print(json.dumps({"ms_per_build": total, "classes": res}), flush=True)


def measure(names, out, steps, warmup, timeout):
    results = {}
    for name in names:
        lib = os.path.join(VARIANTS_DIR, f"libhgp_{name}.so")
        if not os.path.exists(lib):
            raise FileNotFoundError(f"{lib}: run `python -m paper_2605_10312_amd.tune build` first")
        env = dict(os.environ, HGP_LIB=lib)
        print(f"== variant {name}", flush=True)
        r = subprocess.run([sys.executable, "-m", "paper_2605_10312_amd.tune", "_time", "--steps", str(steps),
                            "--warmup", str(warmup)], env=env, capture_output=True, text=True, timeout=timeout)
        if r.returncode != 0:
            print(r.stderr[-3000:], flush=True)
            raise SystemExit(f"variant {name} failed with status {r.returncode}")
        results[name] = json.loads(r.stdout.strip().splitlines()[-1])
        print(f"   {results[name]['ms_per_build']:.2f} ms per J/K build", flush=True)
        with open(out, "w") as fh:
            json.dump(results, fh, indent=1)


def refine(names, out, steps, warmup, timeout, margin=0.02, table=TABLE, workload="mol30", min_l=0):
    """Time the current library (the package's libhgp.so, built from the
    tuning table) beside the named variants in one session, and adopt a
    variant's options for a class only where it beats the current choice by
    more than `margin` (and only for classes with a shell of l >= min_l)."""
    from . import LIB_PATH
    results = {}
    for name, lib in [("current", LIB_PATH)] + [(n, os.path.join(VARIANTS_DIR, f"libhgp_{n}.so")) for n in names]:
        if not os.path.exists(lib):
            raise FileNotFoundError(lib)
        print(f"== {name}", flush=True)
        r = subprocess.run([sys.executable, "-m", "paper_2605_10312_amd.tune", "_time", "--steps", str(steps),
                            "--warmup", str(warmup), "--workload", workload], env=dict(os.environ, HGP_LIB=lib),
                           capture_output=True, text=True, timeout=timeout)
        if r.returncode != 0:
            print(r.stderr[-3000:], flush=True)
            raise SystemExit(f"{name} failed with status {r.returncode}")
        results[name] = json.loads(r.stdout.strip().splitlines()[-1])
        print(f"   {results[name]['ms_per_build']:.2f} ms per J/K build", flush=True)
    with open(out, "w") as fh:
        json.dump(results, fh, indent=1)
    apply_refine(out, margin, table, min_l)


def spills(name, tag):
    """True when variant `name` compiled class `tag` with private scratch (a
    register spill): such a variant is never adopted, however fast."""
    from . import build as b
    lib = os.path.join(VARIANTS_DIR, f"libhgp_{name}.so")
    path = b.resources_path(lib)
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path}: the variant's resource report is missing; rebuild it")
    return b.class_scratch(json.load(open(path)), tag) > 0


def apply_refine(path, margin=0.02, table=TABLE, min_l=0):
    """The table update of `refine`, from its saved timings."""
    results = json.load(open(path))
    cur = json.load(open(table))
    for tag, c in results["current"]["classes"].items():
        if max(int(x) for x in tag) < min_l:
            continue
        best = min(((r["classes"][tag]["ms"], n) for n, r in results.items()
                    if n != "current" and tag in r["classes"] and r["classes"][tag]["tier"] == c["tier"]
                    and not spills(n, tag)),
                   default=None)
        if best and best[0] < (1.0 - margin) * c["ms"]:
            opts = {"tier": c["tier"]}
            opts.update(VARIANTS[best[1]])
            if opts["tier"] == 1:
                opts = {k: v for k, v in opts.items() if k in ("tier", "cap", "waves", "reduce", "loop", "budget")}
            opts["variant"] = best[1]
            opts["ms"] = round(best[0], 4)
            print(f"{tag}: {c['ms']:.3f} -> {best[0]:.3f} ms with {best[1]}")
            cur["classes"][tag] = opts
    with open(table, "w") as fh:
        json.dump(cur, fh, indent=1)
    print(f"updated {table}")


def select(path, table=TABLE):
    from .gen import router
    rerouted = router.load_reroutes(table)      # kept: the build's compile-feedback routes
    res = json.load(open(path))
    classes = sorted({t for r in res.values() for t in r["classes"]})
    chosen = {}
    for tag in classes:
        cands = [(r["classes"][tag]["ms"], name) for name, r in res.items()
                 if tag in r["classes"] and not spills(name, tag)]
        if not cands:
            print(f"{tag}: every variant spills; left to the model")
            continue
        best = min(cands)
        opts = {"tier": res[best[1]]["classes"][tag]["tier"]}
        opts.update({k: v for k, v in VARIANTS[best[1]].items()})
        if opts["tier"] == 1:
            opts = {k: v for k, v in opts.items() if k in ("tier", "cap", "waves", "reduce", "loop")}
        opts["variant"] = best[1]
        opts["ms"] = round(best[0], 4)
        chosen[tag] = opts
        print(f"{tag}: {best[1]:8s} {best[0]:8.3f} ms  " +
              "  ".join(f"{n}={r['classes'][tag]['ms']:.3f}" for n, r in res.items() if tag in r["classes"]))
    os.makedirs(os.path.dirname(table), exist_ok=True)
    with open(table, "w") as fh:
        json.dump({"device": "gfx950", "workload": "mol30_3s2p1d, tau 1e-12", "classes": chosen,
                   "rerouted": rerouted}, fh, indent=1)
    print(f"wrote {table}; estimated J/K build {sum(c['ms'] for c in chosen.values()):.2f} ms")


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    pb = sub.add_parser("build")
    pb.add_argument("--variants", nargs="*", default=list(VARIANTS))
    pb.add_argument("--lmax", type=int, default=2)
    pm = sub.add_parser("measure")
    pm.add_argument("--variants", nargs="*", default=list(VARIANTS))
    pm.add_argument("--out", required=True)
    pm.add_argument("--steps", type=int, default=3)
    pm.add_argument("--warmup", type=int, default=1)
    pm.add_argument("--timeout", type=float, default=120.0)
    pr = sub.add_parser("refine")
    pr.add_argument("--variants", nargs="*", required=True)
    pr.add_argument("--out", required=True)
    pr.add_argument("--steps", type=int, default=3)
    pr.add_argument("--warmup", type=int, default=1)
    pr.add_argument("--timeout", type=float, default=180.0)
    pr.add_argument("--workload", choices=WORKLOADS, default="mol30")
    pr.add_argument("--min-l", type=int, default=0, help="adopt only for classes with a shell of l >= this")
    pa = sub.add_parser("apply")
    pa.add_argument("results")
    pa.add_argument("--min-l", type=int, default=0, help="adopt only for classes with a shell of l >= this")
    ps = sub.add_parser("select")
    ps.add_argument("results")
    pt = sub.add_parser("_time")
    pt.add_argument("--steps", type=int, default=3)
    pt.add_argument("--warmup", type=int, default=1)
    pt.add_argument("--workload", choices=WORKLOADS, default="mol30")
    a = ap.parse_args(argv)
    if a.cmd == "build":
        build_variants(a.variants, a.lmax)
    elif a.cmd == "measure":
        measure(a.variants, a.out, a.steps, a.warmup, a.timeout)
    elif a.cmd == "refine":
        refine(a.variants, a.out, a.steps, a.warmup, a.timeout, workload=a.workload, min_l=a.min_l)
    elif a.cmd == "apply":
        apply_refine(a.results, min_l=a.min_l)
    elif a.cmd == "select":
        select(a.results)
    else:
        time_library(a.steps, a.warmup, a.workload)


if __name__ == "__main__":
    main(sys.argv[1:])
