"""Build libhgp.so for gfx950: generate the class kernels, compile every HIP
translation unit with hipcc and link the shared library in-tree.

    python -m paper_2605_10312_amd.build [--lmax 2] [--jobs 8] [--force]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import hashlib
import json
import os
import shutil
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
GEN = os.path.join(HERE, "_gen")
OBJ = os.path.join(ROOT, "_build", "obj")
LIB = os.path.join(HERE, "libhgp.so")
INCLUDE = os.path.join(ROOT, "include")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-munsafe-fp-atomics",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", CSRC, "-I", INCLUDE]
DEFAULT_LMAX = 4


REGISTER_OPTS = ("waves", "digest", "reduce", "loop", "block")
STAGED_OPTS = ("cap", "waves", "reduce", "loop")


def generate(lmax: int = DEFAULT_LMAX, verbose: bool = False, table=None, overrides=None, gen_dir: str = GEN,
             defaults=None):
    """Write one .hip per canonical class plus the class table into gen_dir.
    Each class is routed to the register or staged tier (gen/router.py).
    defaults (generator options for every class) are applied first, then
    the router's choice (tuning table, else the register model), then
    overrides, a map from class tag to options that wins over both.
    Register-tier options: waves, digest, reduce, loop, block; staged: cap,
    waves, reduce, loop."""
    from .gen import emit, emit_staged, emit_t3, router
    from .gen.cart import canonical_classes

    GEN = gen_dir
    os.makedirs(GEN, exist_ok=True)
    metas = []
    files = []
    for ls in canonical_classes(lmax):
        tag = "".join(str(x) for x in ls)
        r = router.route(ls, table)
        for k, v in (defaults or {}).items():
            if r["source"] == "model" or k not in r:    # a tuning-table entry wins over defaults
                r[k] = v
        if overrides and tag in overrides:
            r.update(overrides[tag])
        if r["tier"] == 2:
            src, meta = emit_t3.emit_class_t3(*ls)
        elif r["tier"] == 1:
            src, meta = emit_staged.emit_class_staged(*ls, **{k: r[k] for k in STAGED_OPTS if k in r})
        else:
            src, meta = emit.emit_class(*ls, **{k: r[k] for k in REGISTER_OPTS if k in r})
        path = os.path.join(GEN, f"class_{meta.tag}.hip")
        _write_if_changed(path, src)
        files.append(path)
        metas.append(meta)
        if verbose:
            print(f"  class {meta.tag}: {meta.vrr_nodes} VRR nodes, PeakLive {meta.peak_live} ({meta.scheduler}), "
                  f"N_hrr {meta.n_hrr}", flush=True)
    table = os.path.join(GEN, "class_table.hip")
    _write_if_changed(table, emit.emit_table(metas))
    files.append(table)
    _write_if_changed(os.path.join(GEN, "classes.json"),
                      json.dumps([m.__dict__ for m in metas], indent=1, default=list))
    for f in os.listdir(GEN):          # drop classes of an earlier, larger lmax
        p = os.path.join(GEN, f)
        if f.endswith(".hip") and p not in files:
            os.remove(p)
    return files, metas


def _write_if_changed(path, text):
    if os.path.exists(path) and open(path).read() == text:
        return
    with open(path + ".tmp", "w") as fh:
        fh.write(text)
    os.replace(path + ".tmp", path)


def class_source_hash(tag: str, gen_dir: str = GEN) -> str | None:
    """Hash of everything a generated class kernel is compiled from (its
    source and the device headers): measurements tied to a kernel, such as
    hardware byte counters, stay valid only while this is unchanged."""
    src = os.path.join(gen_dir, f"class_{tag}.hip")
    if not os.path.exists(src):
        return None
    h = hashlib.sha256()
    for d in [src] + [os.path.join(CSRC, x) for x in ("hgp_device.h", "hgp_types.h", "hgp_t3.h")]:
        h.update(open(d, "rb").read())
    return h.hexdigest()[:16]


def _compile(src: str, force: bool):
    if not src.startswith(CSRC + os.sep):  # generated class files see only these headers
        deps = [src] + [os.path.join(CSRC, h) for h in ("hgp_device.h", "hgp_types.h", "hgp_t3.h")]
    else:
        deps = [src] + [os.path.join(CSRC, f) for f in sorted(os.listdir(CSRC)) if f.endswith(".h")] + \
               [os.path.join(INCLUDE, f) for f in sorted(os.listdir(INCLUDE))]
    h = hashlib.sha256(" ".join(FLAGS).encode())
    for d in deps:
        h.update(open(d, "rb").read())
    obj = os.path.join(OBJ, os.path.basename(src) + "." + h.hexdigest()[:16] + ".o")
    if os.path.exists(obj) and not force:
        return obj, 0.0
    t = time.time()
    cmd = [HIPCC] + FLAGS + ["-c", src, "-o", obj + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-4000:]}")
    os.replace(obj + ".tmp", obj)
    return obj, time.time() - t


def build(lmax: int = DEFAULT_LMAX, jobs: int | None = None, force: bool = False, verbose: bool = True,
          overrides=None, out: str | None = None, gen_dir: str = GEN, defaults=None, table=None) -> str:
    """Generate, compile and link; out (default: the package's libhgp.so)
    and gen_dir let a tuning run build variant libraries side by side."""
    t0 = time.time()
    os.makedirs(OBJ, exist_ok=True)
    gen_files, metas = generate(lmax, verbose=False, overrides=overrides, gen_dir=gen_dir, defaults=defaults,
                                table=table)
    srcs = [os.path.join(CSRC, f) for f in sorted(os.listdir(CSRC)) if f.endswith(".hip")] + gen_files
    jobs = jobs or min(8, os.cpu_count() or 4)
    objs = []
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = {ex.submit(_compile, s, force): s for s in srcs}
        for f in cf.as_completed(futs):
            obj, dt = f.result()
            objs.append(obj)
            if verbose and dt > 0:
                print(f"  compiled {os.path.basename(futs[f])} in {dt:.1f}s", flush=True)
    objs.sort()
    lib = out or LIB
    tmp = lib + ".tmp"
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-4000:]}")
    os.replace(tmp, lib)
    if verbose:
        staged = [m.tag for m in metas if m.tier == 1]
        t3 = [m.tag for m in metas if m.tier == 2]
        t3w = [m.tag for m in metas if m.tier == 3]
        print(f"built {lib} ({len(metas)} classes, l <= {lmax}, staged: {' '.join(staged) or 'none'}, "
              f"HBM scratch: {' '.join(t3) or 'none'}, wave LDS: {' '.join(t3w) or 'none'}) "
              f"in {time.time() - t0:.1f}s", flush=True)
    return lib


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--lmax", type=int, default=DEFAULT_LMAX)
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--force", action="store_true")
    a = ap.parse_args(argv)
    build(a.lmax, a.jobs, a.force)


if __name__ == "__main__":
    main(sys.argv[1:])
