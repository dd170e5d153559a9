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
# the compiler's per-kernel resource report (registers, scratch, LDS, occupancy)
REMARKS = ["-Rpass-analysis=kernel-resource-usage"]


REGISTER_OPTS = ("waves", "digest", "reduce", "loop", "block")
STAGED_OPTS = ("cap", "waves", "reduce", "loop", "jk_digest")
ROW_OPTS = ("budget", "waves", "reduce", "loop", "eri_layout", "jk_digest")


_EMITTED: dict = {}     # (class, routing inputs) -> (source, meta): a rerouting pass regenerates only what changed


def _route_and_emit(ls, table, defaults, override, reroute):
    """Route one class (router model or tuning table, then defaults,
    overrides and the build's rerouting) and emit its source."""
    from .gen import emit, emit_row, emit_staged, emit_t3, router
    r = router.route(ls, table)
    for k, v in (defaults or {}).items():
        if r["source"] == "model" or k not in r:    # a tuning-table entry wins over defaults
            r[k] = v
    if override:
        r.update(override)
    if reroute:
        if reroute.get("tier") == 1 and r.get("tier") != 1 and "form" not in reroute:
            r["form"] = router.model_form(ls)
            if r["form"] == "row":
                r["budget"] = router.ROW_BUDGET
            elif "cap" not in reroute:
                r["cap"] = router.model_cap(ls)
        r.update(reroute)
    if r["tier"] in (2, 3):
        src, meta = emit_t3.emit_class_t3(*ls)
    elif r["tier"] == 1 and r.get("form") == "row":
        src, meta = emit_row.emit_class_row(*ls, **{k: r[k] for k in ROW_OPTS if k in r})
    elif r["tier"] == 1:
        src, meta = emit_staged.emit_class_staged(*ls, **{k: r[k] for k in STAGED_OPTS if k in r})
    else:
        src, meta = emit.emit_class(*ls, **{k: r[k] for k in REGISTER_OPTS if k in r})
    meta.route = {k: v for k, v in r.items() if k not in ("variant", "ms")}
    meta.route["rerouted"] = bool(reroute)
    return src, meta


def generate(lmax: int = DEFAULT_LMAX, verbose: bool = False, table=None, overrides=None, gen_dir: str = GEN,
             defaults=None, reroute=None, jobs: int | None = None, dreg_off=frozenset(), dstage=None):
    """Write one .hip per canonical class plus the class table into gen_dir.
    Each class is routed to a tier (gen/router.py): defaults (generator
    options for every class) are applied first, then the router's choice
    (tuning table, else the register model), then overrides, a map from
    class tag to options that wins over both.  Register-tier options: waves,
    digest, reduce, loop, block; staged: cap, waves, reduce, loop; row form:
    budget, waves, reduce, loop.  reroute (class tag -> options) is applied
    last: the build's answer to a compiler resource report that showed
    spills.  Classes are generated in parallel processes.  Derivative
    classes small enough for registers also get the register form, except
    those in dreg_off (their register kernel spilled); every class gets the
    staged form's Phase 1 at the chunk cap dstage[tag] (default: the
    largest of emit_deriv.STAGE_CAPS; None: tables only)."""
    from .gen import emit, router
    from .gen.cart import canonical_classes

    GEN = gen_dir
    os.makedirs(GEN, exist_ok=True)
    tbl = router.load_table() if table is None else table
    jobs = jobs or min(8, os.cpu_count() or 4)
    classes = list(canonical_classes(lmax))
    args = {}
    for ls in classes:
        tag = "".join(str(x) for x in ls)
        a = (tuple(ls), {tag: tbl[tag]} if tag in tbl else {}, defaults, (overrides or {}).get(tag),
             (reroute or {}).get(tag))
        args[tag] = (json.dumps(a, sort_keys=True, default=str), a)
    todo = [t for t, (key, _) in args.items() if key not in _EMITTED]
    if todo:
        import multiprocessing as mp
        # the slowest classes first so that the pool ends together
        todo.sort(key=lambda t: -sum(int(c) for c in t))
        with cf.ProcessPoolExecutor(max_workers=jobs, mp_context=mp.get_context("fork")) as ex:
            futs = {ex.submit(_route_and_emit, *args[t][1]): t for t in todo}
            for f in cf.as_completed(futs):
                _EMITTED[args[futs[f]][0]] = f.result()
    metas = []
    files = []
    for ls in classes:
        tag = "".join(str(x) for x in ls)
        src, meta = _EMITTED[args[tag][0]]
        path = os.path.join(GEN, f"class_{meta.tag}.hip")
        _write_if_changed(path, src)
        files.append(path)
        for sfx, extra in sorted(getattr(meta, "extra_sources", {}).items()):
            epath = os.path.join(GEN, f"class_{meta.tag}_{sfx}.hip")
            _write_if_changed(epath, extra)
            files.append(epath)
        metas.append(meta)
        if verbose:
            print(f"  class {meta.tag}: {meta.vrr_nodes} VRR nodes, PeakLive {meta.peak_live} ({meta.scheduler}), "
                  f"N_hrr {meta.n_hrr}", flush=True)
    table_path = os.path.join(GEN, "class_table.hip")
    _write_if_changed(table_path, emit.emit_table(metas))
    files.append(table_path)
    # first-derivative tables (wave form) for the classes with l <= DERIV_LMAX
    from .gen import emit_deriv
    dclasses = [ls for ls in classes if max(ls) <= emit_deriv.DERIV_LMAX]
    for ls in dclasses:
        key = ("deriv", tuple(ls))
        if key not in _EMITTED:
            _EMITTED[key] = emit_deriv.emit_deriv_class(*ls)
        path = os.path.join(GEN, f"deriv_{''.join(str(x) for x in ls)}.hip")
        _write_if_changed(path, _EMITTED[key][0])
        files.append(path)
    reg = []
    for ls in dclasses:
        tag = "".join(str(x) for x in ls)
        if tag in dreg_off or not emit_deriv.reg_eligible(ls):
            continue
        key = ("dreg", tuple(ls))
        if key not in _EMITTED:
            _EMITTED[key] = emit_deriv.emit_deriv_reg(*ls)
        path = os.path.join(GEN, f"deriv_reg_{tag}.hip")
        _write_if_changed(path, _EMITTED[key])
        files.append(path)
        reg.append(tag)
    staged, sinfo = [], []
    for ls in dclasses:
        tag = "".join(str(x) for x in ls)
        cap = (dstage or {}).get(tag, emit_deriv.STAGE_CAPS[0])
        if cap is None:
            continue
        key = ("dstage", tuple(ls), cap)
        if key not in _EMITTED:
            _EMITTED[key] = emit_deriv.emit_deriv_staged(*ls, cap=cap)
        srcs, info = _EMITTED[key]
        for p, text in sorted(srcs.items()):
            path = os.path.join(GEN, f"deriv_p1_{tag}p{p}.hip")
            _write_if_changed(path, text)
            files.append(path)
        staged.append(tag)
        sinfo.append(info)
    dtable = os.path.join(GEN, "deriv_table.hip")
    _write_if_changed(dtable, emit_deriv.emit_deriv_table(
        dclasses, reg, {i["tag"]: -(-i["chunks"] // i["parts"]) for i in sinfo}))
    _write_if_changed(os.path.join(GEN, "deriv_forms.json"),
                      json.dumps({"register": reg, "staged": sinfo}, indent=1))
    files.append(dtable)
    _write_if_changed(os.path.join(GEN, "deriv.json"),
                      json.dumps([_EMITTED[("deriv", tuple(ls))][1] for ls in dclasses], indent=1))
    _write_if_changed(os.path.join(GEN, "classes.json"),
                      json.dumps([{k: v for k, v in m.__dict__.items() if k != "extra_sources"} for m in metas],
                                 indent=1, default=list))
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


def _generated_deps(src: str) -> list:
    """A generated source and the library headers it includes, directly or
    through another library header (generated files see only csrc/)."""
    import re
    deps, todo = [src], [src]
    while todo:
        for name in re.findall(r'^#include "([^"]+)"', open(todo.pop()).read(), re.M):
            h = os.path.join(CSRC, name)
            if os.path.exists(h) and h not in deps:
                deps.append(h)
                todo.append(h)
    return deps


def class_source_hash(tag: str, gen_dir: str = GEN) -> str | None:
    """Hash of everything a generated class kernel is compiled from (its
    source and the headers it includes): measurements tied to a kernel, such
    as hardware byte counters, stay valid only while this is unchanged."""
    src = os.path.join(gen_dir, f"class_{tag}.hip")
    if not os.path.exists(src):
        return None
    h = hashlib.sha256()
    for d in _generated_deps(src):
        h.update(open(d, "rb").read())
    return h.hexdigest()[:16]


def _compile(src: str, force: bool):
    if not src.startswith(CSRC + os.sep):
        deps = _generated_deps(src)
    else:
        deps = [src] + [os.path.join(CSRC, f) for f in sorted(os.listdir(CSRC)) if f.endswith(".h")] + \
               [os.path.join(INCLUDE, f) for f in sorted(os.listdir(INCLUDE))]
    h = hashlib.sha256(" ".join(FLAGS).encode())
    for d in deps:
        h.update(open(d, "rb").read())
    obj = os.path.join(OBJ, os.path.basename(src) + "." + h.hexdigest()[:16] + ".o")
    if os.path.exists(obj) and os.path.exists(obj + ".res.json") and not force:
        return obj, 0.0
    t = time.time()
    cmd = [HIPCC] + FLAGS + REMARKS + ["-c", src, "-o", obj + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-4000:]}")
    with open(obj + ".res.json", "w") as fh:
        json.dump(parse_resource_remarks(r.stderr), fh)
    os.replace(obj + ".tmp", obj)
    return obj, time.time() - t


_REMARK_KEYS = {"TotalSGPRs": "sgpr", "VGPRs": "vgpr", "AGPRs": "agpr", "ScratchSize [bytes/lane]": "scratch",
                "Occupancy [waves/SIMD]": "occupancy", "SGPRs Spill": "sgpr_spill", "VGPRs Spill": "vgpr_spill",
                "LDS Size [bytes/block]": "lds", "Dynamic Stack": "dynamic_stack"}


def _demangle_kernel(name: str) -> str:
    """The kernel's own identifier out of an Itanium-mangled name (enough for
    the library's kernels: plain or namespaced functions, templates reported
    with their arguments appended)."""
    if not name.startswith("_Z"):
        return name
    import re
    parts = []
    s = name[2:]
    if s.startswith("N"):
        s = s[1:]
        while s and s[0].isdigit():
            m = re.match(r"(\d+)", s)
            n = int(m.group(1))
            s = s[m.end():]
            parts.append(s[:n])
            s = s[n:]
        base = parts[-1] if parts else name
    else:
        m = re.match(r"(\d+)", s)
        base = s[m.end():m.end() + int(m.group(1))] if m else name
        s = s[m.end() + int(m.group(1)):] if m else ""
    tmpl = ""
    m = re.search(r"ILi(\d+)EE", name)
    if m:
        tmpl = f"<{m.group(1)}>"
    elif re.search(r"ILb1EE", name):
        tmpl = "<true>"
    elif re.search(r"ILb0EE", name):
        tmpl = "<false>"
    return base + tmpl


def parse_resource_remarks(stderr: str) -> dict:
    """{kernel: {vgpr, agpr, sgpr, scratch, occupancy, lds, vgpr_spill, ...}}
    from the compiler's kernel-resource-usage remarks."""
    out, cur = {}, None
    for line in stderr.splitlines():
        if "remark:" not in line or "kernel-resource-usage" not in line:
            continue
        body = line.split("remark:", 1)[1].rsplit("[-Rpass-analysis", 1)[0].strip()
        if body.startswith("Function Name:"):
            mangled = body.split(":", 1)[1].strip()
            cur = {"mangled": mangled}
            out[_demangle_kernel(mangled) + ("" if _demangle_kernel(mangled) not in out else "#" + mangled)] = cur
            continue
        if cur is None or ":" not in body:
            continue
        k, v = body.rsplit(":", 1)
        k = k.strip()
        if k in _REMARK_KEYS:
            v = v.strip()
            cur[_REMARK_KEYS[k]] = (v == "True") if v in ("True", "False") else int(v)
    return out


def check_resources(res: dict) -> list[str]:
    """Kernels that use private scratch (register spills or stack): the
    library's kernels must compile with none."""
    return sorted(k for k, r in res.items() if r.get("scratch", 0) > 0 or r.get("dynamic_stack", False))


def resources_path(lib: str) -> str:
    """The compiler's per-kernel resource report written beside a library."""
    return (lib[:-3] if lib.endswith(".so") else lib) + ".resources.json"


def class_scratch(res: dict, tag: str) -> int:
    """Largest private scratch (bytes per lane) of the kernels of class `tag`
    (a spill into accumulation registers uses none and is not counted)."""
    import re
    return max((r.get("scratch", 0) for k, r in res.items()
                if re.search(r"_" + tag + r"(?:p\d+)?$", k.split("#")[0])), default=0)


def _spilled_classes(res: dict) -> dict:
    """class tag -> names of its kernels that use private scratch."""
    import re
    out: dict = {}
    for k in check_resources(res):
        name = k.split("#")[0]
        if name.startswith(("dreg_", "dp1_")):             # derivative forms: _spilled_dreg
            continue
        m = re.search(r"_(\d{4})(?:p\d+)?$", name)        # class kernels, Phase-1 parts included
        if m:
            out.setdefault(m.group(1), []).append(name)
    return out


def _spilled_dreg(res: dict, prefix: str = "dreg") -> set:
    """Tags of the derivative register kernels (prefix dreg) or staged
    Phase-1 parts (prefix dp1) that use private scratch."""
    import re
    return {m.group(1) for k in check_resources(res)
            for m in [re.match(prefix + r"_(\d{4})(?:p\d+)?$", k.split("#")[0])] if m}


def build(lmax: int = DEFAULT_LMAX, jobs: int | None = None, force: bool = False, verbose: bool = True,
          overrides=None, out: str | None = None, gen_dir: str = GEN, defaults=None, table=None,
          allow_scratch: bool = False) -> str:
    """Generate, compile and link; out (default: the package's libhgp.so)
    and gen_dir let a tuning run build variant libraries side by side.
    A kernel compiled with private scratch (a register spill) fails the
    build unless allow_scratch (tuning variants: the tuner then leaves that
    class's variant out)."""
    from .gen import router
    t0 = time.time()
    os.makedirs(OBJ, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 4)
    # start from the routes earlier builds settled on (only for the library's
    # own table: variant builds with an explicit table start from the model)
    main_table = table is None and defaults is None and overrides is None
    reroute: dict = dict(router.load_reroutes()) if main_table else {}
    compiled: set = set()
    dreg_off: set = set()
    dstage: dict = {}
    for attempt in range(8):
        gen_files, metas = generate(lmax, verbose=False, overrides=overrides, gen_dir=gen_dir, defaults=defaults,
                                    table=table, reroute=reroute, dreg_off=frozenset(dreg_off), dstage=dstage)
        srcs = [os.path.join(CSRC, f) for f in sorted(os.listdir(CSRC)) if f.endswith(".hip")] + gen_files
        objs = []
        with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
            # force recompiles each source once per build, not once per rerouting pass
            futs = {ex.submit(_compile, s, force and s not in compiled): s for s in srcs}
            for f in cf.as_completed(futs):
                obj, dt = f.result()
                objs.append(obj)
                compiled.add(futs[f])
                if verbose and dt > 0:
                    print(f"  compiled {os.path.basename(futs[f])} in {dt:.1f}s", flush=True)
        objs.sort()
        res = {}
        for o in objs:
            with open(o + ".res.json") as fh:
                res.update(json.load(fh))
        # the compiler's resource report has the last word on the register
        # model: a class whose kernels spill moves down the router's ladder
        spilled = _spilled_classes(res)
        dspill = _spilled_dreg(res)
        sspill = _spilled_dreg(res, "dp1")
        if (dspill or sspill) and not allow_scratch:
            # a derivative class whose register kernel spills takes the staged
            # form; a staged one steps down the chunk caps, then keeps only its tables
            from .gen import emit_deriv
            if verbose and dspill:
                print(f"  derivative register forms {' '.join(sorted(dspill))} use private scratch; staged", flush=True)
            dreg_off |= dspill
            caps = list(emit_deriv.STAGE_CAPS)
            for tag in sorted(sspill):
                cur = dstage.get(tag, caps[0])
                dstage[tag] = caps[caps.index(cur) + 1] if cur in caps[:-1] else None
                if verbose:
                    print(f"  derivative staged form {tag} at (cap, waves) {cur} uses private scratch; "
                          f"{dstage[tag] if dstage[tag] else 'tables only'}", flush=True)
        if (not spilled and not dspill and not sspill) or allow_scratch:
            break
        by_tag = {m.tag: m for m in metas}
        for tag, kernels in sorted(spilled.items()):
            nxt = router.fallback(by_tag[tag].route, kernels)
            if nxt is None:
                continue
            if verbose:
                print(f"  class {tag}: {', '.join(sorted(kernels))} use private scratch; rerouting {nxt}", flush=True)
            reroute[tag] = nxt
    bad = check_resources(res)
    if not bad and main_table and out is None and router.save_reroutes(reroute) and verbose:
        print(f"  recorded {len(reroute)} rerouted classes in {router.TABLE}", flush=True)
    if bad and not allow_scratch:
        raise RuntimeError("kernels compiled with private scratch (register spill or stack), which the library "
                           "does not allow: " + ", ".join(f"{k} ({res[k].get('scratch')} B/lane)" for k in bad))
    lib = out or LIB
    tmp = lib + ".tmp"
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-4000:]}")
    os.replace(tmp, lib)
    _write_if_changed(resources_path(lib), json.dumps(res, indent=0, sort_keys=True))
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
