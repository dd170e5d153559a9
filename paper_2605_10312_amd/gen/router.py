"""Tier routing per quartet class (Sec. III-C, Eq. rtotal, redone for gfx950).

The paper routes by the register demand R_total ~ 2 (PeakLive_VRR + N_acc)
against a 255-register limit.  On gfx950 a lane can hold at most 512 32-bit
registers (256 ArchVGPR + 256 AccVGPR, at one wave per SIMD), i.e. 256
doubles, and the accumulator bank is the contracted [e0|f0] set, so the
model here is

    demand = N_hrr + PeakLive + 40      (40: pair/Boys/VRR coefficients)

    register tier (one kernel, everything in VGPR/AGPR)   if demand <= 240
    staged tier, e-chunked form (Phase-1 chunks of        if the VRR graph has
      accumulators + HBM-staged Phase 2)                  <= 3000 nodes and
                                                          N_hrr <= 1024
    staged tier, row form (whole bra rows per chunk with  otherwise, while a
      the ket stage fused, gen/emit_row.py)               ket row has <= 80
                                                          components
    op tables (slot-packed, LDS or HBM scratch)           otherwise

The 240-double line was set from the compiler's resource reports, which have
the last word: the build compiles every class, reads the report, and moves a
class whose kernels use private scratch down a ladder (register -> staged;
staged chunk cap or row budget down a step; last, the op tables), see
fallback().  A tuning table measured on the GPU (tuning/gfx950.json)
overrides the model per class.
"""
from __future__ import annotations

import json
import os

from . import vrr as vrrmod

REGISTER_DOUBLES = 240
DEFAULT_CAP = 96
TABLE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "tuning", "gfx950.json")


STAGED_MAX_NODES = 3000
STAGED_MAX_HRR = 1024


def model_demand(ls):
    g = vrrmod.VRRGraph(*ls)
    _, pl, _ = vrrmod.best_order(g)
    return g.n_hrr() + pl + 40


# The row form keeps whole rows of ket components f (lc <= |f| <= lc + ld) in
# registers where it can.  Past this many per row (a (gf| or (gg| ket: 100,
# 145) almost every row is cut into small tiles, each recomputing most of the
# recurrence (x11.8 for (gg|gg)), and the class takes the op tables instead.
ROW_MAX_KET = 80
# A (gg| bra (145 components) needs the second kernel's bra stage split into
# groups that each redo part of the HRR; the generated code then takes tens
# of minutes to compile, so those classes stay on the op tables as well.
ROW_MAX_BRA = 100
# Row-form chunks: accumulators + the chunk's PeakLive + 40 within this many
# doubles.  The register-tier line (240) left some (ff|ff) chunks spilling: the
# compiler's schedule keeps more values live than the graph order needs.
ROW_BUDGET = 220


def model_tier(ls):
    """0 register, 1 staged (e-chunked, or the row form for classes past the
    e-chunked form's size), 2 op tables."""
    g = vrrmod.VRRGraph(*ls)
    if len(g.nodes) > STAGED_MAX_NODES or g.n_hrr() > STAGED_MAX_HRR:
        if g.n_hrr() + 40 <= REGISTER_DOUBLES and model_demand(ls) <= REGISTER_DOUBLES:
            return 0
        n_bra = sum((l + 1) * (l + 2) // 2 for l in range(ls[0], ls[0] + ls[1] + 1))
        n_ket = sum((l + 1) * (l + 2) // 2 for l in range(ls[2], ls[2] + ls[3] + 1))
        return 1 if n_ket <= ROW_MAX_KET and n_bra <= ROW_MAX_BRA else 2
    return 0 if model_demand(ls) <= REGISTER_DOUBLES else 1


def model_form(ls):
    """Staged classes past the e-chunked form's size take the row form."""
    g = vrrmod.VRRGraph(*ls)
    return "row" if len(g.nodes) > STAGED_MAX_NODES or g.n_hrr() > STAGED_MAX_HRR else "chunk"


def load_table(path=TABLE):
    if path and os.path.exists(path):
        with open(path) as fh:
            return json.load(fh).get("classes", {})
    return {}


def load_reroutes(path=TABLE):
    """Routes the build's compile-feedback pass settled on (class tag ->
    options), recorded beside the measured table so that a fresh build starts
    from them instead of compiling the spilling forms again."""
    if path and os.path.exists(path):
        with open(path) as fh:
            return json.load(fh).get("rerouted", {})
    return {}


def save_reroutes(reroute, path=TABLE):
    data = json.load(open(path)) if os.path.exists(path) else {"device": "gfx950", "classes": {}}
    if data.get("rerouted", {}) == reroute:
        return False
    data["rerouted"] = {k: reroute[k] for k in sorted(reroute)}
    with open(path + ".tmp", "w") as fh:
        json.dump(data, fh, indent=1)
    os.replace(path + ".tmp", path)
    return True


CAPS = (128, 96, 64, 48, 32, 24, 16)


def chunk_demand(g, order, chunk):
    """Accumulators + PeakLive of one chunk's subgraph in the given order, + 40."""
    from .emit_staged import subgraph
    sub = subgraph(g, chunk)
    pos = [v for v in order if v in sub]
    idx = {v: i for i, v in enumerate(pos)}
    last = {}
    for v in pos:
        for c in g.children[v]:
            if c in idx:
                last[v] = max(last.get(v, -1), idx[c])
    live = peak = 0
    dies = {}
    for i, v in enumerate(pos):
        if last.get(v, -1) > i:
            live += 1
            dies.setdefault(last[v], []).append(v)
        peak = max(peak, live)
        live -= len(dies.pop(i, ()))
    return len(chunk) + peak + 40


def model_cap(ls):
    """Largest chunk cap whose every chunk fits the register line."""
    from .emit_staged import chunk_targets
    g = vrrmod.VRRGraph(*ls)
    _, _, order = vrrmod.best_order(g)
    for cap in CAPS:
        if all(chunk_demand(g, order, c) <= REGISTER_DOUBLES for c in chunk_targets(g, cap)):
            return cap
    return CAPS[-1]


def route(ls, table=None):
    """-> dict(tier=0|1|2, cap=int, waves=int, source='model'|'table')"""
    tag = "".join(str(x) for x in ls)
    table = load_table() if table is None else table
    t = dict(table.get(tag, {}))
    tier = t.get("tier", model_tier(ls))
    form = t.get("form", model_form(ls)) if tier == 1 else None
    cap = model_cap(ls) if tier == 1 and form == "chunk" else DEFAULT_CAP
    if tier == 1 and "cap" in t:
        cap = t["cap"]
    r = {"tier": tier, "cap": cap, "waves": 0, "source": "model"}
    if tier == 1:
        r["form"] = form
        if form == "row":
            r["budget"] = ROW_BUDGET
    if t:                      # measured entries win; what they leave out comes from the model
        r.update({k: v for k, v in t.items() if k not in ("variant", "ms")})
        r["source"] = "table"
    return r


def fallback(route, spilled):
    """The next choice for a class whose kernels `spilled` (names) compiled
    with private scratch under `route` (the options it was generated with), or
    None when there is none.  Register tier -> staged tier; staged tier whose
    Phase-1 chunks spill -> the next smaller chunk cap; staged tier whose
    Phase-2 kernels spill (their per-column working set does not fit) ->
    the op-table tiers, which keep every value in LDS or HBM."""
    tier = route.get("tier", 0)
    if tier == 0:
        return {"tier": 1}
    if tier == 1:
        keep = {k: route[k] for k in ("form", "budget", "cap", "jk_digest") if k in route}
        # a J/K kernel whose one-pass digestion does not fit: the six-pass form first
        if any(k.startswith("jk_") for k in spilled) and route.get("jk_digest", "fused") == "fused":
            return {"tier": 1, **keep, "jk_digest": "slots"}
    if tier == 1 and route.get("form") == "row":
        budget = route.get("budget", ROW_BUDGET)
        if all(k.startswith("p1_") for k in spilled) and budget > 160:
            return {"tier": 1, **keep, "budget": budget - 20}
        return {"tier": 2}
    if tier == 1:
        if all(k.startswith("p1_") for k in spilled):
            cap = route.get("cap", DEFAULT_CAP)
            smaller = [c for c in CAPS if c < cap]
            if smaller:
                return {"tier": 1, **keep, "cap": smaller[0]}
        return {"tier": 2}
    return None
