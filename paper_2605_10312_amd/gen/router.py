"""Tier routing per quartet class (Sec. III-C, Eq. rtotal, redone for gfx950).

The paper routes by the register demand R_total ~ 2 (PeakLive_VRR + N_acc)
against a 255-register limit.  On gfx950 a lane can hold at most 512 32-bit
registers (256 ArchVGPR + 256 AccVGPR, at one wave per SIMD), i.e. 256
doubles, and the accumulator bank is the contracted [e0|f0] set, so the
model here is

    demand = N_hrr + PeakLive + 40      (40: pair/Boys/VRR coefficients)

    register tier (one kernel, everything in VGPR/AGPR)   if demand <= 240
    staged tier (Phase-1 chunks + HBM-staged Phase 2)     if the VRR graph has
                                                          <= 3000 nodes and
                                                          N_hrr <= 1024
    HBM-scratch tier (slot-packed op tables)              otherwise

The 240-double line was set from the compiler's resource reports: every
class at or under it compiles without scratch, every class above it spilled.
The staged tier recomputes, per chunk of accumulators, the part of the VRR
graph the chunk needs and emits it as straight-line code; past (dd|dd)'s
size (2330 nodes, 961 accumulators) the recomputation and the code grow
faster than they pay, so larger classes go to the HBM-scratch tier, whose
code does not grow with the class.  A tuning table measured on the GPU
(tuning/gfx950.json) overrides the model per class.
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


def model_tier(ls):
    g = vrrmod.VRRGraph(*ls)
    if len(g.nodes) > STAGED_MAX_NODES or g.n_hrr() > STAGED_MAX_HRR:
        return 0 if g.n_hrr() + 40 <= REGISTER_DOUBLES and model_demand(ls) <= REGISTER_DOUBLES else 2
    return 0 if model_demand(ls) <= REGISTER_DOUBLES else 1


def load_table(path=TABLE):
    if path and os.path.exists(path):
        with open(path) as fh:
            return json.load(fh).get("classes", {})
    return {}


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
    cap = model_cap(ls) if tier == 1 else DEFAULT_CAP
    if tier == 1 and "cap" in t:
        cap = t["cap"]
    r = {"tier": tier, "cap": cap, "waves": 0, "source": "model"}
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
        if all(k.startswith("p1_") for k in spilled):
            cap = route.get("cap", DEFAULT_CAP)
            smaller = [c for c in CAPS if c < cap]
            if smaller:
                return {"tier": 1, "cap": smaller[0]}
        return {"tier": 2}
    return None
