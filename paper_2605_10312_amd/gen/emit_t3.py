"""Generator for the HBM-scratch tier: a class as an op table run by one
generic kernel (csrc/hgp_t3.hip).

For classes whose VRR frontier alone exceeds the register file (PeakLive in
the hundreds to thousands of doubles for (ff|ff) and (gg|gg)), straight-line
code either spills or, chunked, recomputes most of the graph.  Here every
value lives in a slot of a lane-interleaved HBM buffer, slot k of lane i at
sb[k * S + i], so each wave reads and writes whole 512-byte rows.  The
generator does what a register allocator would: it walks the VRR in the
scheduler's order (Sec. III-A) and the Phase-2 stages in their stepwise order
(Sec. III-B) and reuses a slot as soon as its value is dead (the two-pass
lifetime packing of the paper's Tier 2).

Slots 0..L hold base * F_m(T), written by the kernel after the Boys step.
The contracted accumulators [e0|f0] follow (N_hrr slots); then come the
temporaries.  An op is eight uint16 words:

  VRR_BRA / VRR_KET  w0 = op | axis << 4 | k_same << 6 | k_cross << 11,
                     dst, p1, p2, p3, p4, p5 (0xFFFF when absent)
      dst = X[axis] p1 + Y[axis] p2 + k_same o2 (p3 - r p4) + k_cross o2ze p5
      with (X, Y, o2, r) = (P-A, W-P, 1/(2 zeta), rho/zeta) on the bra side
      and (Q-C, W-Q, 1/(2 eta), rho/eta) on the ket side (Eq. vrr);
  ACC                dst += p1 (a target into its accumulator);
  ACC_W              dst += w2 * p1, w2 a slot the kernel fills per primitive
                     quartet (the exponent weights of derivative integrals);
  HRR_BRA / HRR_KET  dst = p1 + (A-B or C-D)[axis] p2 (Eq. hrr);
  LIN / LIN_ACC      dst (+)= c[w5] p1 + c[w6] p2 + c[w7] p3 (a row of the
                     T^(l) transforms, three terms per op, coefficients from
                     the class's table).
"""
from __future__ import annotations

import dataclasses

from . import phase2 as p2mod
from . import vrr as vrrmod
from .cart import nsph
from .emit import ClassMeta, tag_of

OP_VRR_BRA, OP_VRR_KET, OP_ACC, OP_HRR_BRA, OP_HRR_KET, OP_LIN, OP_LIN_ACC, OP_ACC_W = 1, 2, 3, 4, 5, 6, 7, 8
NONE = 0xFFFF
XYZ_AXIS = {"x": 0, "y": 1, "z": 2}


BUNDLE = 8      # ops per group; a group's operand loads are all in flight at once


@dataclasses.dataclass
class T3Tables:
    ops: list            # flat uint16 words, 8 per op, groups of BUNDLE ops
    n_vrr: int           # op slots of the per-primitive part (VRR + ACC), a multiple of BUNDLE
    n_p2: int            # op slots of Phase 2, a multiple of BUNDLE
    coefs: list          # doubles
    outslots: list       # slot of integral (mu, nu, lam, sig), row-major
    nslots: int
    n_hrr: int
    acc0: int            # first accumulator slot
    L: int
    peak_live: int
    scheduler: str
    vrr_flops: int
    p2_flops: int
    n_real_ops: int = 0  # ops before padding


class _Slots:
    """Free-list slot allocator (lowest free slot first)."""

    def __init__(self, first):
        self.next = first
        self.free = []

    def get(self):
        if self.free:
            return self.free.pop()
        s = self.next
        self.next += 1
        return s

    def put(self, s):
        self.free.append(s)


def _group_class(kind):
    return {"vrr": 0, "acc": 1, "hrr": 2, "lin": 3, "linacc": 3}[kind]


def _bundle(ops, K):
    """List-schedule abstract ops into groups of at most K ops of one class
    (VRR, ACC, HRR, transform) such that no op reads a value produced in its
    own group.  Ops are dicts with 'out' (new value or None), 'writes' (value
    written, if it differs from 'out'), 'ins' (values read), 'after' (an op
    that must run in an earlier group) and 'kind'; priority is the original
    position, which keeps the liveness-minimising order as far as
    independence allows."""
    import heapq
    producer = {}
    for k, o in enumerate(ops):
        w = o.get("writes", o["out"])
        if w is not None:
            producer[w] = k                      # the last writer (a chained transform's last part)
    deps = []
    users = [[] for _ in ops]
    for k, o in enumerate(ops):
        d = {producer[v] for v in o["ins"] if v in producer and producer[v] != k}
        if o.get("after") is not None:
            d.add(o["after"])
        deps.append(len(d))
        for j in d:
            users[j].append(k)
    ready = [k for k in range(len(ops)) if deps[k] == 0]
    heapq.heapify(ready)
    groups = []
    while ready:
        first = heapq.heappop(ready)
        cls = _group_class(ops[first]["kind"])
        grp, skipped = [first], []
        while ready and len(grp) < K:
            k = heapq.heappop(ready)
            (grp if _group_class(ops[k]["kind"]) == cls else skipped).append(k)
        for k in skipped:
            heapq.heappush(ready, k)
        groups.append(grp)
        for k in grp:
            for u in users[k]:
                deps[u] -= 1
                if deps[u] == 0:
                    heapq.heappush(ready, u)
    assert sum(len(g) for g in groups) == len(ops), "dependency cycle in the op list"
    return groups


def build_tables(la, lb, lc, ld, rule="ket_zyx", schedulers=None, bundle=BUNDLE) -> T3Tables:
    ls = (la, lb, lc, ld)
    L = sum(ls)
    g = vrrmod.VRRGraph(*ls, rule=rule)
    sched, pl, order = vrrmod.best_order(g) if schedulers is None else vrrmod.best_order(g, schedulers)
    n_hrr = len(g.targets)
    accs = {tid: [(k, None)] for k, tid in enumerate(g.target_ids)}
    hname = {t: f"h{k}" for k, t in enumerate(g.targets)}
    p2 = p2mod.Phase2(la, lb, lc, ld, hname=lambda e, f: hname[(e, f)])
    na, nb, nc, nd = (nsph(x) for x in ls)
    out_names = [p2.out[(mu, nu, lam, sig)] for mu in range(na) for nu in range(nb)
                 for lam in range(nc) for sig in range(nd)]
    return assemble_tables(g, order, sched, pl, L, L + 1, n_hrr, accs, p2.ops, out_names, g.flops(), p2.flops,
                           bundle, tag_of(ls))


def assemble_tables(g, order, sched, pl, L, acc0, n_acc, accs, p2ops, out_names, vrr_flops, p2_flops, bundle,
                    tag) -> T3Tables:
    """Slot-packed op tables from a VRR graph run in `order`, accumulations
    accs[node] = [(accumulator k, weight slot or None), ...] (a weighted
    accumulation adds slot * value), and a Phase-2 op list (SSA, see
    gen/phase2.py) over the accumulators named h<k>, whose results
    out_names are the outputs, in order.  Slots 0..L hold base * F_m(T);
    slots L + 1 .. acc0 - 1 are left to the kernel (per-primitive weights)."""
    # ---- abstract ops of the per-primitive part: VRR nodes in schedule
    # order, each target followed by its accumulations
    aops = []
    for v in order:
        nd = g.nodes[v]
        if nd.kind != "base":
            aops.append({"kind": "vrr", "out": ("n", v), "ins": [("n", x) for x in nd.parents if x is not None],
                         "node": v})
        for k, ws in accs.get(v, ()):
            aops.append({"kind": "acc", "out": None, "ins": [("n", v)], "acc": acc0 + k, "w": ws})
    # ---- Phase 2: the given ops over the accumulators
    pops = []
    for o in p2ops:
        if o[1] == "hrr":
            pops.append({"kind": "hrr", "out": ("p", o[0]), "ins": [("p", o[2]), ("p", o[3])], "op": o})
        else:
            terms = list(o[2])
            prev = None
            for j in range(0, len(terms), 3):
                chunk = terms[j:j + 3]
                d = {"kind": "lin" if j == 0 else "linacc", "out": ("p", o[0]) if j == 0 else None,
                     "writes": ("p", o[0]), "ins": [("p", x) for _, x in chunk], "terms": chunk,
                     "dst": ("p", o[0]), "after": prev}
                pops.append(d)
                prev = len(pops) - 1
    vgroups = _bundle(aops, bundle)
    pgroups = _bundle(pops, bundle)

    words = []
    n_real = 0

    def emit(w):
        words.extend(w)

    def pad(group_len):
        for _ in range(bundle - group_len):
            emit((0, 0, NONE, NONE, NONE, NONE, NONE, NONE))

    # ---- slots, VRR part: base values in 0..L, accumulators fixed, node values
    # allocated at their group and released after the group of their last reader
    slot = {("n", v): g.nodes[v].key[2] for v in range(len(g.nodes)) if g.nodes[v].kind == "base"}
    last = {}
    for gi, grp in enumerate(vgroups):
        for k in grp:
            for x in aops[k]["ins"]:
                last[x] = gi
    alloc = _Slots(acc0 + n_acc)
    for gi, grp in enumerate(vgroups):
        for k in grp:
            o = aops[k]
            if o["kind"] == "vrr":
                nd = g.nodes[o["node"]]
                s = alloc.get()
                slot[o["out"]] = s
                p = [slot[("n", x)] if x is not None else NONE for x in nd.parents]
                code = OP_VRR_BRA if nd.kind == "bra" else OP_VRR_KET
                emit((code | (nd.axis << 4) | (nd.k_same << 6) | (nd.k_cross << 11), s, *p, NONE))
            elif o.get("w") is None:
                emit((OP_ACC, o["acc"], slot[o["ins"][0]], NONE, NONE, NONE, NONE, NONE))
            else:
                emit((OP_ACC_W, o["acc"], slot[o["ins"][0]], o["w"], NONE, NONE, NONE, NONE))
            n_real += 1
        pad(len(grp))
        for k in grp:
            o = aops[k]
            if o["kind"] == "vrr" and last.get(o["out"], -1) <= gi and g.nodes[o["node"]].kind != "base":
                alloc.put(slot[o["out"]])        # never read again (a target, accumulated in this group)
        for x in sorted({x for k in grp for x in aops[k]["ins"]}):      # sorted: the same tables every run
            if last.get(x) == gi and x in slot and slot[x] > L:
                alloc.put(slot[x])
    n_vrr = len(words) // 8
    vrr_top = alloc.next

    # ---- slots, Phase 2: inputs are the accumulators; VRR temporaries are free
    name_slot = {("p", f"h{k}"): acc0 + k for k in range(n_acc)}
    outputs = {("p", v) for v in out_names}
    last = {}
    for gi, grp in enumerate(pgroups):
        for k in grp:
            for x in pops[k]["ins"]:
                last[x] = gi
    alloc2 = _Slots(vrr_top)
    alloc2.free = sorted(range(acc0 + n_acc, vrr_top), reverse=True)
    coefs, cidx = [], {}

    def coef(c):
        c = float(c)
        if c not in cidx:
            cidx[c] = len(coefs)
            coefs.append(c)
        return cidx[c]

    for gi, grp in enumerate(pgroups):
        for k in grp:
            o = pops[k]
            if o["kind"] == "hrr":
                _, _, hi, lo, cname = o["op"]
                s = alloc2.get()
                name_slot[o["out"]] = s
                axis = XYZ_AXIS[cname[-1]]
                code = OP_HRR_BRA if cname.startswith("AB") else OP_HRR_KET
                emit((code | (axis << 4), s, name_slot[("p", hi)], name_slot[("p", lo)], NONE, NONE, NONE, NONE))
            else:
                if o["kind"] == "lin":
                    name_slot[o["out"]] = alloc2.get()
                s = name_slot[o["dst"]]
                srcs = [name_slot[("p", x)] for _, x in o["terms"]] + [NONE] * (3 - len(o["terms"]))
                cs = [coef(c) for c, _ in o["terms"]] + [0] * (3 - len(o["terms"]))
                emit((OP_LIN if o["kind"] == "lin" else OP_LIN_ACC, s, *srcs, *cs))
            n_real += 1
        pad(len(grp))
        for x in sorted({x for k in grp for x in pops[k]["ins"]}):
            if last.get(x) == gi and x not in outputs:
                alloc2.put(name_slot[x])
    n_p2 = len(words) // 8 - n_vrr
    nslots = max(alloc2.next, vrr_top)
    if nslots > 0xFFFE or len(coefs) > 0xFFFF:
        raise ValueError(f"class {tag}: {nslots} slots do not fit 16-bit slot indices")
    outslots = [name_slot[("p", v)] for v in out_names]
    return T3Tables(words, n_vrr, n_p2, coefs, outslots, nslots, n_acc, acc0, L, pl, sched, vrr_flops, p2_flops,
                    n_real)


WAVE = 128              # ops per group of the wave-cooperative variant: two per lane of a wavefront
WAVE_LDS_MAX = 163840   # bytes of LDS one workgroup of that variant may take (gfx950: 160 KB per CU)
GSLOT_MAX_BATCH = 1024  # quartets per launch when the slots live in the scratch buffer (~190 MB for (gg|gg));
                        # batches of T3G_LANE_MIN (csrc/hgp_types.h) or more run the lane-per-quartet tables


@dataclasses.dataclass
class WaveTables:
    """The op tables regrouped WAVE ops a group for the wave-cooperative
    variant (one wavefront per quartet, its slots in LDS, lane j running ops
    j and j + 64 of every group).  Operand fields that the HBM form marks absent name
    the zero slot Z = nslots; padding ops write the sink slot nslots + 1 and
    read Z (transform padding reads coefficient 0)."""
    t: T3Tables
    ops: list
    zero: int
    sink: int
    lds_doubles: int     # slots, Z, sink, coefficients, six D blocks
    lds_bytes: int       # lds_doubles * 8 plus the uint16 output-slot map
    maxblk: int


def wave_layout(ls, t, gslots=False):
    """(maxblk, LDS doubles, LDS bytes); gslots: the slots are not in LDS."""
    na, nb, nc, nd = (nsph(x) for x in ls)
    maxblk = max(na * nb, nc * nd, na * nc, nb * nc, na * nd, nb * nd)
    nint = len(t.outslots)            # the integrals (12 blocks of them for derivative tables)
    doubles = (0 if gslots else t.nslots + 2) + max(len(t.coefs), 1) + 6 * maxblk
    # then the uint16 output-slot map (padded to 16 bytes) and the 16-double VRR constants record
    return maxblk, doubles, doubles * 8 + ((2 * nint + 15) // 16) * 16 + 16 * 8


def build_wave_tables(la, lb, lc, ld, rule="ket_zyx", schedulers=None) -> WaveTables:
    return build_wave_tables_from(build_tables(la, lb, lc, ld, rule, schedulers, bundle=WAVE), (la, lb, lc, ld))


def build_wave_tables_from(t, ls) -> WaveTables:
    """The wave form of tables t built with bundle = WAVE (class ls: the D
    and output blocks of the layout)."""
    assert (t.n_vrr + t.n_p2) % WAVE == 0, "tables grouped for the lane form"
    Z, SINK = t.nslots, t.nslots + 1
    ops = []
    words = t.ops
    for g0 in range(0, len(words) // 8, WAVE):
        first = words[8 * g0] & 15
        lin = first in (OP_LIN, OP_LIN_ACC)
        for k in range(g0, g0 + WAVE):
            w = list(words[8 * k:8 * k + 8])
            if w[0] == 0:
                w = [0, SINK, Z, Z, Z] + ([0, 0, 0] if lin else [Z, Z, Z])
            elif lin:
                w = w[:2] + [Z if x == NONE else x for x in w[2:5]] + w[5:]
            else:
                w = w[:2] + [Z if x == NONE else x for x in w[2:]]
            ops.extend(w)
    maxblk, doubles, nbytes = wave_layout(ls, t)
    return WaveTables(t, ops, Z, SINK, doubles, nbytes, maxblk)


def wave_fits(la, lb, lc, ld, rule="ket_zyx") -> bool:
    t = build_tables(la, lb, lc, ld, rule, bundle=WAVE)
    return wave_layout((la, lb, lc, ld), t)[2] <= WAVE_LDS_MAX


def _u16_lines(vals, per=24):
    out = []
    for k in range(0, len(vals), per):
        out.append("    " + ", ".join(str(v) for v in vals[k:k + per]) + ",")
    return out


def emit_class_t3(la, lb, lc, ld, rule="ket_zyx", schedulers=None, block=64, wave="auto"):
    """Host-side tables plus the launchers that hand them to the generic
    kernels; no device code is generated for the class.  wave: "lds" for the
    wave-cooperative LDS variant (tier 3), "global" for the wave-cooperative
    variant with its slots in the scratch buffer (tier 2), "lane" for the
    lane-per-quartet HBM-scratch variant (tier 2), "auto" for "lds" wherever
    the slots fit WAVE_LDS_MAX and "global" elsewhere."""
    ls = (la, lb, lc, ld)
    tag = tag_of(ls)
    if wave not in ("auto", "lds", "global", "lane"):
        raise ValueError(f"unknown variant {wave!r}")
    wt = None
    gslots = False
    if wave != "lane":
        wt = build_wave_tables(la, lb, lc, ld, rule, schedulers)
        if wave == "global" or (wave == "auto" and wt.lds_bytes > WAVE_LDS_MAX):
            gslots = True
            wt.maxblk, wt.lds_doubles, wt.lds_bytes = wave_layout(ls, wt.t, gslots=True)
    t = wt.t if wt else build_tables(la, lb, lc, ld, rule, schedulers)
    words = wt.ops if wt else t.ops
    tier = 3 if wt and not gslots else 2
    na, nb, nc, nd = (nsph(x) for x in ls)
    if wt and not gslots:
        what = f"the wave-cooperative LDS tier ({wt.lds_bytes} bytes of LDS per quartet)"
    elif wt:
        what = (f"the HBM-scratch tier, wave-cooperative with the slots in the scratch buffer "
                f"({wt.lds_bytes} bytes of LDS per quartet)")
    else:
        what = "the HBM-scratch tier, one lane per quartet"
    out = [f"// Generated: class ({la}{lb}|{lc}{ld}) for {what}, axis rule {rule},",
           f"// VRR order '{t.scheduler}' (PeakLive {t.peak_live}), {t.n_vrr} per-primitive ops,",
           f"// {t.n_p2} Phase-2 ops, {t.nslots} slots per {'quartet' if wt else 'lane'}, "
           f"{len(t.outslots)} spherical integrals.",
           '#include "hgp_t3.h"', "", "#if !defined(__HIP_DEVICE_COMPILE__)", "namespace hgp {", "namespace {", ""]
    def table(name, tt, ws, extra):
        lines = [f"const uint16_t ops_{name}[] = {{"]
        lines.extend(_u16_lines(ws))
        lines.append("};")
        lines.append(f"const uint16_t outslots_{name}[] = {{")
        lines.extend(_u16_lines(tt.outslots))
        lines.append("};")
        lines.append(f"const double coefs_{name}[] = {{")
        for k in range(0, max(len(tt.coefs), 1), 4):
            lines.append("    " + ", ".join(repr(c) for c in (tt.coefs[k:k + 4] or [0.0])) + ",")
        lines.append("};")
        lines.append(f"T3Class t3_{name} = {{{la}, {lb}, {lc}, {ld}, {tt.L}, {na}, {nb}, {nc}, {nd}, {tt.nslots}, "
                     f"{tt.n_hrr}, {tt.acc0}, {tt.n_vrr}, {tt.n_p2}, ops_{name}, {max(len(tt.coefs), 1)}, "
                     f"coefs_{name}, outslots_{name}, {block}{extra}}};")
        lines.append("")
        return lines

    lane_t = None
    if gslots:
        # large batches run the lane-per-quartet kernel on its own tables
        lane_t = build_tables(la, lb, lc, ld, rule, schedulers)
        out.extend(table(f"{tag}_lane", lane_t, lane_t.ops, ""))
    if wt:
        extra = f", {wt.maxblk}, {wt.lds_bytes}, {1 if gslots else 0}" + (f", &t3_{tag}_lane" if gslots else "")
    else:
        extra = ""
    out.extend(table(tag, t, words, extra))
    out.append("}  // namespace")
    pre = "t3w" if wt else "t3"
    out.append(f"int prepare_{tag}() {{ return t3_prepare(t3_{tag}); }}")
    out.append(f"void launch_jk_{tag}(const JKArgs &a, hipStream_t s) {{ {pre}_launch_jk(t3_{tag}, a, s); }}")
    out.append(f"void launch_eri_{tag}(const EriArgs &a, hipStream_t s) {{ {pre}_launch_eri(t3_{tag}, a, s); }}")
    out.append("}  // namespace hgp")
    out.append("#endif")
    # the buffer holds, per quartet of a batch, either variant's slots
    slots_per_quartet = max(t.nslots + 2, lane_t.nslots) if gslots else t.nslots
    meta = ClassMeta(ls, tag, tier, block, t.n_vrr, t.vrr_flops, t.n_hrr, t.peak_live, t.scheduler, t.p2_flops,
                     len(t.outslots), rule, scratch_slots=slots_per_quartet, chunks=1, recompute=1.0, cap=0,
                     digest="", reduce="none", loop="", max_batch=GSLOT_MAX_BATCH if gslots else 0)
    return "\n".join(out) + "\n", meta
