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

OP_VRR_BRA, OP_VRR_KET, OP_ACC, OP_HRR_BRA, OP_HRR_KET, OP_LIN, OP_LIN_ACC = 1, 2, 3, 4, 5, 6, 7
NONE = 0xFFFF
XYZ_AXIS = {"x": 0, "y": 1, "z": 2}


@dataclasses.dataclass
class T3Tables:
    ops: list            # flat uint16 words, 8 per op
    n_vrr: int           # ops of the per-primitive part (VRR + ACC)
    n_p2: int            # ops of Phase 2
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


def build_tables(la, lb, lc, ld, rule="ket_zyx", schedulers=None) -> T3Tables:
    ls = (la, lb, lc, ld)
    L = sum(ls)
    g = vrrmod.VRRGraph(*ls, rule=rule)
    sched, pl, order = vrrmod.best_order(g) if schedulers is None else vrrmod.best_order(g, schedulers)
    n_hrr = len(g.targets)
    acc0 = L + 1
    words = []

    def op(w0, dst, a=NONE, b=NONE, c=NONE, d=NONE, e=NONE, f=NONE):
        words.extend((w0, dst, a, b, c, d, e, f))

    # ---- per-primitive part: VRR in schedule order, targets into accumulators
    pos = {v: k for k, v in enumerate(order)}
    last = [-1] * len(g.nodes)
    for v in order:
        for c in g.children[v]:
            last[v] = max(last[v], pos[c])
    tpos = {tid: k for k, tid in enumerate(g.target_ids)}
    slot = [None] * len(g.nodes)
    alloc = _Slots(acc0 + n_hrr)
    dies = {}
    for k, v in enumerate(order):
        nd = g.nodes[v]
        if nd.kind == "base":
            slot[v] = nd.key[2]                  # base * F_m sits in slot m
        else:
            s = alloc.get()
            slot[v] = s
            p = [slot[x] if x is not None else NONE for x in nd.parents]
            code = OP_VRR_BRA if nd.kind == "bra" else OP_VRR_KET
            op(code | (nd.axis << 4) | (nd.k_same << 6) | (nd.k_cross << 11), s, *p)
        if v in tpos:
            op(OP_ACC, acc0 + tpos[v], slot[v])
        if nd.kind != "base":
            if last[v] > k:
                dies.setdefault(last[v], []).append(v)
            else:
                alloc.put(slot[v])               # a target with no consumer: dead after ACC
        for u in dies.pop(k, ()):
            alloc.put(slot[u])
    n_vrr = len(words) // 8
    vrr_top = alloc.next

    # ---- Phase 2: HRR + stepwise transforms over the accumulators
    hname = {t: f"h{k}" for k, t in enumerate(g.targets)}
    p2 = p2mod.Phase2(la, lb, lc, ld, hname=lambda e, f: hname[(e, f)])
    name_slot = {f"h{k}": acc0 + k for k in range(n_hrr)}
    outputs = set(p2.out.values())
    p2pos = {}
    for k, o in enumerate(p2.ops):
        srcs = (o[2], o[3]) if o[1] == "hrr" else tuple(s for _, s in o[2])
        for s in srcs:
            p2pos[s] = k                         # last use
    alloc2 = _Slots(vrr_top)
    alloc2.free = sorted(range(acc0 + n_hrr, vrr_top), reverse=True)   # VRR temporaries are dead now
    coefs, cidx = [], {}

    def coef(c):
        c = float(c)
        if c not in cidx:
            cidx[c] = len(coefs)
            coefs.append(c)
        return cidx[c]

    for k, o in enumerate(p2.ops):
        d = o[0]
        s = alloc2.get()
        name_slot[d] = s
        if o[1] == "hrr":
            _, _, hi, lo, cname = o
            axis = XYZ_AXIS[cname[-1]]
            code = OP_HRR_BRA if cname.startswith("AB") else OP_HRR_KET
            op(code | (axis << 4), s, name_slot[hi], name_slot[lo])
        else:
            terms = list(o[2])
            for j in range(0, len(terms), 3):
                chunk = terms[j:j + 3]
                srcs = [name_slot[x] for _, x in chunk] + [NONE] * (3 - len(chunk))
                cs = [coef(c) for c, _ in chunk] + [0] * (3 - len(chunk))
                op(OP_LIN if j == 0 else OP_LIN_ACC, s, *srcs, *cs)
        srcs = (o[2], o[3]) if o[1] == "hrr" else tuple(x for _, x in o[2])
        for x in set(srcs):
            if p2pos.get(x) == k and x not in outputs:
                alloc2.put(name_slot[x])
    n_p2 = len(words) // 8 - n_vrr
    nslots = max(alloc2.next, vrr_top)
    if nslots > 0xFFFE or len(coefs) > 0xFFFF:
        raise ValueError(f"class {tag_of(ls)}: {nslots} slots do not fit 16-bit slot indices")
    na, nb, nc, nd = (nsph(x) for x in ls)
    outslots = [name_slot[p2.out[(mu, nu, lam, sig)]] for mu in range(na) for nu in range(nb)
                for lam in range(nc) for sig in range(nd)]
    return T3Tables(words, n_vrr, n_p2, coefs, outslots, nslots, n_hrr, acc0, L, pl, sched, g.flops(), p2.flops)


def _u16_lines(vals, per=24):
    out = []
    for k in range(0, len(vals), per):
        out.append("    " + ", ".join(str(v) for v in vals[k:k + per]) + ",")
    return out


def emit_class_t3(la, lb, lc, ld, rule="ket_zyx", schedulers=None, block=64):
    """Host-side tables plus the launchers that hand them to the generic
    HBM-scratch kernels; no device code is generated for the class."""
    ls = (la, lb, lc, ld)
    tag = tag_of(ls)
    t = build_tables(la, lb, lc, ld, rule, schedulers)
    na, nb, nc, nd = (nsph(x) for x in ls)
    out = [f"// Generated: class ({la}{lb}|{lc}{ld}) for the HBM-scratch tier, axis rule {rule},",
           f"// VRR order '{t.scheduler}' (PeakLive {t.peak_live}), {t.n_vrr} per-primitive ops,",
           f"// {t.n_p2} Phase-2 ops, {t.nslots} slots per lane, {len(t.outslots)} spherical integrals.",
           '#include "hgp_t3.h"', "", "#if !defined(__HIP_DEVICE_COMPILE__)", "namespace hgp {", "namespace {", ""]
    out.append(f"const uint16_t ops_{tag}[] = {{")
    out.extend(_u16_lines(t.ops))
    out.append("};")
    out.append(f"const uint16_t outslots_{tag}[] = {{")
    out.extend(_u16_lines(t.outslots))
    out.append("};")
    out.append(f"const double coefs_{tag}[] = {{")
    for k in range(0, max(len(t.coefs), 1), 4):
        out.append("    " + ", ".join(repr(c) for c in (t.coefs[k:k + 4] or [0.0])) + ",")
    out.append("};")
    out.append(f"T3Class t3_{tag} = {{{la}, {lb}, {lc}, {ld}, {t.L}, {na}, {nb}, {nc}, {nd}, {t.nslots}, {t.n_hrr}, "
               f"{t.acc0}, {t.n_vrr}, {t.n_p2}, ops_{tag}, {max(len(t.coefs), 1)}, coefs_{tag}, outslots_{tag}, {block}}};")
    out.append("")
    out.append("}  // namespace")
    out.append(f"int prepare_{tag}() {{ return t3_prepare(t3_{tag}); }}")
    out.append(f"void launch_jk_{tag}(const JKArgs &a, hipStream_t s) {{ t3_launch_jk(t3_{tag}, a, s); }}")
    out.append(f"void launch_eri_{tag}(const EriArgs &a, hipStream_t s) {{ t3_launch_eri(t3_{tag}, a, s); }}")
    out.append("}  // namespace hgp")
    out.append("#endif")
    meta = ClassMeta(ls, tag, 2, block, t.n_vrr, t.vrr_flops, t.n_hrr, t.peak_live, t.scheduler, t.p2_flops,
                     len(t.outslots), rule, scratch_slots=t.nslots, chunks=1, recompute=1.0, cap=0, digest="",
                     reduce="none", loop="")
    return "\n".join(out) + "\n", meta
