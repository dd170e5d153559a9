"""HIP emission of the row tier: the staged form for classes whose
accumulator bank and VRR frontier do not fit the register file, arranged so
that the contracted accumulators H never leave the registers.

The paper's Tier 2 (Sec. III-C.2) buffers the whole accumulator bank in
global memory between Phase 1 and Phase 2.  Here Phase 1 is split by bra
component e ("rows" of the target grid [e0|f0], f over every ket
component), and the ket half of Phase 2 runs inside Phase 1:

  Kernel 1, one lane per (quartet, chunk).  A chunk is either
    - a group of whole rows that fits the register line together: the lane
      runs the primitive loop over only the chunk's VRR subgraph (ordered for
      the smallest live set), keeps the rows' accumulators in registers, and
      after the loop applies, row by row, the ket HRR and T(lc) x T(ld)
      (Eq. hrr's ket mirror, Eq. stepwise-sph), storing the (e|lam sig)
      values to the slot-major buffer; or
    - a tile of one row (a subset of its ket components) when even one row
      does not fit: its raw accumulators go to the buffer.
  Kernel 2, one lane per quartet: the ket stage of the tiled rows (from the
    buffer), then per ket function (lam sig) the bra HRR and T(la) x T(lb)
    over the nE values (e|lam sig), giving the integrals, which go to the
    caller's layout (integrals out) or to the buffer for the J/K digestion
    (the six contractions of the 8-fold symmetric Scatter).

Stepwise fusion applied ket-first is the same exact rearrangement of Eq.
materialize-sph as the bra-first order: each index is still transformed as
soon as its recurrence is complete.  Compared with the e-chunked staged tier
this saves one write and one read of N_hrr doubles per quartet and replaces
them with nE * nc * nd, e.g. 3626 instead of 5476 for (ff|ff).

The runtime treats the class as a staged class (a Phase-1 kernel over
quartet x chunk items, then a per-quartet kernel, both in batches through the
slot buffer).
"""
from __future__ import annotations

import dataclasses

from . import phase2 as p2mod
from . import vrr as vrrmod
from .cart import levels
from .emit import ClassMeta, XYZ, loop_close, loop_prelude, tag_of, waves_attr
from .emit_staged import FusedDigest, _names_in, _op_line, node_flops, slot_digestion, subgraph

REGISTER_DOUBLES = 240
ROW_SCHEDULERS = ("dfs_su_e", "dfs_su_f", "dfs")


class SubGraph:
    """The sub-DAG of a VRR graph that reaches a set of targets, renumbered,
    so the schedulers can order it on its own."""

    def __init__(self, g, tids):
        self.back = sorted(subgraph(g, tids))
        idx = {v: i for i, v in enumerate(self.back)}
        self.nodes = []
        for v in self.back:
            nd = g.nodes[v]
            ps = tuple(idx[p] if p is not None else None for p in nd.parents)
            self.nodes.append(vrrmod.Node(nd.key, nd.kind, nd.axis, ps, nd.k_same, nd.k_cross))
        self.children = [[] for _ in self.nodes]
        for v, nd in enumerate(self.nodes):
            for p in nd.parents:
                if p is not None:
                    self.children[p].append(v)
        self.target_ids = [idx[t] for t in tids]


class _SSA:
    """Straight-line ops in Phase2's encoding: (dst, 'hrr', hi, lo, coef) for
    dst = hi + coef * lo, (dst, 'lin', ((c, src), ...)) for dst = sum c * src."""

    def __init__(self, prefix):
        self.ops, self.n, self.prefix, self.flops = [], 0, prefix, 0

    def _new(self):
        self.n += 1
        return f"{self.prefix}{self.n - 1}"

    def hrr(self, hi, lo, coef):
        d = self._new()
        self.ops.append((d, "hrr", hi, lo, coef))
        self.flops += 2
        return d

    def lin(self, terms):
        if len(terms) == 1 and terms[0][0] == 1.0:
            return terms[0][1]
        d = self._new()
        self.ops.append((d, "lin", tuple(terms)))
        self.flops += 2 * len(terms) - 1
        return d


def side_stage(l1, l2, src, coefs, prefix, second=None):
    """One side of the stepwise Phase 2 for a fixed index on the other side:
    the HRR that moves angular momentum onto the second shell,
    (x y+1_i| = (x+1_i y| + R_i (x y| with R = coefs (A - B or C - D), from the
    inputs src(e) for l1 <= |e| <= l1 + l2, then T(l1) on the first index and
    T(l2) on the second (Eq. hrr, Eq. stepwise-sph).  Only the outputs whose
    second spherical index is in `second` (default all) are formed, from the
    part of the recurrence they need.  -> (ops, {(i1, i2): name})."""
    from .cart import add, comps
    from .sph import tmatrix
    rows = lambda l: tmatrix(l) if l >= 2 else tuple(((j, 1.0),) for j in range(len(comps(l))))
    r1, r2 = rows(l1), rows(l2)
    second = list(range(len(r2))) if second is None else list(second)
    b = _SSA(prefix)
    need = sorted({j for nu in second for j, _ in r2[nu]})
    memo = {}

    def X(a, y):
        if sum(y) == 0:
            return src(a)
        if (a, y) in memo:
            return memo[(a, y)]
        i = max(k for k in range(3) if y[k] > 0)
        y1 = add(y, i, -1)
        memo[(a, y)] = b.hrr(X(add(a, i, +1), y1), X(a, y1), coefs[i])
        return memo[(a, y)]

    c2 = comps(l2)
    xy = {(a, j): X(a, c2[j]) for a in comps(l1) for j in need}
    s1 = {}
    for j in need:
        for mu, row in enumerate(r1):
            s1[(mu, j)] = b.lin([(c, xy[(comps(l1)[k], j)]) for k, c in row])
    out = {}
    for mu in range(len(r1)):
        for nu in second:
            out[(mu, nu)] = b.lin([(c, s1[(mu, j)]) for j, c in r2[nu]])
    return b.ops, out


def split(n, parts):
    """range(n) in `parts` contiguous groups."""
    parts = max(1, min(parts, n))
    return [list(range(n))[i * n // parts:(i + 1) * n // parts] for i in range(parts)]


# kernel 2 forms a stage in one piece while it has at most this many inputs;
# beyond, in groups of second-index functions, each reloading its inputs
STAGE_INLINE_INPUTS = 100
STAGE_GROUPS = 3
# Phase-1 chunks per kernel (and translation unit)
P1_PART_CHUNKS = 16


def chunk_order(g, tids):
    """(PeakLive, order in g's node ids) of the chunk's subgraph, scheduled alone."""
    s = SubGraph(g, tids)
    _, pl, order = vrrmod.best_order(s, ROW_SCHEDULERS)
    return pl, [s.back[v] for v in order]


@dataclasses.dataclass
class Chunk:
    kind: str          # 'rows': whole rows, ket stage fused; 'tile': part of one row, raw accumulators stored
    rows: list         # bra components e (one for a tile)
    targets: list      # target node ids, row by row
    order: list        # VRR node ids in emission order
    peak_live: int


@dataclasses.dataclass
class RowPlan:
    ls: tuple
    g: object
    E: list
    F: list
    chunks: list
    tile_rows: list            # rows whose ket stage runs in kernel 2
    kp2: object                # Phase2 of the swapped class: its bra stages are our ket stages
    tindex: dict               # (e, f) -> index into g.targets
    na: int
    nb: int
    nc: int
    nd: int
    budget: int
    bra_groups: int = 1
    ket_groups: int = 1

    def k2_bra(self, lam, sig):
        """Kernel 2's bra stage for ket function (lam, sig): a list of groups
        (ops, {e: input name}, {(mu, nu): output name}); inputs come from the
        (e|lam sig) slots."""
        from .cart import levels  # noqa: F401
        E = self.E
        if self.bra_groups == 1:
            a0, a1 = {(m, n): (x, y) for (m, n, x, y) in self.kp2.ket_stages}[(lam, sig)]
            ins = {e: self.kp2.s2[(lam, sig, e)] for e in E}
            outs = {(mu, nu): self.kp2.out[(lam, sig, mu, nu)] for mu in range(self.na) for nu in range(self.nb)}
            return [(self.kp2.ops[a0:a1], ins, outs)]
        groups = []
        for gi, nus in enumerate(split(self.nb, self.bra_groups)):
            ops, outs = side_stage(self.ls[0], self.ls[1], lambda e: f"in_{E.index(e)}", ("ABx", "ABy", "ABz"),
                                   f"b{gi}_", nus)
            groups.append((ops, {e: f"in_{k}" for k, e in enumerate(E)}, outs))
        return groups

    def k2_ket(self, e):
        """Kernel 2's ket stage of a tiled row e: groups (ops, {f: input name},
        {(lam, sig): output name}); inputs come from the row's H slots."""
        F = self.F
        if self.ket_groups == 1:
            a0, a1 = {f2: (x, y) for (f2, x, y) in self.kp2.bra_stages}[e]
            ins = {f: self.hname(e, f) for f in F}
            outs = {(lam, sig): self.kp2.s2[(lam, sig, e)] for lam in range(self.nc) for sig in range(self.nd)}
            return [(self.kp2.ops[a0:a1], ins, outs)]
        groups = []
        for gi, sigs in enumerate(split(self.nd, self.ket_groups)):
            ops, outs = side_stage(self.ls[2], self.ls[3], lambda f: f"in_{F.index(f)}", ("CDx", "CDy", "CDz"),
                                   f"k{gi}_", sigs)
            groups.append((ops, {f: f"in_{k}" for k, f in enumerate(F)}, outs))
        return groups

    def wave_bra(self):
        """The integrals-out kernel's bra stage, one ket function per lane:
        the same ops for every (lam, sig), inputs (e|lam sig) for each bra
        component e.  -> (ops, {e: input name}, {(mu, nu): output name})."""
        E = self.E
        ops, outs = side_stage(self.ls[0], self.ls[1], lambda e: f"in_{E.index(e)}", ("ABx", "ABy", "ABz"), "w")
        return ops, {e: f"in_{k}" for k, e in enumerate(E)}, outs

    def wave_ket(self):
        """The ket stage of one tiled row, the same ops for every row: inputs
        H[e, f] for each ket component f -> (ops, {f: name}, {(lam, sig): name})."""
        F = self.F
        ops, outs = side_stage(self.ls[2], self.ls[3], lambda f: f"in_{F.index(f)}", ("CDx", "CDy", "CDz"), "t")
        return ops, {f: f"in_{k}" for k, f in enumerate(F)}, outs

    @property
    def ncd(self):
        return self.nc * self.nd

    def zslot(self, ei, lam, sig):
        return ei * self.ncd + lam * self.nd + sig

    def hslot(self, tr, fi):
        return len(self.E) * self.ncd + tr * len(self.F) + fi

    @property
    def nslots_ints(self):
        return len(self.E) * self.ncd + len(self.tile_rows) * len(self.F)

    def islot(self, mu, nu, lam, sig):
        return self.nslots_ints + ((mu * self.nb + nu) * self.nc + lam) * self.nd + sig

    @property
    def nslots(self):
        return self.nslots_ints + self.na * self.nb * self.ncd

    def hname(self, e, f):
        return f"h{self.tindex[(e, f)]}"


def plan_rows(la, lb, lc, ld, budget=REGISTER_DOUBLES, rule="ket_zyx"):
    """Chunks of the target grid: consecutive whole rows packed while
    rows x nF accumulators + the subgraph's PeakLive + 40 stays within the
    register budget (in doubles); a row that does not fit alone is split into
    the fewest equal tiles that do."""
    g = vrrmod.VRRGraph(la, lb, lc, ld, rule=rule)
    E = list(levels(la, la + lb))
    F = list(levels(lc, lc + ld))
    tindex = {t: k for k, t in enumerate(g.targets)}
    row_t = {e: [g.target_ids[tindex[(e, f)]] for f in F] for e in E}
    chunks, tile_rows, cur = [], [], []

    def flush():
        if cur:
            tids = [t for e in cur for t in row_t[e]]
            pl, order = chunk_order(g, tids)
            chunks.append(Chunk("rows", list(cur), tids, order, pl))
            cur.clear()

    for e in E:
        pl, _ = chunk_order(g, row_t[e])
        if len(F) + pl + 40 > budget:
            flush()
            k = 2
            while True:
                ts = row_t[e]
                parts = [ts[i * len(ts) // k:(i + 1) * len(ts) // k] for i in range(k)]
                res = [chunk_order(g, p) for p in parts]
                if all(len(p) + r[0] + 40 <= budget for p, r in zip(parts, res)) or k >= len(ts):
                    break
                k += 1
            for p, (ppl, order) in zip(parts, res):
                chunks.append(Chunk("tile", [e], p, order, ppl))
            tile_rows.append(e)
            continue
        if cur:
            tids = [t for x in cur + [e] for t in row_t[x]]
            pl2, _ = chunk_order(g, tids)
            if len(tids) + pl2 + 40 > budget:
                flush()
        cur.append(e)
    flush()
    hn = lambda e, f: f"h{tindex[(e, f)]}"
    # the swapped class: its "bra" is our ket (HRR in C - D, T(lc), T(ld)) and
    # its "ket" is our bra (HRR in A - B, T(la), T(lb))
    kp2 = p2mod.Phase2(lc, ld, la, lb, hname=lambda x, y: hn(y, x), ab=("CDx", "CDy", "CDz"),
                       cd=("ABx", "ABy", "ABz"))
    groups = lambda n_in: 1 if n_in <= STAGE_INLINE_INPUTS else STAGE_GROUPS
    return RowPlan((la, lb, lc, ld), g, E, F, chunks, tile_rows, kp2, tindex, kp2.nc, kp2.nd, kp2.na, kp2.nb,
                   budget, groups(len(E)), groups(len(F)))


def recompute_factor(plan):
    tot = sum(node_flops(plan.g, set(c.order), len(c.targets)) for c in plan.chunks)
    return tot / plan.g.flops()


def _vrr_lines(g, order, tnames, ind, f32=False):
    """Straight-line VRR of one chunk in `order`; the chunk's own targets
    (tnames) are added to their accumulators.  f32: single precision, with the
    coefficients' float copies (suffix f) and the base values Bf[m]."""
    lines = []
    ty, fm, sfx, one = ("float", "fmaf", "f", "f") if f32 else ("double", "fma", "", "")
    for v in order:
        nd = g.nodes[v]
        if nd.kind == "base":
            expr = f"Bf[{nd.key[2]}]" if f32 else f"base * F[{nd.key[2]}]"
        else:
            p1, p2, p3, p4, p5 = nd.parents
            ax = XYZ[nd.axis]
            if nd.kind == "bra":
                c1, c2, o2, rr = f"PA{ax}", f"WP{ax}", "o2z", "rz"
            else:
                c1, c2, o2, rr = f"QC{ax}", f"WQ{ax}", "o2e", "re"
            expr = f"{fm}({c1}{sfx}, v{p1}, {c2}{sfx} * v{p2})"
            if nd.k_same:
                k = "" if nd.k_same == 1 else f"{nd.k_same}.0{one} * "
                expr = f"{fm}({k}{o2}{sfx}, {fm}(-{rr}{sfx}, v{p4}, v{p3}), {expr})"
            if nd.k_cross:
                k = "" if nd.k_cross == 1 else f"{nd.k_cross}.0{one} * "
                expr = f"{fm}({k}o2ze{sfx}, v{p5}, {expr})"
        lines.append(f"{ind}const {ty} v{v} = {expr};")
        if v in tnames:
            lines.append(f"{ind}{tnames[v]} += v{v};")
    return lines


def _f32_prelude(L, ind):
    """Float copies of one primitive quartet's VRR coefficients and base values
    (the pair quantities and the Boys function stay FP64)."""
    return [
        f"{ind}float Bf[{L + 1}];",
        f"{ind}for (int m = 0; m <= {L}; ++m) Bf[m] = (float)(base * F[m]);",
        f"{ind}const float PAxf = (float)PAx, PAyf = (float)PAy, PAzf = (float)PAz;",
        f"{ind}const float QCxf = (float)QCx, QCyf = (float)QCy, QCzf = (float)QCz;",
        f"{ind}const float WPxf = (float)WPx, WPyf = (float)WPy, WPzf = (float)WPz;",
        f"{ind}const float WQxf = (float)WQx, WQyf = (float)WQy, WQzf = (float)WQz;",
        f"{ind}const float o2zf = (float)o2z, o2ef = (float)o2e, o2zef = (float)o2ze, rzf = (float)rz, ref = (float)re;",
        f"{ind}(void)PAxf; (void)PAyf; (void)PAzf; (void)QCxf; (void)QCyf; (void)QCzf; (void)WPxf; (void)WPyf;",
        f"{ind}(void)WPzf; (void)WQxf; (void)WQyf; (void)WQzf; (void)o2zf; (void)o2ef; (void)o2zef; (void)rzf; (void)ref;",
    ]


def emit_class_row(la, lb, lc, ld, budget=REGISTER_DOUBLES, rule="ket_zyx", block=64, waves=0, reduce="segmented",
                   loop="late", plan=None, eri_layout="quartet", jk_digest="fused"):
    """eri_layout: how Phase 1 hands the (e|lam sig) values to the
    integrals-out kernel: 'quartet' (each quartet's values contiguous: the
    one-wave-per-quartet kernel reads them with coalesced loads, Phase 1
    stores them a row per lane) or 'slot' (slot-major as for J/K: Phase 1
    stores coalesced, the integrals-out kernel gathers).  jk_digest: 'fused'
    (the J/K kernel digests each ket function's integrals while they are in
    registers) or 'slots' (stores them, then six contractions stream them
    back)."""
    ls = (la, lb, lc, ld)
    tag = tag_of(ls)
    assert block == 64, "Phase 1 stages its quartet-major stores per wave"
    plan = plan or plan_rows(la, lb, lc, ld, budget, rule)
    g, E, F, kp2 = plan.g, plan.E, plan.F, plan.kp2
    na, nb, nc, nd = plan.na, plan.nb, plan.nc, plan.nd
    nout = na * nb * nc * nd
    nch = len(plan.chunks)
    eidx = {e: i for i, e in enumerate(E)}
    kstage = {f2: (a0, a1) for (f2, a0, a1) in kp2.bra_stages}        # our ket stage of row e
    bstage = [(mu2, nu2, a0, a1) for (mu2, nu2, a0, a1) in kp2.ket_stages]   # our bra stage of (lam, sig)
    full = g.flops()
    rec = recompute_factor(plan)
    tslot = {t: k for k, t in enumerate(g.target_ids)}
    tile_index = {e: i for i, e in enumerate(plan.tile_rows)}
    fidx = {f: i for i, f in enumerate(F)}

    out = []
    w = out.append
    w(f"// Generated: class ({la}{lb}|{lc}{ld}), row tier: {nch} Phase-1 chunks "
      f"({sum(1 for c in plan.chunks if c.kind == 'rows')} of whole rows, {len(plan.tile_rows)} rows tiled),")
    w(f"// register budget {budget} doubles, VRR recomputation x{rec:.2f}, axis rule {rule}; {len(g.nodes)} VRR nodes,")
    w(f"// {full} VRR FLOP per primitive quartet unchunked, N_hrr {len(g.targets)}, Phase-2 {kp2.flops} FLOP,")
    w(f"// {plan.nslots} buffer slots per quartet ({len(E)} x {plan.ncd} ket-transformed values).")
    w('#include "hgp_device.h"')
    w("")
    w("namespace hgp {")
    w("namespace {")
    w("")

    def ket_stage_lines(e, src, ind):
        """Ket HRR + T(lc) T(ld) of row e; src(f) -> expression of H[e, f];
        stores the (e|lam sig) values to their slots."""
        a0, a1 = kstage[e]
        ops = kp2.ops[a0:a1]
        used = set()
        for op in ops:
            used.update(n for n in _names_in(op) if n.startswith("h"))
        outs = [(lam, sig) for lam in range(nc) for sig in range(nd)]
        for (lam, sig) in outs:
            nm = kp2.s2[(lam, sig, e)]
            if nm.startswith("h"):
                used.add(nm)
        lines = [f"{ind}{{   // ket HRR + T(lc) T(ld) of bra component {e}"]
        for h in sorted(used, key=lambda x: int(x[1:])):
            f = g.targets[int(h[1:])][1]
            lines.append(f"{ind}    const double r_{h} = {src(f)};")
        ren = {h: f"r_{h}" for h in used}
        for op in ops:
            lines.append(f"{ind}    " + _op_line(op, ren))
        vals = [ren.get(kp2.s2[(lam, sig, e)], kp2.s2[(lam, sig, e)]) for (lam, sig) in outs]
        lines.extend(run_store(plan.zslot(eidx[e], 0, 0), vals, ind + "    "))
        lines.append(f"{ind}}}")
        lines.append(f"{ind}HGP_STAGE(li);")
        return lines

    def run_store(base, vals, ind):
        """Store vals to the consecutive slots base, base+1, ...: slot-major,
        one store per value, or (quartet-major, integrals out) through the
        wave's LDS tile so that each quartet's run is written by consecutive
        lanes (coalesced)."""
        cnt = len(vals)
        lines = [f"{ind}if (a.qmajor) {{"]
        for c, v in enumerate(vals):
            lines.append(f"{ind}    zt[threadIdx.x * {cnt} + {c}] = {v};")
        lines.append(f"{ind}    hgp_store_runs<{cnt}>(zt, sb, i0, a.n, {plan.nslots}u, {base}u);")
        lines.append(f"{ind}}} else {{")
        for c, v in enumerate(vals):
            lines.append(f"{ind}    sb[{base + c}u * S32 + li] = {v};")
        lines.append(f"{ind}}}")
        return lines

    # ---------------------------------------------------------------- Phase 1 (+ fused ket stage)
    # The chunks are spread over parts of at most P1_PART_CHUNKS, each its own
    # kernel in its own translation unit: the compiler allocates registers per
    # part, and the parts compile in parallel.
    parts = split(nch, -(-nch // P1_PART_CHUNKS))
    part_src = {}
    for (prec, pfx, key), (pi, idxs) in [(x, y) for x in (("f64", "p1_", "p"), ("f32", "p1f_", "q"))
                                         for y in enumerate(parts)]:
        f32 = prec == "f32"
        po = []
        pw = po.append
        pw(f"// Generated: class ({la}{lb}|{lc}{ld}), row tier, Phase-1 part {pi} of {len(parts)} "
           f"(chunks {idxs[0]}..{idxs[-1]} of {nch})" +
           (", VRR and contraction in FP32 (pair quantities, Boys, ket stage in FP64)." if f32 else "."))
        pw('#include "hgp_device.h"')
        pw("")
        pw("namespace hgp {")
        pw("namespace {")
        pw("")
        npc = len(idxs)
        zmax = max([plan.ncd] + [len(plan.chunks[ci].targets) for ci in idxs if plan.chunks[ci].kind == "tile"])
        pw("// Quartet-major stores: a run of CNT consecutive slots of each of the wave's")
        pw("// quartets, staged by every lane in zt[lane * CNT + c], written by consecutive")
        pw("// lanes one quartet at a time.")
        pw("template <int CNT>")
        pw("__device__ __forceinline__ void hgp_store_runs(double *zt, double *sb, int64_t i0, int64_t n, uint32_t ns,")
        pw("                                               uint32_t base)")
        pw("{")
        pw("    __syncthreads();")
        pw("    for (int q = 0; q < 64 && i0 + q < n; ++q)")
        pw("        for (int c = threadIdx.x; c < CNT; c += 64)")
        pw("            sb[(uint64_t)(i0 + q) * ns + base + c] = zt[q * CNT + c];")
        pw("    __syncthreads();")
        pw("}")
        pw("")
        pw(f"// item (block / {npc}) * {block} + thread, chunk = block % {npc}.")
        pw(f"__global__ __launch_bounds__({block}){waves_attr(waves)} void {pfx}{tag}p{pi}(P1Args a)")
        pw("{")
        pw(f"    __shared__ double zt[64 * {zmax}];")
        pw(f"    const int chunk = (int)(blockIdx.x % {npc});")
        pw(f"    const int64_t i0 = (int64_t)(blockIdx.x / {npc}) * 64;")
        pw("    const int64_t iraw = i0 + threadIdx.x;")
        pw("    // quartet-major: every lane stays for the wave's cooperative stores (lanes past")
        pw("    // the end redo the last item and store nothing of their own)")
        pw("    if (iraw >= a.n && !a.qmajor) return;")
        pw("    const int64_t i = iraw < a.n ? iraw : a.n - 1;")
        pw("    const int bra = a.idx[i * a.istride], ket = a.idx[i * a.istride + 1];")
        pw("    const PairInfo pb = a.pairs[bra], pk = a.pairs[ket];")
        pw("    const PairGeo gb = a.geo[bra], gk = a.geo[ket];")
        pw("    const PrimPair *__restrict__ prims = a.prims;")
        pw("    const double *__restrict__ boys = a.boys;")
        pw("    double *const sb = a.scratch;")
        pw("    // slot k of item i: sb[k * S32 + li] with S32 the batch stride (slot-major), or with")
        pw(f"    // S32 = 1 and li = i * {plan.nslots} (quartet-major, integrals out)")
        pw(f"    const uint32_t S32 = a.qmajor ? 1u : (uint32_t)a.stride;")
        pw(f"    uint32_t li = a.qmajor ? (uint32_t)i * {plan.nslots}u : (uint32_t)i;")
        pw("    switch (chunk) {")
        for lci, ci in enumerate(idxs):
            ch = plan.chunks[ci]
            Lc = max(g.nodes[v].key[2] for v in ch.order if g.nodes[v].kind == "base")
            tnames = {t: f"h{tslot[t]}" for t in ch.targets}
            pw(f"    case {lci}: {{   // chunk {ci}, {ch.kind}: rows {[eidx[e] for e in ch.rows]}, "
               f"{len(ch.targets)} accumulators, {len(ch.order)} VRR nodes, PeakLive {ch.peak_live}")
            names = [tnames[t] for t in ch.targets]
            acc = {t: (f"{tnames[t]}f" if f32 else tnames[t]) for t in ch.targets}
            ty, zero = ("float", "0.0f") if f32 else ("double", "0.0")
            anames = [acc[t] for t in ch.targets]
            for k in range(0, len(anames), 8):
                pw(f"        {ty} " + ", ".join(f"{h} = {zero}" for h in anames[k:k + 8]) + ";")
            po.extend(loop_prelude(Lc, "        ", loop))
            if f32:
                po.extend(_f32_prelude(Lc, "            "))
            po.extend(_vrr_lines(g, ch.order, acc, "            ", f32))
            po.extend(loop_close("        "))
            if f32:
                for k in range(0, len(names), 8):
                    pw("        const double " + ", ".join(f"{h} = (double){h}f" for h in names[k:k + 8]) + ";")
            if ch.kind == "rows":
                pw("        const double CDx = gk.abx, CDy = gk.aby, CDz = gk.abz;")
                pw("        (void)CDx; (void)CDy; (void)CDz;")
                for e in ch.rows:
                    po.extend(ket_stage_lines(e, lambda f, e=e: plan.hname(e, f), "        "))
            else:
                e = ch.rows[0]
                fs = [fidx[g.nodes[t].key[1]] for t in ch.targets]
                assert fs == list(range(fs[0], fs[0] + len(fs))), "a tile is a contiguous run of ket components"
                po.extend(run_store(plan.hslot(tile_index[e], fs[0]), [f"h{tslot[t]}" for t in ch.targets], "        "))
            pw("        break;")
            pw("    }")
        pw("    default:")
        pw("        break;")
        pw("    }")
        pw("}")
        pw("")
        pw("}  // namespace")
        pw("")
        pw(f"void launch_{pfx}{tag}p{pi}(const P1Args &a, hipStream_t s)")
        pw("{")
        pw(f"    const int64_t blocks = (a.n + {block - 1}) / {block};")
        pw(f"    if (blocks > 0) hipLaunchKernelGGL({pfx}{tag}p{pi}, dim3((unsigned)(blocks * {npc})), dim3({block}), 0, s, a);")
        pw("}")
        pw("")
        pw("}  // namespace hgp")
        part_src[f"{key}{pi}"] = "\n".join(po) + "\n"

    # ---------------------------------------------------------------- Phase 2 (bra half)
    def group_lines(ops, ins, outs, load, sink, ind):
        """One stage group: load the inputs its ops (or outputs) use, run the
        ops, hand each output to sink(key, expr, ind), then fence."""
        used = {n for op in ops for n in _names_in(op)} | set(outs.values())
        lines = [f"{ind}{{"]
        ren = {}
        for k, (key, nm) in enumerate(ins.items()):
            if nm in used:
                ren[nm] = f"y{k}"
                lines.append(f"{ind}    const double y{k} = {load(key)};")
        for op in ops:
            lines.append(f"{ind}    " + _op_line(op, ren))
        for key, nm in outs.items():
            lines.extend(sink(key, ren.get(nm, nm), ind + "    "))
        lines.append(f"{ind}}}")
        lines.append(f"{ind}HGP_STAGE(li);")
        return lines

    def phase2_lines(sink, ind="    ", digest=None):
        """Kernel 2's work for one quartet up to the integrals: the ket stage of
        the tiled rows (from their H slots), then per ket function (lam, sig)
        the bra HRR + T(la) T(lb) from the (e|lam sig) slots; sink(mu, nu, lam,
        sig, expr, ind) emits each integral's use.  A stage with many inputs
        runs in groups of second-index functions, each reloading its inputs.
        digest: a FusedDigest over slices (lam, sig); each stage's integrals
        then go to registers c<mu>_<nu> and are digested after the stage."""
        lines = []
        if plan.tile_rows:
            lines.append(f"{ind}const double CDx = gk.abx, CDy = gk.aby, CDz = gk.abz;")
            lines.append(f"{ind}(void)CDx; (void)CDy; (void)CDz;")
            for e in plan.tile_rows:
                tr = tile_index[e]
                for ops, ins, outs in plan.k2_ket(e):
                    lines.extend(group_lines(
                        ops, ins, outs, lambda f, tr=tr: f"sb[{plan.hslot(tr, fidx[f])}u * S32 + li]",
                        lambda key, x, i2, e=e: [f"{i2}sb[{plan.zslot(eidx[e], key[0], key[1])}u * S32 + li] = {x};"],
                        ind))
        lines.append(f"{ind}const double ABx = gb.abx, ABy = gb.aby, ABz = gb.abz;")
        lines.append(f"{ind}(void)ABx; (void)ABy; (void)ABz;")
        for lam in range(nc):
            if digest is not None:
                lines.extend(digest.outer_begin(lam, ind))
            for sig in range(nd):
                lines.append(f"{ind}// bra HRR + T(la) T(lb) for ket functions ({lam}, {sig})")
                si = ind
                if digest is not None:
                    lines.append(f"{ind}{{")
                    si = ind + "    "
                    cs = [f"c{mu}_{nu}" for mu in range(na) for nu in range(nb)]
                    for k in range(0, len(cs), 8):
                        lines.append(f"{si}double " + ", ".join(cs[k:k + 8]) + ";")
                    snk = lambda mu, nu, lam_, sig_, x, i2: [f"{i2}c{mu}_{nu} = {x};"]
                else:
                    snk = sink
                for ops, ins, outs in plan.k2_bra(lam, sig):
                    lines.extend(group_lines(
                        ops, ins, outs, lambda e, lam=lam, sig=sig: f"sb[{plan.zslot(eidx[e], lam, sig)}u * S32 + li]",
                        lambda key, x, i2, lam=lam, sig=sig, snk=snk: snk(key[0], key[1], lam, sig, x, i2), si))
                if digest is not None:
                    lines.extend(digest.slice(lam, sig, lambda r, s_: f"c{r}_{s_}", si))
                    lines.append(f"{ind}}}")
            if digest is not None:
                lines.extend(digest.outer_end(lam, ind))
        return lines

    # ---------------------------------------------------------------- kernel 2: integrals out, one wave per quartet
    # Phase 1 wrote the quartet's values contiguously (quartet-major).  First
    # the lanes take the tiled rows, one each: ket HRR + T(lc) T(ld) from the
    # row's raw accumulators into the LDS tile zt.  Then lane j takes ket
    # function j = (lam, sig): it reads (e|lam sig) for every e (from zt for
    # tiled rows, else from the buffer, where the lanes read consecutive
    # doubles), runs the bra HRR + T(la) T(lb), and writes the (mu nu|lam sig)
    # values, which for a fixed (mu, nu) lie next to each other in the
    # caller's block, so the stores are coalesced too.
    # A wave takes P = 64 // ncd quartets at once when several fit (lanes
    # sub * ncd .. sub * ncd + ncd - 1 for quartet sub); the Schwarz mode
    # (one value per quartet, a reduction over the quartet's lanes) runs P = 1.
    diag_class = (la, lb) == (lc, ld)
    ncd = plan.ncd
    assert ncd <= 64, "one ket function per lane"
    NS = plan.nslots
    P = max(1, 64 // ncd)
    wops, wins, wouts = plan.wave_bra()
    nt = len(plan.tile_rows)

    def zbase(q):
        return f"a.scratch + (uint64_t)({q}) * {NS}u" if eri_layout == "quartet" else f"a.scratch + ({q})"

    w("template <int P>")
    w(f"__global__ __launch_bounds__(64) void eri_{tag}(EriArgs a)")
    w("{")
    if nt:
        w(f"    __shared__ double zt[P * {nt * ncd}];")
    w("    const int j = threadIdx.x;")
    w("    const int64_t q0 = (int64_t)blockIdx.x * P;      // first quartet of this wave")
    w("    if (q0 >= a.ntask) return;")
    w(f"    const int sub = P == 1 ? 0 : j / {ncd};")
    w(f"    const int jj = j - sub * {ncd};                  // ket function of this lane")
    w(f"    const bool act = sub < P && jj < {ncd} && q0 + sub < a.ntask;")
    w("    const int64_t i = act ? q0 + sub : q0;")
    w("    const EriTask t = a.tasks[i];")
    w(f"    const double *__restrict__ zq = {zbase('i')};")
    w(f"    const uint32_t ZS = {'1u' if eri_layout == 'quartet' else '(uint32_t)a.stride'};")
    if nt:
        tops, tins, touts = plan.wave_ket()
        w(f"    for (int job = j; job < P * {nt}; job += 64) {{   // tiled row tr of quartet qs")
        w(f"        const int qs = job / {nt}, tr = job - qs * {nt};")
        w("        if (q0 + qs >= a.ntask) continue;")
        w("        const EriTask etask = a.tasks[q0 + qs];")
        w("        const PairGeo gk = a.geo[etask.ket];")
        w("        const double CDx = gk.abx, CDy = gk.aby, CDz = gk.abz;")
        w("        (void)CDx; (void)CDy; (void)CDz;")
        w(f"        const double *__restrict__ hrow = {zbase('q0 + qs')} + ({plan.hslot(0, 0)}u + tr * {len(F)}u) * ZS;")
        tused = {n for op in tops for n in _names_in(op)} | set(touts.values())
        for k, f in enumerate(F):
            nm = tins[f]
            if nm in tused:
                w(f"        const double {nm} = hrow[{k}u * ZS];")
        for op in tops:
            w("        " + _op_line(op, {}))
        for lam in range(nc):
            for sig in range(nd):
                w(f"        zt[(qs * {nt} + tr) * {ncd} + {lam * nd + sig}] = {touts[(lam, sig)]};")
        w("    }")
        w("    __syncthreads();")
    w("    const PairGeo gb = a.geo[t.bra];")
    w("    const double ABx = gb.abx, ABy = gb.aby, ABz = gb.abz;")
    w("    (void)ABx; (void)ABy; (void)ABz;")
    w("    double dg = 0.0;")
    w("    if (act) {")
    w(f"        const int lam = jj / {nd}, sig = jj - lam * {nd};")
    used = {n for op in wops for n in _names_in(op)} | set(wouts.values())
    for k, e in enumerate(E):
        nm = wins[e]
        if nm not in used:
            continue
        if e in tile_index:
            w(f"        const double {nm} = zt[(sub * {nt} + {tile_index[e]}) * {ncd} + jj];")
        else:
            w(f"        const double {nm} = zq[({plan.zslot(k, 0, 0)}u + jj) * ZS];")
    for op in wops:
        w("        " + _op_line(op, {}))
    w("        if (a.mode == 0) {")
    w("            double *__restrict__ o = a.out + t.off + lam * t.s2 + sig * t.s3;")
    for mu in range(na):
        for nu in range(nb):
            w(f"            o[{mu} * t.s0 + {nu} * t.s1] = {wouts[(mu, nu)]};")
    w("        }")
    if diag_class:
        for mu in range(na):
            for nu in range(nb):
                w(f"        if (lam == {mu} && sig == {nu}) dg = fabs({wouts[(mu, nu)]});")
    w("    }")
    if diag_class:
        w("    if (P == 1 && a.mode == 1) {                  // Schwarz factor: largest diagonal element")
        w("#pragma unroll")
        w("        for (int o = 32; o > 0; o >>= 1) dg = fmax(dg, __shfl_xor(dg, o, 64));")
        w("        if (j == 0) a.out[i] = sqrt(dg);")
        w("    }")
    w("    (void)dg;")
    w("}")
    w("")
    # ---------------------------------------------------------------- kernel 2: J/K (own translation unit)
    jo = []
    jw = jo.append
    jw(f"// Generated: class ({la}{lb}|{lc}{ld}), row tier, Phase 2 + J/K digestion.")
    jw('#include "hgp_device.h"')
    jw("")
    jw("namespace hgp {")
    jw("namespace {")
    jw("")
    jw(f"__global__ __launch_bounds__({block}) void jk_{tag}(JKArgs a)")
    jw("{")
    jw(f"    const int64_t i = (int64_t)blockIdx.x * {block} + threadIdx.x;")
    jw("    if (i >= a.nq) return;")
    jw("    double *const sb = a.scratch;")
    jw("    const uint32_t S32 = (uint32_t)a.stride;")
    jw("    uint32_t li = (uint32_t)i;")
    jw("    const double *__restrict__ D = a.D;")
    jw("    const int N = a.nbf;")
    jw("    const int2 pq = a.quartets[i];")
    jw("    const PairInfo pb = a.pairs[pq.x], pk = a.pairs[pq.y];")
    jw("    const PairGeo gb = a.geo[pq.x], gk = a.geo[pq.y];")
    jw("    const int fa = pb.fa, fb = pb.fb, fc = pk.fa, fd = pk.fb;")
    jw("    const double s = (pb.same ? 0.5 : 1.0) * (pk.same ? 0.5 : 1.0) * (pq.x == pq.y ? 0.5 : 1.0);")
    jw("    const double sj = a.want_j ? 2.0 * s : 0.0, sk = a.want_k ? s : 0.0;")
    if jk_digest == "fused":
        # each ket function's integrals digested as the bra stage makes them
        fdg = FusedDigest((na, nb, nc, nd), 2, 3, reduce)
        jo.extend(fdg.prologue())
        jo.extend(phase2_lines(None, digest=fdg))
        jo.extend(fdg.epilogue())
    else:
        jo.extend(phase2_lines(lambda mu, nu, lam, sig, x, ind: [f"{ind}sb[{plan.islot(mu, nu, lam, sig)}u * S32 + li] = {x};"]))
        jo.extend(slot_digestion(na, nb, nc, nd, lambda mu, nu, lam, sig: f"sb[{plan.islot(mu, nu, lam, sig)}u * S32 + li]",
                                 reduce))
    jw("}")
    jw("")
    jw("}  // namespace")
    jw("")
    jw(f"void launch_jk_{tag}(const JKArgs &a, hipStream_t s)")
    jw("{")
    jw(f"    const int64_t blocks = (a.nq + {block - 1}) / {block};")
    jw(f"    if (blocks > 0) hipLaunchKernelGGL(jk_{tag}, dim3((unsigned)blocks), dim3({block}), 0, s, a);")
    jw("}")
    jw("")
    jw("}  // namespace hgp")
    part_src["jk"] = "\n".join(jo) + "\n"

    w("}  // namespace")
    w("")
    for pfx in ("p1_", "p1f_"):
        for pi in range(len(parts)):
            w(f"void launch_{pfx}{tag}p{pi}(const P1Args &a, hipStream_t s);")
        w(f"void launch_{pfx}{tag}(const P1Args &a, hipStream_t s)")
        w("{")
        for pi in range(len(parts)):
            w(f"    launch_{pfx}{tag}p{pi}(a, s);")
        w("}")
    w(f"void launch_eri_{tag}(const EriArgs &a, hipStream_t s)")
    w("{")
    w("    if (a.ntask <= 0) return;")
    if P > 1:
        w("    if (a.mode == 0) {")
        w(f"        hipLaunchKernelGGL(eri_{tag}<{P}>, dim3((unsigned)((a.ntask + {P - 1}) / {P})), dim3(64), 0, s, a);")
        w("        return;")
        w("    }")
    w(f"    hipLaunchKernelGGL(eri_{tag}<1>, dim3((unsigned)a.ntask), dim3(64), 0, s, a);")
    w("}")

    w("")
    w("}  // namespace hgp")
    pl_max = max(c.peak_live for c in plan.chunks)
    meta = ClassMeta(ls, tag, 1, block, len(g.nodes), full, len(g.targets), pl_max, "per-chunk", kp2.flops, nout, rule,
                     scratch_slots=plan.nslots, chunks=nch, recompute=rec, cap=budget, waves=waves, digest="",
                     reduce=reduce, loop=loop)
    meta.form = "row"
    meta.p1_32 = True                # Phase 1 also in FP32 (launch_p1f_<class>) for mixed precision
    meta.eri_wave = eri_layout == "quartet"        # Phase 1 writes quartet-major for integrals out
    meta.eri_tiles = False          # the tiled rows' ket stage runs inside the integrals-out kernel
    meta.parts = len(parts)
    meta.jk_digest = jk_digest
    meta.extra_sources = part_src
    return "\n".join(out) + "\n", meta
