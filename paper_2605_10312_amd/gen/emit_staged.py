"""HIP emission of the staged (HBM-scratch) tier for classes whose accumulator
bank and VRR frontier do not fit the register file together (Sec. III-C's
Regime II; the paper's buffered Tier 2, Sec. III-C.2, redesigned for gfx950).

The class list is processed in batches of B quartets (B = the scratch
buffer's lane count).  A slot-major buffer in HBM holds, for quartet i of the
batch, slot k at scratch[k * B + i], so consecutive lanes touch consecutive
addresses.  Per batch, two kernels:

  Kernel 1 (Phase 1): one lane per (quartet, chunk).  The targets [e0|f0] are
    split by bra component e into chunks of at most `cap` accumulators; a
    lane runs the primitive loops over only its chunk's VRR subgraph (the
    sub-DAG reaching its targets), keeps the accumulators in registers and
    stores them once.  Blocks alternate over chunks, so each wavefront runs
    one chunk's code and small classes still fill the GPU.
  Kernel 2 (Phase 2 + digestion), one lane per quartet:
    bra stage, one ket component f at a time: load H[:, f], bra HRR, T(la)
      then T(lb), store the spherical (m n|f) values over H[:, f]'s slots;
    ket stage, one (m, n) at a time: load (m n|f) for all f, ket HRR, T(lc)
      then T(ld), store the final integrals to their own slots;
    digestion (J/K): the six contractions of the 8-fold symmetric Scatter,
      each streaming the integrals back, FP64 atomics.  The integrals-out
      variant copies them to the caller's layout instead.

Compared with a single register-resident evaluation, chunking recomputes the
VRR nodes shared between chunks (the generator reports the factor); in
exchange every stage runs without compiler spills.
"""
from __future__ import annotations

from . import phase2 as p2mod
from . import vrr as vrrmod
from .cart import levels
from .emit import ClassMeta, XYZ, _fmt, loop_close, loop_prelude, tag_of, waves_attr


def chunk_targets(g, cap):
    """Group the targets by bra component e (in level order), packing whole
    e rows (all f) into chunks of at most cap accumulators."""
    la, lb, lc, ld = g.ls
    nf = len(levels(lc, lc + ld))
    per_row = max(1, cap // nf)
    es = list(levels(la, la + lb))
    rows = [es[i:i + per_row] for i in range(0, len(es), per_row)]
    out = []
    for r in rows:
        rs = set(r)
        out.append([t for t in g.target_ids if g.nodes[t].key[0] in rs])
    return out


def subgraph(g, tids):
    seen = set()
    st = list(tids)
    while st:
        v = st.pop()
        if v in seen:
            continue
        seen.add(v)
        for p in g.nodes[v].parents:
            if p is not None:
                st.append(p)
    return seen


def node_flops(g, nodes, ntarg):
    n = 0
    for v in nodes:
        nd = g.nodes[v]
        if nd.kind == "base":
            n += 1
            continue
        n += 3 + (4 if nd.k_same else 0) + (2 if nd.k_cross else 0)
    return n + ntarg


def _vrr_chunk_lines(g, order, tnames, ind):
    lines = []
    for v in order:
        nd = g.nodes[v]
        if nd.kind == "base":
            expr = f"base * F[{nd.key[2]}]"
        else:
            p1, p2, p3, p4, p5 = nd.parents
            ax = XYZ[nd.axis]
            if nd.kind == "bra":
                c1, c2, o2, rr = f"PA{ax}", f"WP{ax}", "o2z", "rz"
            else:
                c1, c2, o2, rr = f"QC{ax}", f"WQ{ax}", "o2e", "re"
            expr = f"fma({c1}, v{p1}, {c2} * v{p2})"
            if nd.k_same:
                k = "" if nd.k_same == 1 else f"{nd.k_same}.0 * "
                expr = f"fma({k}{o2}, fma(-{rr}, v{p4}, v{p3}), {expr})"
            if nd.k_cross:
                k = "" if nd.k_cross == 1 else f"{nd.k_cross}.0 * "
                expr = f"fma({k}o2ze, v{p5}, {expr})"
        lines.append(f"{ind}const double v{v} = {expr};")
        if v in tnames:
            lines.append(f"{ind}{tnames[v]} += v{v};")
    return lines


def _op_line(op, ren):
    r = lambda n: ren.get(n, n)
    if op[1] == "hrr":
        d, _, hi, lo, coef = op
        return f"const double {d} = fma({coef}, {r(lo)}, {r(hi)});"
    d, _, terms = op
    expr = f"{_fmt(terms[0][0])} * {r(terms[0][1])}"
    for c, s in terms[1:]:
        expr = f"fma({_fmt(c)}, {r(s)}, {expr})"
    return f"const double {d} = {expr};"


def _names_in(op):
    if op[1] == "hrr":
        return [op[2], op[3]]
    return [s for _, s in op[2]]


def emit_class_staged(la, lb, lc, ld, cap=96, rule="ket_zyx", block=64, schedulers=None, waves=0,
                      reduce="segmented", loop="late", jk_digest="fused"):
    ls = (la, lb, lc, ld)
    tag = tag_of(ls)
    g = vrrmod.VRRGraph(la, lb, lc, ld, rule=rule)
    sched, pl, order = vrrmod.best_order(g) if schedulers is None else vrrmod.best_order(g, schedulers)
    tslot = {tid: k for k, tid in enumerate(g.target_ids)}          # H slot of each target node
    hname_of = {t: f"h{k}" for k, t in enumerate(g.targets)}
    p2 = p2mod.Phase2(la, lb, lc, ld, hname=lambda e, f: hname_of[(e, f)])
    na, nb, nc, nd = p2.na, p2.nb, p2.nc, p2.nd
    nout = na * nb * nc * nd
    E = list(levels(la, la + lb))
    assert na * nb <= len(E)
    hslot = {f"h{k}": k for k in range(len(g.targets))}
    tindex = {t: k for k, t in enumerate(g.targets)}
    n_h = len(g.targets)
    islot = lambda mu, nu, lam, sig: n_h + ((mu * nb + nu) * nc + lam) * nd + sig
    # H slots, then (for the six-pass digestion only) the integrals
    nslots = n_h + (nout if jk_digest == "slots" else 0)
    chunks = chunk_targets(g, cap)
    full = g.flops()
    recompute = sum(node_flops(g, subgraph(g, c), len(c)) for c in chunks) / full

    out = []
    w = out.append
    nch = len(chunks)
    w(f"// Generated: class ({la}{lb}|{lc}{ld}), staged tier: {nch} Phase-1 chunks of <= {cap} accumulators")
    w(f"// (VRR recomputation x{recompute:.2f}), axis rule {rule}, VRR order '{sched}'; {len(g.nodes)} VRR nodes,")
    w(f"// {full} VRR FLOP per primitive quartet unchunked, N_hrr {n_h}, Phase-2 {p2.flops} FLOP, {nslots} buffer")
    w(f"// slots per quartet.")
    w('#include "hgp_device.h"')
    w("")
    w("namespace hgp {")
    w("namespace {")
    w("")
    # ---------------------------------------------------------------- Phase 1 kernel
    w(f"// Phase 1: item (block / {nch}) * {block} + thread, chunk = block % {nch}.")
    w(f"__global__ __launch_bounds__({block}){waves_attr(waves)} void p1_{tag}(P1Args a)")
    w("{")
    w(f"    const int chunk = (int)(blockIdx.x % {nch});")
    w(f"    const int64_t i = (int64_t)(blockIdx.x / {nch}) * {block} + threadIdx.x;")
    w("    if (i >= a.n) return;")
    w("    const int bra = a.idx[i * a.istride], ket = a.idx[i * a.istride + 1];")
    w("    const PairInfo pb = a.pairs[bra], pk = a.pairs[ket];")
    w("    const PairGeo gb = a.geo[bra], gk = a.geo[ket];")
    w("    const PrimPair *__restrict__ prims = a.prims;")
    w("    const double *__restrict__ boys = a.boys;")
    w("    double *const sb = a.scratch;")
    w("    const uint32_t S32 = (uint32_t)a.stride;")
    w("    uint32_t li = (uint32_t)i;")
    w("    switch (chunk) {")
    pos = {v: i for i, v in enumerate(order)}
    for ci, ch in enumerate(chunks):
        sub = subgraph(g, ch)
        corder = sorted(sub, key=lambda v: pos[v])
        Lc = max(g.nodes[v].key[2] for v in sub if g.nodes[v].kind == "base")
        tnames = {t: f"h{tslot[t]}" for t in ch}
        w(f"    case {ci}: {{   // {len(ch)} accumulators, {len(sub)} VRR nodes")
        names = [tnames[t] for t in ch]
        for k in range(0, len(names), 8):
            w("        double " + ", ".join(f"{h} = 0.0" for h in names[k:k + 8]) + ";")
        out.extend(loop_prelude(Lc, "        ", loop))
        out.extend(_vrr_chunk_lines(g, corder, tnames, "            "))
        out.extend(loop_close("        "))
        for t in ch:
            w(f"        sb[{tslot[t]}u * S32 + li] = h{tslot[t]};")
        w("        break;")
        w("    }")
    w("    default:")
    w("        break;")
    w("    }")
    w("}")
    w("")
    # ---------------------------------------------------------------- Phase 2 (device function)
    w(f"// Phase 2, bra stage, for one quartet whose accumulators sit in slots 0..{n_h - 1}: per ket")
    w(f"// component f, the spherical (m n|f) values replace H[:, f] in place.")
    w(f"__device__ __forceinline__ void bra_stage_{tag}(const PairGeo &gb, double *const sb, uint32_t li, const uint32_t S32)")
    w("{")
    w("    const double ABx = gb.abx, ABy = gb.aby, ABz = gb.abz;")
    w("    (void)ABx; (void)ABy; (void)ABz;")
    s2slot = {}
    for (f, a0, a1) in p2.bra_stages:
        ops = p2.ops[a0:a1]
        used = set()
        for op in ops:
            used.update(n for n in _names_in(op) if n in hslot)
        outs = [(mu, nu) for mu in range(na) for nu in range(nb)]
        for (mu, nu) in outs:
            nm = p2.s2[(mu, nu, f)]
            if nm in hslot:
                used.add(nm)
        w(f"    {{   // bra HRR + T(la) T(lb) for ket component {f}")
        for h in sorted(used, key=lambda x: hslot[x]):
            w(f"        const double {h} = sb[{hslot[h]}u * S32 + li];")
        for op in ops:
            w("        " + _op_line(op, {}))
        for (mu, nu) in outs:
            slot = hslot[hname_of[(E[mu * nb + nu], f)]]
            s2slot[(mu, nu, f)] = slot
            w(f"        sb[{slot}u * S32 + li] = {p2.s2[(mu, nu, f)]};")
        w("    }")
        w("    HGP_STAGE(li);")
    w("}")
    w("")
    F = list(levels(lc, lc + ld))

    def ket_stage(mu, nu, a0, a1, sink, ind="    ", after=None):
        """Ket HRR + T(lc) T(ld) for bra functions (mu, nu); sink(lam, sig, name)
        emits the use of each integral while it is still in a register;
        after(names, ind) -> lines that use the stage's integrals together
        (names[(lam, sig)]) before its scope closes."""
        ops = p2.ops[a0:a1]
        w(f"{ind}{{   // ket HRR + T(lc) T(ld) for bra functions ({mu}, {nu})")
        ren = {}
        for k, f in enumerate(F):
            nm = p2.s2[(mu, nu, f)]
            ren[nm] = f"y{k}"
            w(f"{ind}    const double y{k} = sb[{s2slot[(mu, nu, f)]}u * S32 + li];")
        for op in ops:
            w(f"{ind}    " + _op_line(op, ren))
        names = {}
        for lam in range(nc):
            for sig in range(nd):
                nm = p2.out[(mu, nu, lam, sig)]
                names[(lam, sig)] = ren.get(nm, nm)
                if sink is not None:
                    sink(mu, nu, lam, sig, names[(lam, sig)], ind + "    ")
        if after is not None:
            for line in after(names, ind + "    "):
                w(line)
        w(f"{ind}}}")
        w(f"{ind}HGP_STAGE(li);")

    # ---------------------------------------------------------------- Phase 2 + digestion kernel
    # Digestion of (m n|l s) with the 8-fold symmetric Scatter: the ket stages
    # store the integrals, then six contractions stream them back
    #   J'[ab] += 2s sum_ls I D[cd],  J'[cd] += 2s sum_mn I D[ab],
    #   K'[ac] += s sum_ns I D[bd],   K'[bc] += s sum_ms I D[ad],
    #   K'[ad] += s sum_nl I D[bc],   K'[bd] += s sum_ml I D[ac].
    w(f"__global__ __launch_bounds__({block}) void jk_{tag}(JKArgs a)")
    w("{")
    w(f"    const int64_t i = (int64_t)blockIdx.x * {block} + threadIdx.x;")
    w("    if (i >= a.nq) return;")
    w("    double *const sb = a.scratch;")
    w("    const uint32_t S32 = (uint32_t)a.stride;")
    w("    uint32_t li = (uint32_t)i;")
    w("    const double *__restrict__ D = a.D;")
    w("    const int N = a.nbf;")
    w("    const int2 pq = a.quartets[i];")
    w("    const PairInfo pb = a.pairs[pq.x], pk = a.pairs[pq.y];")
    w("    const PairGeo gb = a.geo[pq.x], gk = a.geo[pq.y];")
    w(f"    bra_stage_{tag}(gb, sb, li, S32);")
    w("    const double CDx = gk.abx, CDy = gk.aby, CDz = gk.abz;")
    w("    (void)CDx; (void)CDy; (void)CDz;")
    w("    const int fa = pb.fa, fb = pb.fb, fc = pk.fa, fd = pk.fb;")
    w("    const double s = (pb.same ? 0.5 : 1.0) * (pk.same ? 0.5 : 1.0) * (pq.x == pq.y ? 0.5 : 1.0);")
    w("    const double sj = a.want_j ? 2.0 * s : 0.0, sk = a.want_k ? s : 0.0;")

    def store_sink(mu, nu, lam, sig, name, ind):
        w(f"{ind}sb[{islot(mu, nu, lam, sig)}u * S32 + li] = {name};")

    if jk_digest == "fused":
        # each bra function pair's integrals digested as the ket stage makes them
        fdg = FusedDigest((na, nb, nc, nd), 0, 1, reduce)
        out.extend(fdg.prologue())
        for (mu, nu, a0, a1) in p2.ket_stages:
            if nu == 0:
                out.extend(fdg.outer_begin(mu))
            ket_stage(mu, nu, a0, a1, None,
                      after=lambda names, ind, mu=mu, nu=nu: fdg.slice(mu, nu, lambda r, s_: names[(r, s_)], ind))
            if nu == nb - 1:
                out.extend(fdg.outer_end(mu))
        out.extend(fdg.epilogue())
    else:
        for (mu, nu, a0, a1) in p2.ket_stages:
            ket_stage(mu, nu, a0, a1, store_sink)
        out.extend(slot_digestion(na, nb, nc, nd, lambda mu, nu, lam, sig: f"sb[{islot(mu, nu, lam, sig)}u * S32 + li]",
                                  reduce))
    w("}")
    w("")
    # ---------------------------------------------------------------- Phase 2 + integrals-out kernel
    diag_class = (la, lb) == (lc, ld)
    w(f"__global__ __launch_bounds__({block}) void eri_{tag}(EriArgs a)")
    w("{")
    w(f"    const int64_t i = (int64_t)blockIdx.x * {block} + threadIdx.x;")
    w("    if (i >= a.ntask) return;")
    w("    double *const sb = a.scratch;")
    w("    const uint32_t S32 = (uint32_t)a.stride;")
    w("    uint32_t li = (uint32_t)i;")
    w("    const EriTask t = a.tasks[i];")
    w("    const PairGeo gb = a.geo[t.bra], gk = a.geo[t.ket];")
    w(f"    bra_stage_{tag}(gb, sb, li, S32);")
    w("    const double CDx = gk.abx, CDy = gk.aby, CDz = gk.abz;")
    w("    (void)CDx; (void)CDy; (void)CDz;")
    w("    double *__restrict__ o = a.out + t.off;")
    if diag_class:
        w("    double dmax = 0.0;")

    def eri_sink(mu, nu, lam, sig, name, ind):
        if diag_class and (mu, nu) == (lam, sig):
            w(f"{ind}dmax = fmax(dmax, fabs({name}));")
        w(f"{ind}if (a.mode == 0) o[{mu} * t.s0 + {nu} * t.s1 + {lam} * t.s2 + {sig} * t.s3] = {name};")

    for (mu, nu, a0, a1) in p2.ket_stages:
        ket_stage(mu, nu, a0, a1, eri_sink)
    if diag_class:
        w("    if (a.mode == 1) a.out[i] = sqrt(dmax);")
    w("}")
    w("")
    w("}  // namespace")
    w("")
    w(f"void launch_p1_{tag}(const P1Args &a, hipStream_t s)")
    w("{")
    w(f"    const int64_t blocks = (a.n + {block - 1}) / {block};")
    w(f"    if (blocks > 0) hipLaunchKernelGGL(p1_{tag}, dim3((unsigned)(blocks * {nch})), dim3({block}), 0, s, a);")
    w("}")
    for kind, cnt in (("jk", "nq"), ("eri", "ntask")):
        args = "JKArgs" if kind == "jk" else "EriArgs"
        w(f"void launch_{kind}_{tag}(const {args} &a, hipStream_t s)")
        w("{")
        w(f"    const int64_t blocks = (a.{cnt} + {block - 1}) / {block};")
        w(f"    if (blocks > 0) hipLaunchKernelGGL({kind}_{tag}, dim3((unsigned)blocks), dim3({block}), 0, s, a);")
        w("}")
    w("")
    w("}  // namespace hgp")
    meta = ClassMeta(ls, tag, 1, block, len(g.nodes), full, n_h, pl, sched, p2.flops, nout, rule,
                     scratch_slots=nslots, chunks=len(chunks), recompute=recompute, cap=cap, waves=waves,
                     digest="", reduce=reduce, loop=loop)
    meta.jk_digest = jk_digest
    return "\n".join(out) + "\n", meta


def slot_digestion(na, nb, nc, nd, I, reduce="segmented"):
    """J/K digestion of one quartet whose spherical integrals sit in the slot
    buffer (I(mu, nu, lam, sig) -> C expression of the stored value), with
    the 8-fold symmetric Scatter: six contractions, each streaming the
    integrals back, one output element at a time (a dot product with D
    entries, then one atomic):
      J'[ab] += 2s sum_ls I D[cd],  J'[cd] += 2s sum_mn I D[ab],
      K'[ac] += s sum_ns I D[bd],   K'[bc] += s sum_ms I D[ad],
      K'[ad] += s sum_nl I D[bc],   K'[bd] += s sum_ml I D[ac].
    In scope: s-scaled sj, sk, pq, pk, fa..fd, N, D, li.  reduce='segmented':
    J'[ab], K'[ac] and K'[bc] terms are first summed along the wave's runs of
    lanes with the same target and the run's last lane adds them."""
    out = []
    w = out.append

    def contraction(outer, inner, target, scale, seg=None):
        vals = []
        for k, o in enumerate(outer):
            terms = inner(*o)
            expr = f"{terms[0][0]} * {terms[0][1]}"
            for x, y in terms[1:]:
                expr = f"fma({x}, {y}, {expr})"
            if seg is None:
                w(f"        atomicAdd({target(*o)}, {scale} * ({expr}));")
            else:
                w(f"        const double {seg[2]}{k} = hgp_seg_sum({scale} * ({expr}), {seg[0]});")
                vals.append((f"{seg[2]}{k}", target(*o)))
            w("        HGP_STAGE(li);")
        if seg is not None:
            w(f"        if ({seg[1]}) {{")
            for v, t in vals:
                w(f"            atomicAdd({t}, {v});")
            w("        }")

    segmented = reduce == "segmented"
    w("    if (a.want_j) {")
    if segmented:
        w("        const int seg_ab = hgp_seg_start(pq.x);")
        w("        const bool tail_ab = hgp_seg_tail(pq.x);")
    contraction([(mu, nu) for mu in range(na) for nu in range(nb)],
                lambda mu, nu: [(I(mu, nu, lam, sig), f"D[(int64_t)(fc + {lam}) * N + fd + {sig}]")
                                for lam in range(nc) for sig in range(nd)],
                lambda mu, nu: f"a.J + (int64_t)(fa + {mu}) * N + fb + {nu}", "sj",
                ("seg_ab", "tail_ab", "jr") if segmented else None)
    contraction([(lam, sig) for lam in range(nc) for sig in range(nd)],
                lambda lam, sig: [(I(mu, nu, lam, sig), f"D[(int64_t)(fa + {mu}) * N + fb + {nu}]")
                                  for mu in range(na) for nu in range(nb)],
                lambda lam, sig: f"a.J + (int64_t)(fc + {lam}) * N + fd + {sig}", "sj")
    w("    }")
    w("    if (a.want_k) {")
    if segmented:
        w("        const long long key_ac = ((long long)pq.x << 32) | (unsigned)pk.sh_a;")
        w("        const int seg_ac = hgp_seg_start(key_ac);")
        w("        const bool tail_ac = hgp_seg_tail(key_ac);")
    contraction([(mu, lam) for mu in range(na) for lam in range(nc)],
                lambda mu, lam: [(I(mu, nu, lam, sig), f"D[(int64_t)(fb + {nu}) * N + fd + {sig}]")
                                 for nu in range(nb) for sig in range(nd)],
                lambda mu, lam: f"a.K + (int64_t)(fa + {mu}) * N + fc + {lam}", "sk",
                ("seg_ac", "tail_ac", "kac") if segmented else None)
    contraction([(nu, lam) for nu in range(nb) for lam in range(nc)],
                lambda nu, lam: [(I(mu, nu, lam, sig), f"D[(int64_t)(fa + {mu}) * N + fd + {sig}]")
                                 for mu in range(na) for sig in range(nd)],
                lambda nu, lam: f"a.K + (int64_t)(fb + {nu}) * N + fc + {lam}", "sk",
                ("seg_ac", "tail_ac", "kbc") if segmented else None)
    contraction([(mu, sig) for mu in range(na) for sig in range(nd)],
                lambda mu, sig: [(I(mu, nu, lam, sig), f"D[(int64_t)(fb + {nu}) * N + fc + {lam}]")
                                 for nu in range(nb) for lam in range(nc)],
                lambda mu, sig: f"a.K + (int64_t)(fa + {mu}) * N + fd + {sig}", "sk")
    contraction([(nu, sig) for nu in range(nb) for sig in range(nd)],
                lambda nu, sig: [(I(mu, nu, lam, sig), f"D[(int64_t)(fa + {mu}) * N + fc + {lam}]")
                                 for mu in range(na) for lam in range(nc)],
                lambda nu, sig: f"a.K + (int64_t)(fb + {nu}) * N + fd + {sig}", "sk")
    w("    }")
    return out


# The six contractions of the 8-fold symmetric Scatter (Alg. 2): target index
# pair, density index pair, scale, matrix, segmented-reduction key.  Index 0..3
# = mu, nu, lam, sig of (mu nu|lam sig); their first functions fa, fb, fc, fd.
_CONTRACTIONS = (
    ("jab", (0, 1), (2, 3), "sj", "J", "ab"),
    ("jcd", (2, 3), (0, 1), "sj", "J", None),
    ("kac", (0, 2), (1, 3), "sk", "K", "ac"),
    ("kbc", (1, 2), (0, 3), "sk", "K", "ac"),
    ("kad", (0, 3), (1, 2), "sk", "K", None),
    ("kbd", (1, 3), (0, 2), "sk", "K", None),
)
_FOFF = ("fa", "fb", "fc", "fd")


class FusedDigest:
    """J/K digestion that takes each integral once, while it is still in a
    register, instead of storing the integrals and streaming them back six
    times.  Phase 2 produces the integrals in slices: slice (p, q) over an
    outer index P and an inner index Q holds the values for every (r, s) of
    the other two indices.  Per contraction, an output element that lies in
    {P, Q} is complete within one slice (one dot product, one atomic); one that
    lies in {R, S}, or pairs Q with R or S, collects over every slice (its
    accumulators live across the whole loop); one that pairs P with R or S
    collects over the inner loop (accumulators reset per outer index).  The
    J'[ab], K'[ac] and K'[bc] outputs keep the wave's segmented reductions.
    sizes = (na, nb, nc, nd); outer, inner = P, Q."""

    def __init__(self, sizes, outer, inner, reduce="segmented"):
        self.n = sizes
        self.P, self.Q = outer, inner
        self.R, self.S = [k for k in range(4) if k not in (outer, inner)]
        self.seg = reduce == "segmented"
        self.kind = {}
        for name, tgt, dd, sc, mat, key in _CONTRACTIONS:
            st = set(tgt)
            if st == {self.P, self.Q}:
                self.kind[name] = "slice"
            elif self.P in st:
                self.kind[name] = "outer"
            else:
                self.kind[name] = "all"

    def _elems(self, tgt):
        return [(i, j) for i in range(self.n[tgt[0]]) for j in range(self.n[tgt[1]])]

    def _acc(self, name, i, j):
        return f"{name}_{i}_{j}"

    def _guard(self, mat):
        return "a.want_j" if mat == "J" else "a.want_k"

    def _emit(self, name, tgt, sc, mat, key, elems, expr, ind):
        """Add scale * expr(i, j) to the matrix at each element."""
        lines = []
        ptr = lambda i, j: f"a.{mat} + (int64_t)({_FOFF[tgt[0]]} + {i}) * N + {_FOFF[tgt[1]]} + {j}"
        if key is not None and self.seg:
            vals = []
            for k, (i, j) in enumerate(elems):
                lines.append(f"{ind}const double {name}r{k} = hgp_seg_sum({sc} * ({expr(i, j)}), seg_{key});")
                vals.append((f"{name}r{k}", ptr(i, j)))
            lines.append(f"{ind}if (tail_{key}) {{")
            for v, p in vals:
                lines.append(f"{ind}    atomicAdd({p}, {v});")
            lines.append(f"{ind}}}")
        else:
            for (i, j) in elems:
                lines.append(f"{ind}atomicAdd({ptr(i, j)}, {sc} * ({expr(i, j)}));")
        return lines

    def prologue(self, ind="    "):
        """Segment keys and the accumulators that live across the whole loop."""
        lines = []
        if self.seg:
            lines.append(f"{ind}const int seg_ab = hgp_seg_start(pq.x);")
            lines.append(f"{ind}const bool tail_ab = hgp_seg_tail(pq.x);")
            lines.append(f"{ind}const long long key_ac = ((long long)pq.x << 32) | (unsigned)pk.sh_a;")
            lines.append(f"{ind}const int seg_ac = hgp_seg_start(key_ac);")
            lines.append(f"{ind}const bool tail_ac = hgp_seg_tail(key_ac);")
            lines.append(f"{ind}(void)seg_ab; (void)tail_ab; (void)seg_ac; (void)tail_ac;")
        for name, tgt, dd, sc, mat, key in _CONTRACTIONS:
            if self.kind[name] == "all":
                accs = [self._acc(name, i, j) for (i, j) in self._elems(tgt)]
                for k in range(0, len(accs), 8):
                    lines.append(f"{ind}double " + ", ".join(f"{x} = 0.0" for x in accs[k:k + 8]) + ";")
        return lines

    def outer_begin(self, p, ind="    "):
        """Opens the outer iteration's scope (closed by outer_end)."""
        lines = [f"{ind}{{   // outer index {p}"]
        for name, tgt, dd, sc, mat, key in _CONTRACTIONS:
            if self.kind[name] == "outer":
                other = tgt[1] if tgt[0] == self.P else tgt[0]
                accs = [f"{name}_o{r}" for r in range(self.n[other])]
                lines.append(f"{ind}double " + ", ".join(f"{x} = 0.0" for x in accs) + ";")
        return lines

    def slice(self, p, q, val, ind="    "):
        """One slice: val(r, s) names the integral with index P = p, Q = q,
        R = r, S = s."""
        lines = []
        n = self.n
        for name, tgt, dd, sc, mat, key in _CONTRACTIONS:
            kind = self.kind[name]
            # the terms of every output element this slice touches
            terms = {}
            for r in range(n[self.R]):
                for s_ in range(n[self.S]):
                    idx = [0] * 4
                    idx[self.P], idx[self.Q], idx[self.R], idx[self.S] = p, q, r, s_
                    el = (idx[tgt[0]], idx[tgt[1]])
                    d = f"D[(int64_t)({_FOFF[dd[0]]} + {idx[dd[0]]}) * N + {_FOFF[dd[1]]} + {idx[dd[1]]}]"
                    terms.setdefault(el, []).append((val(r, s_), d))
            body = []
            if kind == "slice":
                (el, tl), = terms.items()
                expr = f"{tl[0][0]} * {tl[0][1]}"
                for x, y in tl[1:]:
                    expr = f"fma({x}, {y}, {expr})"
                body.extend(self._emit(name, tgt, sc, mat, key, [el], lambda i, j, e=expr: e, ind + "    "))
            else:
                for el, tl in terms.items():
                    if kind == "outer":
                        other = el[1] if tgt[0] == self.P else el[0]
                        acc = f"{name}_o{other}"
                    else:
                        acc = self._acc(name, *el)
                    expr = acc
                    for x, y in tl:
                        expr = f"fma({x}, {y}, {expr})"
                    body.append(f"{ind}    {acc} = {expr};")
            lines.append(f"{ind}if ({self._guard(mat)}) {{")
            lines.extend(body)
            lines.append(f"{ind}}}")
        lines.append(f"{ind}HGP_STAGE(li);")
        return lines

    def outer_end(self, p, ind="    "):
        lines = []
        for name, tgt, dd, sc, mat, key in _CONTRACTIONS:
            if self.kind[name] != "outer":
                continue
            if tgt[0] == self.P:
                elems = [(p, r) for r in range(self.n[tgt[1]])]
                expr = lambda i, j, nm=name: f"{nm}_o{j}"
            else:
                elems = [(r, p) for r in range(self.n[tgt[0]])]
                expr = lambda i, j, nm=name: f"{nm}_o{i}"
            lines.append(f"{ind}if ({self._guard(mat)}) {{")
            lines.extend(self._emit(name, tgt, sc, mat, key, elems, expr, ind + "    "))
            lines.append(f"{ind}}}")
        lines.append(f"{ind}}}")
        lines.append(f"{ind}HGP_STAGE(li);")
        return lines

    def epilogue(self, ind="    "):
        lines = []
        for name, tgt, dd, sc, mat, key in _CONTRACTIONS:
            if self.kind[name] != "all":
                continue
            lines.append(f"{ind}if ({self._guard(mat)}) {{")
            lines.extend(self._emit(name, tgt, sc, mat, key, self._elems(tgt),
                                    lambda i, j, nm=name: self._acc(nm, i, j), ind + "    "))
            lines.append(f"{ind}}}")
        return lines
