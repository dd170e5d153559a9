"""HIP source emission for one canonical quartet class (la lb|lc ld).

Each class becomes one translation unit holding
  - an inlined quartet evaluator: the primitive loops with the Boys function
    and the straight-line VRR in the chosen order, the contraction into the
    accumulator bank H, then the Phase-2 HRR + stepwise spherical transform
    (Alg. 2's structure, Sec. III-C.1);
  - a J/K kernel, one lane per unique shell quartet, with the digestion into
    the unsymmetrised J', K' fused after Phase 2 (FP64 global atomics);
  - an integrals-out kernel (blocks written with caller strides, or the
    Schwarz factor of a diagonal quartet);
  - host launchers with C linkage for the runtime's class table.
"""
from __future__ import annotations

import dataclasses

from . import phase2 as p2mod
from . import vrr as vrrmod
from .cart import comps, levels
from .sph import tmatrix

XYZ = "xyz"


@dataclasses.dataclass
class ClassMeta:
    ls: tuple
    tag: str
    tier: int
    block: int
    vrr_nodes: int
    vrr_flops: int
    n_hrr: int
    peak_live: int
    scheduler: str
    p2_flops: int
    n_out: int
    rule: str
    scratch_slots: int = 0
    chunks: int = 1
    recompute: float = 1.0
    cap: int = 0
    waves: int = 0
    digest: str = "loads_first"
    reduce: str = "segmented"
    loop: str = "late"
    mixed: bool = False
    max_batch: int = 0      # quartets per batch at most (0: no limit beyond the buffer)


def tag_of(ls):
    return "".join(str(x) for x in ls)


def _fmt(c: float) -> str:
    r = repr(float(c))
    return r if ("." in r or "e" in r) else r + ".0"


def _vrr_lines(g, order, hnames, indent, f32=False):
    """Straight-line VRR in `order`; targets are added to their accumulators.
    f32: single precision (coefficients carry an 'f' suffix, base values come
    from Bf[m], set from the FP64 prefactor and Boys values)."""
    lines = []
    tpos = {tid: k for k, tid in enumerate(g.target_ids)}
    used = set()
    ty, fma_, sfx, one = ("float", "fmaf", "f", "f") if f32 else ("double", "fma", "", "")
    for v in order:
        nd = g.nodes[v]
        name = f"v{v}"
        if nd.kind == "base":
            expr = f"Bf[{nd.key[2]}]" if f32 else f"base * F[{nd.key[2]}]"
        else:
            p1, p2, p3, p4, p5 = nd.parents
            ax = XYZ[nd.axis]
            if nd.kind == "bra":
                c1, c2, o2, rr = f"PA{ax}", f"WP{ax}", "o2z", "rz"
            else:
                c1, c2, o2, rr = f"QC{ax}", f"WQ{ax}", "o2e", "re"
            used.update([c1, c2])
            expr = f"{fma_}({c1}{sfx}, v{p1}, {c2}{sfx} * v{p2})"
            if nd.k_same:
                k = "" if nd.k_same == 1 else f"{nd.k_same}.0{one} * "
                expr = f"{fma_}({k}{o2}{sfx}, {fma_}(-{rr}{sfx}, v{p4}, v{p3}), {expr})"
                used.update([o2, rr])
            if nd.k_cross:
                k = "" if nd.k_cross == 1 else f"{nd.k_cross}.0{one} * "
                expr = f"{fma_}({k}o2ze{sfx}, v{p5}, {expr})"
                used.add("o2ze")
        lines.append(f"{indent}const {ty} {name} = {expr};")
        if v in tpos:
            lines.append(f"{indent}{hnames[tpos[v]]} += {name};")
    return lines, used


def _p2_lines(p2, indent, f32=False):
    lines = []
    ty, fma_ = ("float", "fmaf") if f32 else ("double", "fma")
    fmt = (lambda c: _fmt(c) + "f") if f32 else _fmt
    for op in p2.ops:
        if op[1] == "hrr":
            d, _, hi, lo, coef = op
            lines.append(f"{indent}const {ty} {d} = {fma_}({coef}, {lo}, {hi});")
        else:
            d, _, terms = op
            expr = f"{fmt(terms[0][0])} * {terms[0][1]}"
            for c, s in terms[1:]:
                expr = f"{fma_}({fmt(c)}, {s}, {expr})"
            lines.append(f"{indent}const {ty} {d} = {expr};")
    return lines


def loop_prelude(L, ind, style="late", weights=False, seg=False):
    """The primitive-quartet loop up to the VRR (Alg. 2's GaussianPairs and
    Boys steps), flattened over bra x ket primitive pairs.
    style 'prefetch': the next iteration's pair records are loaded at the top
    of the iteration into a second set of registers (copied over at the end).
    style 'late': they are loaded into the same registers as soon as the
    current records have been turned into the derived quantities, so no
    second set and no copies are needed; the loads still have the Boys step
    and the whole VRR to arrive.
    weights ('late' only): the current primitive quartet's 2 alpha, 2 beta
    (bra pair's exponents) and 2 gamma (ket pair's first exponent) as wa, wb,
    wg, the weights of first-derivative integrals.
    seg ('late' only): the loop runs segment s of nseg (both in scope) of the
    flattened primitive quartets, t in [ntot s / nseg, ntot (s + 1) / nseg)."""
    i2 = ind + "    "
    head = [
        f"{ind}const double Ax = gb.ax, Ay = gb.ay, Az = gb.az;",
        f"{ind}const double Cx = gk.ax, Cy = gk.ay, Cz = gk.az;",
        f"{ind}const PrimPair *__restrict__ pbp = prims + pb.prim_off;",
        f"{ind}const PrimPair *__restrict__ pkp = prims + pk.prim_off;",
        f"{ind}const int nkp = pk.nprim, ntot = pb.nprim * pk.nprim;",
    ]
    derived = [
        f"{i2}const double PAx = Px - Ax, PAy = Py - Ay, PAz = Pz - Az;",
        f"{i2}const double QCx = Qx - Cx, QCy = Qy - Cy, QCz = Qz - Cz;",
        f"{i2}const double PQx = Px - Qx, PQy = Py - Qy, PQz = Pz - Qz;",
        f"{i2}const double ze = zeta + eta;",
        f"{i2}const double ize = hgp_rcp(ze);",
        f"{i2}const double rz = eta * ize, re = zeta * ize, o2ze = 0.5 * ize;",
        f"{i2}const double T = zeta * rz * (PQx * PQx + PQy * PQy + PQz * PQz);",
        f"{i2}const double base = Kb * Kk * hgp_rsqrt(ze);",
    ]
    tail = [
        f"{i2}double F[{L + 1}];",
        f"{i2}boys_fm<{L}>(T, boys, F);",
        f"{i2}const double WPx = -rz * PQx, WPy = -rz * PQy, WPz = -rz * PQz;",
        f"{i2}const double WQx = re * PQx, WQy = re * PQy, WQz = re * PQz;",
        f"{i2}(void)o2z; (void)o2e; (void)o2ze; (void)PAx; (void)PAy; (void)PAz; (void)QCx; (void)QCy; (void)QCz;",
        f"{i2}(void)WPx; (void)WPy; (void)WPz; (void)WQx; (void)WQy; (void)WQz; (void)re;",
    ]
    if style == "prefetch":
        return head + [
            f"{ind}double nzeta = pbp[0].zeta, no2z = pbp[0].o2z, nPx = pbp[0].px, nPy = pbp[0].py, nPz = pbp[0].pz, nKb = pbp[0].k;",
            f"{ind}double neta = pkp[0].zeta, no2e = pkp[0].o2z, nQx = pkp[0].px, nQy = pkp[0].py, nQz = pkp[0].pz, nKk = pkp[0].k;",
            f"{ind}int ip = 0, jp = 0;",
            f"{ind}for (int t = 0; t < ntot; ++t) {{",
            f"{i2}const double zeta = nzeta, o2z = no2z, Px = nPx, Py = nPy, Pz = nPz, Kb = nKb;",
            f"{i2}const double eta = neta, o2e = no2e, Qx = nQx, Qy = nQy, Qz = nQz, Kk = nKk;",
            f"{i2}if (++jp == nkp) {{ jp = 0; ++ip; }}",
            f"{i2}if (t + 1 < ntot) {{",
            f"{i2}    const PrimPair *b = pbp + ip, *k = pkp + jp;",
            f"{i2}    nzeta = b->zeta; no2z = b->o2z; nPx = b->px; nPy = b->py; nPz = b->pz; nKb = b->k;",
            f"{i2}    neta = k->zeta; no2e = k->o2z; nQx = k->px; nQy = k->py; nQz = k->pz; nKk = k->k;",
            f"{i2}}}",
        ] + derived + tail
    if style != "late":
        raise ValueError(f"unknown loop style {style!r}")
    r0b, r0k, t0 = ("pbp[0]", "pkp[0]", "0")
    seg_lines = []
    if seg:
        seg_lines = [f"{ind}const int t_lo = (int)(((int64_t)ntot * s) / nseg), t_hi = (int)(((int64_t)ntot * (s + 1)) / nseg);",
                     f"{ind}const int ip0 = t_lo / nkp, jp0 = t_lo - ip0 * nkp;      // t_lo < ntot: both in range"]
        r0b, r0k, t0 = ("pbp[ip0]", "pkp[jp0]", "t_lo")
    w_init = [f"{ind}double rea = {r0b}.ea, reb = {r0b}.eb, rga = {r0k}.ea;"] if weights else []
    w_cur = [f"{i2}const double wa = 2.0 * rea, wb = 2.0 * reb, wg = 2.0 * rga;"] if weights else []
    w_next = [f"{i2}    rea = b->ea; reb = b->eb; rga = k->ea;"] if weights else []
    ij = [f"{ind}int ip = ip0, jp = jp0;"] if seg else [f"{ind}int ip = 0, jp = 0;"]
    return head + [
        f"{ind}const int nbm1 = pb.nprim - 1;",
    ] + seg_lines + [
        f"{ind}double rzeta = {r0b}.zeta, ro2z = {r0b}.o2z, rPx = {r0b}.px, rPy = {r0b}.py, rPz = {r0b}.pz, rKb = {r0b}.k;",
        f"{ind}double reta = {r0k}.zeta, ro2e = {r0k}.o2z, rQx = {r0k}.px, rQy = {r0k}.py, rQz = {r0k}.pz, rKk = {r0k}.k;",
    ] + w_init + ij + [
        f"{ind}for (int t = {t0}; t < {'t_hi' if seg else 'ntot'}; ++t) {{",
        f"{i2}const double zeta = rzeta, o2z = ro2z, Px = rPx, Py = rPy, Pz = rPz, Kb = rKb;",
        f"{i2}const double eta = reta, o2e = ro2e, Qx = rQx, Qy = rQy, Qz = rQz, Kk = rKk;",
    ] + w_cur + derived + [
        # the records of iteration t + 1 (clamped in range on the last iteration)
        f"{i2}if (++jp == nkp) {{ jp = 0; ++ip; }}",
        f"{i2}{{",
        f"{i2}    const PrimPair *b = pbp + min(ip, nbm1), *k = pkp + jp;",
        f"{i2}    rzeta = b->zeta; ro2z = b->o2z; rPx = b->px; rPy = b->py; rPz = b->pz; rKb = b->k;",
        f"{i2}    reta = k->zeta; ro2e = k->o2z; rQx = k->px; rQy = k->py; rQz = k->pz; rKk = k->k;",
    ] + w_next + [
        f"{i2}}}",
    ] + tail


def loop_close(ind):
    return [f"{ind}}}"]


def waves_attr(waves):
    return f" __attribute__((amdgpu_waves_per_eu({waves}, {waves})))" if waves else ""


def _dot(terms):
    expr = f"{terms[0][0]} * {terms[0][1]}"
    for x, y in terms[1:]:
        expr = f"fma({x}, {y}, {expr})"
    return expr


def digest_lines(na, nb, nc, nd, I, J, K, digest="loads_first", reduce="segmented", ind="    "):
    """J/K digestion of one unique quartet's spherical block I(mu, nu, lam, sig)
    (a C expression per integral) into the unsymmetrised J', K' with the
    degeneracy factor s already in scope (pq, pk, fa, fb, fc, fd, N, D too):
      J'[ab] += 2s sum_cd I D_cd,  J'[cd] += 2s sum_ab I D_ab,
      K'[ac] += s sum_bd I D_bd,   K'[bc] += s sum_ad I D_ad,
      K'[ad] += s sum_bc I D_bc,   K'[bd] += s sum_ac I D_ac.
    digest = 'loads_first' reads every D element the quartet needs before the
    first atomic: a GFX9 wave waits on one in-order counter for loads and
    atomics alike, so a D load issued after an atomic would also wait for that
    atomic's round trip to memory.  'interleaved' loads each D block just
    before its contraction.
    reduce: 'segmented' adds the J'[ab] terms along runs of lanes with the
    same bra pair and the K'[ac], K'[bc] terms along runs with the same bra
    pair and ket shell c (each lane's term carries its own degeneracy
    factor); the run's last lane issues the atomic.  'uniform' does this for
    J'[ab] only and only when the whole wave holds one bra pair.  'none':
    one atomic per lane and element."""
    out = []
    w = out.append
    dblocks = {"cd": ("fc", "fd", nc, nd), "ab": ("fa", "fb", na, nb), "bd": ("fb", "fd", nb, nd),
               "ad": ("fa", "fd", na, nd), "bc": ("fb", "fc", nb, nc), "ac": ("fa", "fc", na, nc)}

    def loads(nm, i2=ind + "    "):
        r0, c0, nr, ncol = dblocks[nm]
        for i in range(nr):
            for j in range(ncol):
                w(f"{i2}const double d{nm}_{i}_{j} = D[({r0} + {i}) * N + {c0} + {j}];")

    def jab_terms(mu, nu):
        return _dot([(I(mu, nu, lam, sig), f"dcd_{lam}_{sig}") for lam in range(nc) for sig in range(nd)])

    def jab_atomics(i2):
        for mu in range(na):
            for nu in range(nb):
                w(f"{i2}atomicAdd({J} + (fa + {mu}) * N + fb + {nu}, s2 * ({jab_terms(mu, nu)}));")

    def jcd_atomics(i2):
        for lam in range(nc):
            for sig in range(nd):
                e = _dot([(I(mu, nu, lam, sig), f"dab_{mu}_{nu}") for mu in range(na) for nu in range(nb)])
                w(f"{i2}atomicAdd({J} + (fc + {lam}) * N + fd + {sig}, s2 * ({e}));")

    def seg_block(i2, outer, terms, target, scale, start, tail, nm):
        """Values summed along runs (start lane in `start`), each added by the run's
        last lane right away, so that no more than one sum is live at a time."""
        for k, o in enumerate(outer):
            w(f"{i2}{{ const double {nm} = hgp_seg_sum({scale} * ({_dot(terms(*o))}), {start}); "
              f"if ({tail}) atomicAdd({target(*o)}, {nm}); }}")

    def plain_block(i2, outer, terms, target, scale):
        for o in outer:
            w(f"{i2}atomicAdd({target(*o)}, {scale} * ({_dot(terms(*o))}));")

    kac = ([(mu, lam) for mu in range(na) for lam in range(nc)],
           lambda mu, lam: [(I(mu, nu, lam, sig), f"dbd_{nu}_{sig}") for nu in range(nb) for sig in range(nd)],
           lambda mu, lam: f"{K} + (fa + {mu}) * N + fc + {lam}")
    kbc = ([(nu, lam) for nu in range(nb) for lam in range(nc)],
           lambda nu, lam: [(I(mu, nu, lam, sig), f"dad_{mu}_{sig}") for mu in range(na) for sig in range(nd)],
           lambda nu, lam: f"{K} + (fb + {nu}) * N + fc + {lam}")
    kad = ([(mu, sig) for mu in range(na) for sig in range(nd)],
           lambda mu, sig: [(I(mu, nu, lam, sig), f"dbc_{nu}_{lam}") for nu in range(nb) for lam in range(nc)],
           lambda mu, sig: f"{K} + (fa + {mu}) * N + fd + {sig}")
    kbd = ([(nu, sig) for nu in range(nb) for sig in range(nd)],
           lambda nu, sig: [(I(mu, nu, lam, sig), f"dac_{mu}_{lam}") for mu in range(na) for lam in range(nc)],
           lambda nu, sig: f"{K} + (fb + {nu}) * N + fd + {sig}")
    jab = ([(mu, nu) for mu in range(na) for nu in range(nb)],
           lambda mu, nu: [(I(mu, nu, lam, sig), f"dcd_{lam}_{sig}") for lam in range(nc) for sig in range(nd)],
           lambda mu, nu: f"{J} + (fa + {mu}) * N + fb + {nu}")

    def jab_block(i2):
        if reduce == "segmented":
            w(f"{i2}const int seg_ab = hgp_seg_start(pq.x);")
            w(f"{i2}const bool tail_ab = hgp_seg_tail(pq.x);")
            seg_block(i2, *jab, "s2", "seg_ab", "tail_ab", "jr")
        elif reduce == "uniform":
            # the bra pair is wave-uniform when every lane is active and holds the first lane's bra
            w(f"{i2}if (__builtin_amdgcn_read_exec() == ~0ull && hgp_wave_all(pq.x == __builtin_amdgcn_readfirstlane(pq.x))) {{")
            for mu in range(na):
                for nu in range(nb):
                    w(f"{i2}    const double jr_{mu}_{nu} = hgp_wave_sum(s2 * ({jab_terms(mu, nu)}));")
            w(f"{i2}    if (__lane_id() == 0) {{")
            for mu in range(na):
                for nu in range(nb):
                    w(f"{i2}        atomicAdd({J} + (fa + {mu}) * N + fb + {nu}, jr_{mu}_{nu});")
            w(f"{i2}    }}")
            w(f"{i2}}} else {{")
            jab_atomics(i2 + "    ")
            w(f"{i2}}}")
        else:
            jab_atomics(i2)

    def k_block(i2):
        if reduce == "segmented":
            w(f"{i2}const long long key_ac = ((long long)pq.x << 32) | (unsigned)pk.sh_a;")
            w(f"{i2}const int seg_ac = hgp_seg_start(key_ac);")
            w(f"{i2}const bool tail_ac = hgp_seg_tail(key_ac);")
            seg_block(i2, *kac, "s", "seg_ac", "tail_ac", "kac")
            seg_block(i2, *kbc, "s", "seg_ac", "tail_ac", "kbc")
        else:
            plain_block(i2, *kac, "s")
            plain_block(i2, *kbc, "s")
        plain_block(i2, *kad, "s")
        plain_block(i2, *kbd, "s")

    if digest not in ("loads_first", "interleaved"):
        raise ValueError(f"unknown digest style {digest!r}")
    w(f"{ind}if (a.want_j) {{")
    w(f"{ind}    const double s2 = 2.0 * s;")
    loads("cd")
    if digest == "loads_first":
        loads("ab")
    jab_block(ind + "    ")
    if digest == "interleaved":
        loads("ab")
    jcd_atomics(ind + "    ")
    w(f"{ind}}}")
    w(f"{ind}if (a.want_k) {{")
    for nm in ("bd", "ad", "bc", "ac"):
        loads(nm)
    k_block(ind + "    ")
    w(f"{ind}}}")
    return out


def _quartet_fn(name, L, g, order, hnames, p2, loop, f32, na, nb, nc, nd):
    """The device function computing one contracted quartet's spherical
    block into double I[]: primitive loop (pair combination and Boys always
    in FP64), VRR + accumulation, Phase 2.  f32: the VRR and the contraction
    sums run in single precision; the accumulators are widened to FP64
    before Phase 2, whose horizontal recurrence can cancel heavily between
    large intermediates and would amplify single-precision rounding."""
    out = []
    w = out.append
    acc = [h + "f" for h in hnames] if f32 else hnames
    ty = "float" if f32 else "double"
    zero = "0.0f" if f32 else "0.0"
    vlines, _ = _vrr_lines(g, order, acc, "        ", f32)
    w(f"__device__ __forceinline__ void {name}(const PairInfo &pb, const PairGeo &gb, const PairInfo &pk,")
    w(f"                                              const PairGeo &gk, const PrimPair *__restrict__ prims,")
    w(f"                                              const double *__restrict__ boys, double *__restrict__ I)")
    w("{")
    for k in range(0, len(acc), 8):
        w(f"    {ty} " + ", ".join(f"{h} = {zero}" for h in acc[k:k + 8]) + ";")
    out.extend(loop_prelude(L, "    ", loop))
    if f32:
        i2 = "        "
        w(f"{i2}float Bf[{L + 1}];")
        w(f"{i2}for (int m = 0; m <= {L}; ++m) Bf[m] = (float)(base * F[m]);")
        for nm in ("PA", "QC", "WP", "WQ"):
            w(f"{i2}const float " + ", ".join(f"{nm}{a}f = (float){nm}{a}" for a in "xyz") + ";")
        w(f"{i2}const float o2zf = (float)o2z, o2ef = (float)o2e, o2zef = (float)o2ze, rzf = (float)rz, ref = (float)re;")
        w(f"{i2}(void)PAxf; (void)PAyf; (void)PAzf; (void)QCxf; (void)QCyf; (void)QCzf; (void)WPxf; (void)WPyf;")
        w(f"{i2}(void)WPzf; (void)WQxf; (void)WQyf; (void)WQzf; (void)o2zf; (void)o2ef; (void)o2zef; (void)rzf; (void)ref;")
    out.extend(vlines)
    out.extend(loop_close("    "))
    if f32:
        for k in range(0, len(hnames), 8):
            w("    const double " + ", ".join(f"{h} = (double){h}f" for h in hnames[k:k + 8]) + ";")
    w("    const double ABx = gb.abx, ABy = gb.aby, ABz = gb.abz;")
    w("    const double CDx = gk.abx, CDy = gk.aby, CDz = gk.abz;")
    w("    (void)ABx; (void)ABy; (void)ABz; (void)CDx; (void)CDy; (void)CDz;")
    out.extend(_p2_lines(p2, "    "))
    for mu in range(na):
        for nu in range(nb):
            for lam in range(nc):
                for sig in range(nd):
                    k = ((mu * nb + nu) * nc + lam) * nd + sig
                    w(f"    I[{k}] = {p2.out[(mu, nu, lam, sig)]};")
    w("}")
    w("")
    return out


def emit_class(la, lb, lc, ld, rule="ket_zyx", block=256, schedulers=None, waves=0, digest="loads_first",
               reduce="segmented", loop="late", mixed=True):
    ls = (la, lb, lc, ld)
    tag = tag_of(ls)
    L = sum(ls)
    g = vrrmod.VRRGraph(la, lb, lc, ld, rule=rule)
    sched, pl, order = vrrmod.best_order(g) if schedulers is None else vrrmod.best_order(g, schedulers)
    hnames = [f"h{k}" for k in range(len(g.targets))]
    hmap = {t: hnames[k] for k, t in enumerate(g.targets)}
    p2 = p2mod.Phase2(la, lb, lc, ld, hname=lambda e, f: hmap[(e, f)])
    na, nb, nc, nd = (len(tmatrix(l)) for l in ls)
    nout = na * nb * nc * nd
    I = {k: v for k, v in p2.out.items()}

    out = []
    w = out.append
    w(f"// Generated: class ({la}{lb}|{lc}{ld}), axis rule {rule}, VRR order '{sched}' (PeakLive {pl}),")
    w(f"// {len(g.nodes)} VRR nodes, {g.flops()} VRR FLOP per primitive quartet, N_hrr {len(g.targets)},")
    w(f"// Phase-2 {p2.flops} FLOP per contracted quartet, {nout} spherical integrals.")
    w('#include "hgp_device.h"')
    w("")
    w("namespace hgp {")
    w("namespace {")
    w("")
    out.extend(_quartet_fn(f"quartet_{tag}", L, g, order, hnames, p2, loop, False, na, nb, nc, nd))
    if mixed:
        out.extend(_quartet_fn(f"quartet32_{tag}", L, g, order, hnames, p2, loop, True, na, nb, nc, nd))
    # ---------------------------------------------------------------- J/K kernel
    def idx(mu, nu, lam, sig):
        return ((mu * nb + nu) * nc + lam) * nd + sig

    # jk_: FP64 throughout; jk32_: the same with the VRR and contraction in
    # FP32 (mixed plans route quartets with a small Schwarz bound here);
    # Phase 2 and digestion in FP64
    for kname, qname, ity in [(f"jk_{tag}", f"quartet_{tag}", "double")] + \
            ([(f"jk32_{tag}", f"quartet32_{tag}", "double")] if mixed else []):
        w(f"__global__ __launch_bounds__({block}){waves_attr(waves)} void {kname}(JKArgs a)")
        w("{")
        w(f"    const int64_t q = (int64_t)blockIdx.x * {block} + threadIdx.x;")
        w("    if (q >= a.nq) return;")
        w("    const int2 pq = a.quartets[q];")
        w("    const PairInfo pb = a.pairs[pq.x], pk = a.pairs[pq.y];")
        w("    const PairGeo gb = a.geo[pq.x], gk = a.geo[pq.y];")
        w(f"    {ity} I[{nout}];")
        w(f"    {qname}(pb, gb, pk, gk, a.prims, a.boys, I);")
        w("    const double *__restrict__ D = a.D;")
        w("    const int N = a.nbf;")
        w("    const int fa = pb.fa, fb = pb.fb, fc = pk.fa, fd = pk.fb;")
        w("    const double s = (pb.same ? 0.5 : 1.0) * (pk.same ? 0.5 : 1.0) * (pq.x == pq.y ? 0.5 : 1.0);")
        cast = "" if ity == "double" else "(double)"
        out.extend(digest_lines(na, nb, nc, nd, lambda mu, nu, lam, sig: f"{cast}I[{idx(mu, nu, lam, sig)}]",
                                "a.J", "a.K", digest, reduce))
        w("}")
        w("")
    # ---------------------------------------------------------------- integrals-out kernels
    # eri_: FP64; eri32_ (mixed precision): the VRR and contraction in FP32
    if mixed:
        w(f"__global__ __launch_bounds__({block}){waves_attr(waves)} void eri32_{tag}(EriArgs a)")
        w("{")
        w(f"    const int64_t q = (int64_t)blockIdx.x * {block} + threadIdx.x;")
        w("    if (q >= a.ntask) return;")
        w("    const EriTask t = a.tasks[q];")
        w("    const PairInfo pb = a.pairs[t.bra], pk = a.pairs[t.ket];")
        w("    const PairGeo gb = a.geo[t.bra], gk = a.geo[t.ket];")
        w(f"    double I[{nout}];")
        w(f"    quartet32_{tag}(pb, gb, pk, gk, a.prims, a.boys, I);")
        w("    double *__restrict__ o = a.out + t.off;")
        for mu in range(na):
            for nu in range(nb):
                for lam in range(nc):
                    for sig in range(nd):
                        w(f"    o[{mu} * t.s0 + {nu} * t.s1 + {lam} * t.s2 + {sig} * t.s3] = I[{idx(mu, nu, lam, sig)}];")
        w("}")
        w("")
    diag_class = (la, lb) == (lc, ld)
    w(f"__global__ __launch_bounds__({block}){waves_attr(waves)} void eri_{tag}(EriArgs a)")
    w("{")
    w(f"    const int64_t q = (int64_t)blockIdx.x * {block} + threadIdx.x;")
    w("    if (q >= a.ntask) return;")
    w("    const EriTask t = a.tasks[q];")
    w("    const PairInfo pb = a.pairs[t.bra], pk = a.pairs[t.ket];")
    w("    const PairGeo gb = a.geo[t.bra], gk = a.geo[t.ket];")
    w(f"    double I[{nout}];")
    w(f"    quartet_{tag}(pb, gb, pk, gk, a.prims, a.boys, I);")
    if diag_class:
        w("    if (a.mode == 1) {")
        w("        double m = 0.0;")
        for mu in range(na):
            for nu in range(nb):
                w(f"        m = fmax(m, fabs(I[{idx(mu, nu, mu, nu)}]));")
        w("        a.out[q] = sqrt(m);")
        w("        return;")
        w("    }")
    w("    double *__restrict__ o = a.out + t.off;")
    for mu in range(na):
        for nu in range(nb):
            for lam in range(nc):
                for sig in range(nd):
                    w(f"    o[{mu} * t.s0 + {nu} * t.s1 + {lam} * t.s2 + {sig} * t.s3] = I[{idx(mu, nu, lam, sig)}];")
    w("}")
    w("")
    w("}  // namespace")
    w("")
    w(f"void launch_jk_{tag}(const JKArgs &a, hipStream_t s)")
    w("{")
    w(f"    hipLaunchKernelGGL(jk_{tag}, dim3((unsigned)((a.nq + {block - 1}) / {block})), dim3({block}), 0, s, a);")
    w("}")
    w(f"void launch_eri_{tag}(const EriArgs &a, hipStream_t s)")
    w("{")
    w(f"    hipLaunchKernelGGL(eri_{tag}, dim3((unsigned)((a.ntask + {block - 1}) / {block})), dim3({block}), 0, s, a);")
    w("}")
    if mixed:
        w(f"void launch_jk32_{tag}(const JKArgs &a, hipStream_t s)")
        w("{")
        w(f"    hipLaunchKernelGGL(jk32_{tag}, dim3((unsigned)((a.nq + {block - 1}) / {block})), dim3({block}), 0, s, a);")
        w("}")
        w(f"void launch_eri32_{tag}(const EriArgs &a, hipStream_t s)")
        w("{")
        w(f"    hipLaunchKernelGGL(eri32_{tag}, dim3((unsigned)((a.ntask + {block - 1}) / {block})), dim3({block}), 0, s, a);")
        w("}")
    w("")
    w("}  // namespace hgp")
    meta = ClassMeta(ls, tag, 0, block, len(g.nodes), g.flops(), len(g.targets), pl, sched, p2.flops, nout, rule,
                     waves=waves, digest=digest, reduce=reduce, loop=loop, mixed=mixed)
    return "\n".join(out) + "\n", meta


def emit_table(metas):
    out = ['// Generated: the class table the runtime dispatches on (host code only).', '#include "hgp_types.h"', "",
           "#if !defined(__HIP_DEVICE_COMPILE__)", "namespace hgp {"]
    for m in metas:
        out.append(f"void launch_jk_{m.tag}(const JKArgs &, hipStream_t);")
        out.append(f"void launch_eri_{m.tag}(const EriArgs &, hipStream_t);")
        if m.tier == 1:
            out.append(f"void launch_p1_{m.tag}(const P1Args &, hipStream_t);")
        if m.tier in (2, 3):
            out.append(f"int prepare_{m.tag}();")
        if m.mixed:
            out.append(f"void launch_jk32_{m.tag}(const JKArgs &, hipStream_t);")
        if getattr(m, "eri_tiles", False):
            out.append(f"void launch_erit_{m.tag}(const EriArgs &, hipStream_t);")
        if getattr(m, "p1_32", False):
            out.append(f"void launch_p1f_{m.tag}(const P1Args &, hipStream_t);")
        if m.mixed and m.tier == 0:
            out.append(f"void launch_eri32_{m.tag}(const EriArgs &, hipStream_t);")
    out.append("")
    out.append("extern const ClassKernels g_class_table[] = {")
    for m in metas:
        la, lb, lc, ld = m.ls
        p1 = f"launch_p1_{m.tag}" if m.tier == 1 else "nullptr"
        prep = f"prepare_{m.tag}" if m.tier in (2, 3) else "nullptr"
        jk32 = f"launch_jk32_{m.tag}" if m.mixed else "nullptr"
        tiles = f"launch_erit_{m.tag}" if getattr(m, "eri_tiles", False) else "nullptr"
        out.append(f"    {{{la}, {lb}, {lc}, {ld}, {m.tier}, launch_jk_{m.tag}, launch_eri_{m.tag}, {p1}, {prep}, {jk32}, {m.block}, "
                   f"{m.vrr_flops}.0, {m.p2_flops}.0, {m.n_hrr}, {m.peak_live}, {m.scratch_slots}, {m.chunks}, "
                   f"{m.max_batch}, {1 if getattr(m, 'eri_wave', False) else 0}, {tiles}, "
                   f"{'launch_p1f_' + m.tag if getattr(m, 'p1_32', False) else 'nullptr'}, "
                   f"{'launch_eri32_' + m.tag if m.mixed and m.tier == 0 else 'nullptr'}}},")
    out.append("};")
    out.append(f"extern const int g_num_classes = {len(metas)};")
    out.append("")
    out.append("}  // namespace hgp")
    out.append("#endif")
    return "\n".join(out) + "\n"
