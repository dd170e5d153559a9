"""First-derivative integrals d/dR (ab|cd), the adjacent step of the method
for nuclear gradients (the paper's Sec. IV counts first-derivative kernel
variants; Sec. VII names derivative integrals as the next step), in three
forms of one program (deriv_program): op tables for the wave-cooperative
interpreter (csrc/hgp_t3.hip); a register form, one lane per quartet, for
the classes whose accumulators fit in registers; and a staged form whose
Phase 1 runs the VRR in register-resident chunks into a buffer, from which
the interpreter runs the tables' Phase 2.

Differentiating a primitive Cartesian Gaussian x_A^a e^(-alpha r_A^2) in its
centre A along axis i gives 2 alpha x_A^(a+1_i) e^.. - a_i x_A^(a-1_i) e^..,
so, per primitive quartet and with the same normalisation and contraction
coefficients,

  dA_i (ab|cd) = 2 alpha (a+1_i b|cd) - a_i (a-1_i b|cd),
  dB_i (ab|cd) = 2 beta  (a b+1_i|cd) - b_i (a b-1_i|cd),
  dC_i (ab|cd) = 2 gamma (ab|c+1_i d) - c_i (ab|c-1_i d),
  dD_i (ab|cd) = -(dA_i + dB_i + dC_i)   (translational invariance).

The exponent weights belong inside the contraction sum, and the HRR and the
shell transforms are linear with shell-pair coefficients, so the method's
order stays: one VRR per primitive quartet (Eq. vrr) over the union of the
[e0|f0] the six shifted classes need, accumulated into four banks -- the
2alpha-, 2beta- and 2gamma-weighted ones and the unweighted one -- then per
centre the HRR (Eq. hrr) of the two shifted classes in the Cartesian basis,
their combination, and T(la) T(lb) T(lc) T(ld) on the result (Eq. cart2sph).
The weights are three slots that the interpreter fills per primitive
quartet from the primitive pair records (ACC_W ops), or three registers
(wa, wb, wg) in the register-resident forms.

Outputs, in order: [centre A, B, C, D][axis x, y, z][mu][nu][lam][sig] of the
canonical class.
"""
from __future__ import annotations

from . import phase2 as p2mod
from . import vrr as vrrmod
from .cart import add, comps, levels, nsph
from .emit_t3 import BUNDLE, assemble_tables
from .sph import tmatrix


class TargetGraph(vrrmod.VRRGraph):
    """The VRR graph (same axis rule and parents as the class graphs) of an
    arbitrary set of targets (e, f) at m = 0."""

    def __init__(self, targets, L, rule="ket_zyx"):
        self.ls = None
        self.L = L
        self.rule = rule
        self.nodes = []
        self.index = {}
        self.targets = list(targets)
        self.target_ids = [self._need((e, f, 0)) for (e, f) in self.targets]
        self.children = [[] for _ in self.nodes]
        for v, nd in enumerate(self.nodes):
            for p in nd.parents:
                if p is not None:
                    self.children[p].append(v)
        self.is_target = [False] * len(self.nodes)
        for t in self.target_ids:
            self.is_target[t] = True


def _rng(lo, hi):
    return levels(max(lo, 0), hi) if hi >= max(lo, 0) else ()


def deriv_pieces(la, lb, lc, ld):
    """The shifted classes: (centre, weight bank, l's of the shifted class,
    which index moves, +1 or -1)."""
    out = []
    for r, l in enumerate((la, lb, lc, ld)[:3]):
        up = [la, lb, lc, ld]
        up[r] += 1
        out.append((r, "abg"[r], tuple(up), +1))
        if l > 0:
            dn = [la, lb, lc, ld]
            dn[r] -= 1
            out.append((r, "0", tuple(dn), -1))
    return out


class DerivProgram:
    """Everything both forms run for one derivative class: the VRR graph of
    the accumulator targets and its order, the banks (acc_index: (bank,
    (e, f)) per accumulator; accs: target node -> [(accumulator, bank)]),
    per shifted class its Cartesian HRR ops (piece_ops, in deriv_pieces
    order), per (centre, axis) of A, B, C the combination and transform ops
    (centre_ops) and the names of the spherical derivatives (sph_out), the
    ops of centre D by translational invariance (d_ops), and the flat op
    list and output names the tables take."""


def deriv_program(la, lb, lc, ld, rule="ket_zyx"):
    ls = (la, lb, lc, ld)
    P = DerivProgram()
    P.ls = ls
    P.L = L = sum(ls) + 1
    P.pieces = pieces = deriv_pieces(*ls)
    # accumulator banks: the [e0|f0] each shifted class's HRR reads
    banks = {}
    for (r, w, sl, _) in pieces:
        for e in _rng(sl[0], sl[0] + sl[1]):
            for f in _rng(sl[2], sl[2] + sl[3]):
                banks.setdefault(w, {})[(e, f)] = None
    acc_index = {}
    for w in ("a", "b", "g", "0"):
        for key in banks.get(w, {}):
            acc_index[(w, key)] = len(acc_index)
    P.acc_index = acc_index
    targets = sorted({key for (w, key) in acc_index}, key=lambda t: (sum(t[0]), t[0], sum(t[1]), t[1]))
    P.g = g = TargetGraph(targets, L, rule)
    P.sched, P.pl, P.order = vrrmod.best_order(g)
    tid = {t: g.target_ids[k] for k, t in enumerate(g.targets)}
    P.accs = {}
    for (w, key), k in acc_index.items():
        P.accs.setdefault(tid[key], []).append((k, w))
    # ---- Phase 2: per shifted class the Cartesian HRR, then per centre the
    # combination and the four transforms
    ops = []
    cur_list = [ops]
    P.piece_ops = []
    cart = {}                     # (centre, sign) -> {(a, b, c, d) cart tuples: name}
    for n, (r, w, sl, sgn) in enumerate(pieces):
        p2 = p2mod.Phase2(*sl, hname=lambda e, f, w=w: f"h{acc_index[(w, (e, f))]}", prefix=f"s{n}_",
                          spherical=False)
        ops.extend(p2.ops)
        P.piece_ops.append(list(p2.ops))
        ca, cb, cc, cd = (comps(x) for x in sl)
        cart[(r, sgn)] = {(ca[i], cb[j], cc[k], cd[m]): nm for (i, j, k, m), nm in p2.out.items()}
    counter = [0]

    def new(prefix):
        counter[0] += 1
        return f"{prefix}{counter[0]}"

    def lin(terms, prefix):
        terms = [(c, x) for c, x in terms if c != 0.0]
        if len(terms) == 1 and terms[0][0] == 1.0:
            return terms[0][1]
        d = new(prefix)
        ops.append((d, "lin", tuple(terms)))
        cur_list[0].append((d, "lin", tuple(terms)))
        return d

    C0 = [comps(x) for x in ls]
    T = [tmatrix(x) for x in ls]
    P.nsph = na, nb, nc, nd = tuple(nsph(x) for x in ls)
    sph_out = {}
    P.centre_ops = {}
    for r in range(3):
        for i in range(3):
            cur_list[0] = P.centre_ops[(r, i)] = []
            # Cartesian derivative tensor along axis i of centre r
            dc = {}
            for a in C0[0]:
                for b in C0[1]:
                    for c in C0[2]:
                        for d in C0[3]:
                            q = [a, b, c, d]
                            up = list(q)
                            up[r] = add(q[r], i, +1)
                            terms = [(1.0, cart[(r, +1)][tuple(up)])]
                            if q[r][i] > 0:
                                dn = list(q)
                                dn[r] = add(q[r], i, -1)
                                terms.append((-float(q[r][i]), cart[(r, -1)][tuple(dn)]))
                            dc[(a, b, c, d)] = lin(terms, "dc")
            # transforms, one index at a time: a, then b, c, d
            cur = {(ka, b, c, d): v for (a, b, c, d), v in dc.items() for ka in [C0[0].index(a)]}
            stage = {}
            for mu, row in enumerate(T[0]):
                for b in C0[1]:
                    for c in C0[2]:
                        for d in C0[3]:
                            stage[(mu, b, c, d)] = lin([(cf, cur[(j, b, c, d)]) for j, cf in row], "ta")
            cur, stage = stage, {}
            for mu in range(na):
                for nu, row in enumerate(T[1]):
                    for c in C0[2]:
                        for d in C0[3]:
                            stage[(mu, nu, c, d)] = lin([(cf, cur[(mu, C0[1][j], c, d)]) for j, cf in row], "tb")
            cur, stage = stage, {}
            for mu in range(na):
                for nu in range(nb):
                    for lam, row in enumerate(T[2]):
                        for d in C0[3]:
                            stage[(mu, nu, lam, d)] = lin([(cf, cur[(mu, nu, C0[2][j], d)]) for j, cf in row], "tc")
            cur, stage = stage, {}
            for mu in range(na):
                for nu in range(nb):
                    for lam in range(nc):
                        for sig, row in enumerate(T[3]):
                            stage[(mu, nu, lam, sig)] = lin([(cf, cur[(mu, nu, lam, C0[3][j])]) for j, cf in row],
                                                            "td")
            sph_out[(r, i)] = stage
    # centre D by translational invariance
    cur_list[0] = P.d_ops = []
    for i in range(3):
        sph_out[(3, i)] = {k: lin([(-1.0, sph_out[(r, i)][k]) for r in range(3)], "dd")
                           for k in sph_out[(0, i)]}
    P.sph_out = sph_out
    P.ops = ops
    P.out_names = [sph_out[(r, i)][(mu, nu, lam, sig)] for r in range(4) for i in range(3) for mu in range(na)
                   for nu in range(nb) for lam in range(nc) for sig in range(nd)]
    P.p2_flops = sum(2 if o[1] == "hrr" else 2 * len(o[2]) - 1 for o in ops)
    # per primitive quartet: the VRR nodes, one add per unweighted and one FMA
    # (2 FLOP) per weighted accumulation
    P.vrr_flops = g.flops() - len(g.targets) + sum(1 if w == "0" else 2 for (w, _) in acc_index)
    return P


def build_deriv_tables(la, lb, lc, ld, rule="ket_zyx", bundle=BUNDLE):
    P = deriv_program(la, lb, lc, ld, rule)
    L = P.L
    # weight slots after the base values: 2 alpha, 2 beta, 2 gamma
    wslot = {"a": L + 1, "b": L + 2, "g": L + 3, "0": None}
    acc0 = L + 4
    accs = {v: [(k, wslot[w]) for (k, w) in lst] for v, lst in P.accs.items()}
    # (an output may repeat or be an accumulator itself, where s and p
    # shells make the transforms and a combination identities: the output
    # slots are then shared or kept, never freed)
    return assemble_tables(P.g, P.order, P.sched, P.pl, L, acc0, len(P.acc_index), accs, P.ops, P.out_names,
                           P.vrr_flops, P.p2_flops, bundle, f"d{la}{lb}{lc}{ld}")


DERIV_LMAX = 2          # derivative tables are built for the classes with l <= 2


def emit_deriv_class(la, lb, lc, ld, rule="ket_zyx"):
    """Host-side wave-form tables of the derivative class and its
    descriptor; the generic t3w_deriv_kernel runs them."""
    from .emit_t3 import WAVE, WAVE_LDS_MAX, _u16_lines, build_wave_tables_from
    ls = (la, lb, lc, ld)
    tag = "".join(str(x) for x in ls)
    w = build_wave_tables_from(build_deriv_tables(*ls, rule=rule, bundle=WAVE), ls)
    if w.lds_bytes > WAVE_LDS_MAX:
        raise ValueError(f"derivative class {tag}: {w.lds_bytes} bytes of LDS per quartet")
    t = w.t
    na, nb, nc, nd = (nsph(x) for x in ls)
    name = f"d{tag}"
    out = [f"// Generated: first-derivative integrals of class ({la}{lb}|{lc}{ld}), wave-form op tables:",
           f"// {t.n_vrr} per-primitive ops, {t.n_p2} Phase-2 ops, {t.nslots} slots, {w.lds_bytes} bytes of LDS.",
           '#include "hgp_t3.h"', "", "#if !defined(__HIP_DEVICE_COMPILE__)", "namespace hgp {", "namespace {", "",
           f"const uint16_t ops_{name}[] = {{"]
    out.extend(_u16_lines(w.ops))
    out.append("};")
    out.append(f"const uint16_t outslots_{name}[] = {{")
    out.extend(_u16_lines(t.outslots))
    out.append("};")
    out.append(f"const double coefs_{name}[] = {{")
    for k in range(0, max(len(t.coefs), 1), 4):
        out.append("    " + ", ".join(repr(c) for c in (t.coefs[k:k + 4] or [0.0])) + ",")
    out.append("};")
    out.append("}  // namespace")
    out.append(f"extern const T3Class t3_{name} = {{{la}, {lb}, {lc}, {ld}, {t.L}, {na}, {nb}, {nc}, {nd}, "
               f"{t.nslots}, {t.n_hrr}, {t.acc0}, {t.n_vrr}, {t.n_p2}, ops_{name}, {max(len(t.coefs), 1)}, "
               f"coefs_{name}, outslots_{name}, 64, {w.maxblk}, {w.lds_bytes}, 0, nullptr, 12}};")
    out.append("}  // namespace hgp")
    out.append("#endif")
    info = {"tag": tag, "nslots": t.nslots, "n_vrr": t.n_vrr, "n_p2": t.n_p2, "lds_bytes": w.lds_bytes,
            "vrr_flops": t.vrr_flops, "p2_flops": t.p2_flops}
    return "\n".join(out) + "\n", info


def emit_deriv_table(classes, reg=(), staged=()):
    """The descriptor table of the derivative classes built into the library;
    reg: the tags of the classes that also have the register form; staged:
    {tag: chunks per Phase-1 launch} of those with the staged form's Phase-1
    kernels."""
    out = ["// Generated: the first-derivative classes of the library.", '#include "hgp_t3.h"', "",
           "#if !defined(__HIP_DEVICE_COMPILE__)", "namespace hgp {"]
    for ls in classes:
        tag = "".join(str(x) for x in ls)
        out.append(f"extern const T3Class t3_d{tag};")
        if tag in reg:
            out.append(f"void launch_dreg_{tag}(const EriArgs &, const int32_t *, int, hipStream_t);")
        if tag in staged:
            out.append(f"void launch_dp1_{tag}(const EriArgs &, const int32_t *, int, hipStream_t);")
    out.append("extern const DerivClass g_deriv_table[] = {")
    for ls in classes:
        tag = "".join(str(x) for x in ls)
        fn = f"launch_dreg_{tag}" if tag in reg else "nullptr"
        p1 = f"launch_dp1_{tag}" if tag in staged else "nullptr"
        cpl = (staged or {}).get(tag, 0) if isinstance(staged, dict) else 0
        out.append(f"    {{{ls[0]}, {ls[1]}, {ls[2]}, {ls[3]}, &t3_d{tag}, {fn}, {p1}, {cpl}}},")
    if not classes:
        out.append("    {0, 0, 0, 0, nullptr, nullptr, nullptr, 0},")
    out.append("};")
    out.append(f"extern const int g_num_deriv = {len(classes)};")
    out.append("}  // namespace hgp")
    out.append("#endif")
    return "\n".join(out) + "\n"


# ---------------------------------------------------------------------------
# Register form: one lane per quartet, every value in registers.  The same
# program as the tables (deriv_program), emitted as straight-line code: the
# weighted accumulation inside the primitive loop, then per centre A, B, C
# the Cartesian HRR of its two shifted classes, the combination and the
# transforms, each result stored as soon as it exists.  Centre D is the
# negated running sum of the other three (translational invariance), so
# only 3 n_sph^4 sums stay live across the centres.

REG_MAX_ACC = 224       # classes with more accumulators keep the wave-form tables
REG_BLOCK = 128


def _vrr_weighted(P, ind):
    """The VRR in P.order (emit._vrr_lines' statements) with each target
    added to its accumulators, weighted by its bank's exponent."""
    from .emit import _vrr_lines

    class _Graph:                        # the class graph without its targets: accumulation is emitted here
        nodes = P.g.nodes
        target_ids = []

    lines, _ = _vrr_lines(_Graph, P.order, [], ind)
    wname = {"a": "wa", "b": "wb", "g": "wg"}
    out = []
    for v, ln in zip(P.order, lines):
        out.append(ln)
        for (k, w) in P.accs.get(v, []):
            out.append(f"{ind}h{k} += v{v};" if w == "0" else f"{ind}h{k} = fma({wname[w]}, v{v}, h{k});")
    return out


def _phase2_stores(P, ind):
    """Phase 2 in centre order with the stores: HGP_DSTORE(o<r>, axis, mu,
    nu, lam, sig, value) writes block [centre r][axis] of the canonical
    element; o3 is centre D."""
    from .emit import _p2_lines

    class _Ops:
        def __init__(self, ops):
            self.ops = ops

    na, nb, nc, nd = P.nsph
    elems = [(mu, nu, lam, sig) for mu in range(na) for nu in range(nb) for lam in range(nc) for sig in range(nd)]
    out = []
    for r in range(3):
        for n, pc in enumerate(P.pieces):
            if pc[0] == r:
                out.extend(_p2_lines(_Ops(P.piece_ops[n]), ind))
        for i in range(3):
            out.extend(_p2_lines(_Ops(P.centre_ops[(r, i)]), ind))
            for el in elems:
                v = P.sph_out[(r, i)][el]
                ds = f"ds{i}_{'_'.join(map(str, el))}"
                out.append(f"{ind}HGP_DSTORE(o{r}, {i}, {', '.join(map(str, el))}, {v});")
                if r == 0:
                    out.append(f"{ind}double {ds} = {v};")
                elif r == 1:
                    out.append(f"{ind}{ds} += {v};")
                else:
                    out.append(f"{ind}HGP_DSTORE(o3, {i}, {', '.join(map(str, el))}, -({ds} + {v}));")
    return out


def reg_eligible(ls):
    return len(deriv_program(*ls).acc_index) <= REG_MAX_ACC


def emit_deriv_reg(la, lb, lc, ld, rule="ket_zyx", block=REG_BLOCK):
    """HIP source of the register-form derivative kernel dreg_<tag> and its
    launcher (same task layout and centre code as t3w_deriv_kernel)."""
    from .emit import loop_close, loop_prelude
    ls = (la, lb, lc, ld)
    tag = "".join(str(x) for x in ls)
    P = deriv_program(*ls, rule=rule)
    na, nb, nc, nd = P.nsph
    nacc = len(P.acc_index)
    out = [f"// Generated: first-derivative integrals of class ({la}{lb}|{lc}{ld}), register form:",
           f"// {len(P.g.nodes)} VRR nodes (PeakLive {P.pl}), {nacc} weighted accumulators, "
           f"{P.vrr_flops} FLOP per primitive quartet, {P.p2_flops} FLOP of Phase 2.",
           '#include "hgp_device.h"', "", "namespace hgp {", "namespace {", "",
           f"__global__ __launch_bounds__({block}) void dreg_{tag}(EriArgs a, const int32_t *__restrict__ code)",
           "{"]
    w = out.append
    w(f"    const int64_t q = (int64_t)blockIdx.x * {block} + threadIdx.x;")
    w("    if (q >= a.ntask) return;")
    w("    const EriTask tk = a.tasks[q];")
    w("    const PairInfo pb = a.pairs[tk.bra], pk = a.pairs[tk.ket];")
    w("    const PairGeo gb = a.geo[tk.bra], gk = a.geo[tk.ket];")
    w("    const PrimPair *__restrict__ prims = a.prims;")
    w("    const double *__restrict__ boys = a.boys;")
    for k0 in range(0, nacc, 8):
        w("    double " + ", ".join(f"h{k} = 0.0" for k in range(k0, min(nacc, k0 + 8))) + ";")
    out.extend(loop_prelude(P.L, "    ", "late", weights=True))
    out.extend(_vrr_weighted(P, "        "))
    out.extend(loop_close("    "))
    w("    const double ABx = gb.abx, ABy = gb.aby, ABz = gb.abz;")
    w("    const double CDx = gk.abx, CDy = gk.aby, CDz = gk.abz;")
    w("    (void)ABx; (void)ABy; (void)ABz; (void)CDx; (void)CDy; (void)CDz;")
    nint = na * nb * nc * nd
    w(f"    constexpr int64_t NINT = {nint};")
    w("    const int32_t pos = code[tk.bra >> 1];")
    w("    double *__restrict__ o = a.out + tk.off;")
    for r in range(4):
        w(f"    double *__restrict__ o{r} = o + 3 * ((pos >> {2 * r}) & 3) * NINT;")
    w("#define HGP_DSTORE(p, ax, mu, nu, lam, sig, v) \\")
    w("    (p)[(ax) * NINT + (mu) * tk.s0 + (nu) * tk.s1 + (lam) * tk.s2 + (sig) * tk.s3] = (v)")
    out.extend(_phase2_stores(P, "    "))
    w("#undef HGP_DSTORE")
    w("}")
    w("")
    w("}  // namespace")
    w("")
    w(f"void launch_dreg_{tag}(const EriArgs &a, const int32_t *code, int, hipStream_t s)")
    w("{")
    w(f"    hipLaunchKernelGGL(dreg_{tag}, dim3((unsigned)((a.ntask + {block - 1}) / {block})), dim3({block}), 0, s, "
      "a, code);")
    w("}")
    w("")
    w("}  // namespace hgp")
    return "\n".join(out) + "\n"


# ---------------------------------------------------------------------------
# Staged form, for the classes whose accumulators do not fit in registers:
# Phase 1 runs one lane per (quartet, chunk, segment), a chunk being a run of
# the targets (e, f) in (|e|, e, |f|, f) order carrying at most `cap`
# accumulators of all banks, with the VRR subgraph of its targets scheduled
# on its own (nodes that chunks share are recomputed), and segment s of nseg
# a proportional share of the quartet's primitive quartets (so that classes
# with few quartets still fill the device).  After its primitive loop a lane
# stores its partial weighted accumulators to the slot-major buffer,
# accumulator k of batch quartet i at scratch[(s * n_acc + k) * stride + i].
# Phase 2 is the wave-form tables' Phase 2, which sums the nseg partials of
# each accumulator in segment order (t3w_launch_deriv_p2).

# (accumulators per chunk, waves per SIMD asked of the compiler, 0: none): the
# build steps down this list while a Phase-1 part of the class spills.  Two
# waves per SIMD at caps 48/32 measured slower on the 400 000-quartet sample
# for 17 of the 20 staged classes (35.9 against 29.0 ms a call): the extra
# recomputation (x2-2.9 instead of x1.2-2) costs more than the occupancy gains.
STAGE_CAPS = ((96, 0), (64, 0), (40, 0))
STAGE_PART = 16               # chunks per Phase-1 kernel (one translation unit each)


def stage_chunks(P, cap):
    """[(targets, [(global accumulator, bank)] per target)] in target order."""
    out, cur, n = [], [], 0
    for k, t in enumerate(P.g.targets):
        c = len(P.accs[P.g.target_ids[k]])
        if cur and n + c > cap:
            out.append(cur)
            cur, n = [], 0
        cur.append(t)
        n += c
    if cur:
        out.append(cur)
    return out


def chunk_vrr(P, targets, ind=""):
    """One chunk's VRR statements with its weighted accumulation, its
    accumulators (global numbers, ascending), its node count and PeakLive."""
    from .emit import _vrr_lines
    g = TargetGraph(targets, P.L)
    _, pl, order = vrrmod.best_order(g)
    full = {t: P.g.target_ids[k] for k, t in enumerate(P.g.targets)}
    accs = {g.target_ids[j]: P.accs[full[t]] for j, t in enumerate(g.targets)}
    ks = sorted(k for lst in accs.values() for (k, _) in lst)

    class _Graph:
        nodes = g.nodes
        target_ids = []

    lines, _ = _vrr_lines(_Graph, order, [], ind)
    wname = {"a": "wa", "b": "wb", "g": "wg"}
    out = []
    for v, ln in zip(order, lines):
        out.append(ln)
        for (k, w) in accs.get(v, []):
            out.append(f"{ind}h{k} += v{v};" if w == "0" else f"{ind}h{k} = fma({wname[w]}, v{v}, h{k});")
    return out, ks, len(g.nodes), pl


def _chunk_lines(P, targets, ind):
    """Accumulator declarations, the primitive loop (segment s of nseg) with
    the chunk's VRR and weighted accumulation, and the stores, for one chunk."""
    from .emit import loop_close, loop_prelude
    vrr, ks, nn, pl = chunk_vrr(P, targets, ind + "    ")
    out = []
    for k0 in range(0, len(ks), 8):
        out.append(f"{ind}double " + ", ".join(f"h{k} = 0.0" for k in ks[k0:k0 + 8]) + ";")
    out.extend(loop_prelude(P.L, ind, "late", weights=True, seg=True))
    out.extend(vrr)
    out.extend(loop_close(ind))
    for k in ks:
        out.append(f"{ind}S[{k} * a.stride] = h{k};")
    return out, nn, pl


def emit_deriv_staged(la, lb, lc, ld, cap=STAGE_CAPS[0], rule="ket_zyx", block=REG_BLOCK):
    """Sources of the staged form's Phase-1 kernels: {part: source}, and its
    description; cap = (accumulators per chunk, waves per SIMD or 0).  Part 0
    also holds the class launcher launch_dp1_<tag>, which runs every part
    over the batch a.tasks[0 .. a.ntask)."""
    from .emit import waves_attr
    cap, waves = cap if isinstance(cap, tuple) else (cap, 0)
    ls = (la, lb, lc, ld)
    tag = "".join(str(x) for x in ls)
    P = deriv_program(*ls, rule=rule)
    chunks = stage_chunks(P, cap)
    nparts = (len(chunks) + STAGE_PART - 1) // STAGE_PART
    srcs = {}
    nodes = 0
    maxpl = 0
    for p in range(nparts):
        part = chunks[p * STAGE_PART:(p + 1) * STAGE_PART]
        out = [f"// Generated: first-derivative integrals of class ({la}{lb}|{lc}{ld}), staged form, Phase 1 part {p}:",
               f"// chunks {p * STAGE_PART} .. {p * STAGE_PART + len(part) - 1} of {len(chunks)} "
               f"(at most {cap} weighted accumulators each).",
               '#include "hgp_device.h"', "", "namespace hgp {", "namespace {", "",
               f"__global__ __launch_bounds__({block}){waves_attr(waves)} void dp1_{tag}p{p}(EriArgs a, int nseg)", "{"]
        w = out.append
        w(f"    const int64_t item = (int64_t)blockIdx.x * {block} + threadIdx.x;")
        w("    const int64_t n = a.ntask, per = (int64_t)nseg * n;")
        w(f"    if (item >= {len(part)} * per) return;")
        w("    const int c = (int)(item / per);              // chunk- then segment-major: a wave's lanes share both")
        w("    const int s = (int)((item - c * per) / n);")
        w("    const int64_t i = item - c * per - s * n;")
        w("    const EriTask tk = a.tasks[i];")
        w("    const PairInfo pb = a.pairs[tk.bra], pk = a.pairs[tk.ket];")
        w("    const PairGeo gb = a.geo[tk.bra], gk = a.geo[tk.ket];")
        w("    const PrimPair *__restrict__ prims = a.prims;")
        w("    const double *__restrict__ boys = a.boys;")
        w(f"    double *__restrict__ S = a.scratch + (int64_t)s * {len(P.acc_index)} * a.stride + i;")
        w("    switch (c) {")
        for j, targets in enumerate(part):
            w(f"    case {j}: {{")
            lines, nn, pl = _chunk_lines(P, targets, "        ")
            nodes += nn
            maxpl = max(maxpl, pl)
            out.extend(lines)
            w("        break;")
            w("    }")
        w("    default:")
        w("        break;")
        w("    }")
        w("}")
        w("")
        w("}  // namespace")
        w("")
        w(f"void launch_dp1_{tag}p{p}(const EriArgs &a, int nseg, hipStream_t s)")
        w("{")
        w(f"    const int64_t items = {len(part)} * (int64_t)nseg * a.ntask;")
        w(f"    hipLaunchKernelGGL(dp1_{tag}p{p}, dim3((unsigned)((items + {block - 1}) / {block})), dim3({block}), 0, "
          "s, a, nseg);")
        w("}")
        if p == 0:
            w("")
            for q in range(1, nparts):
                w(f"void launch_dp1_{tag}p{q}(const EriArgs &a, int nseg, hipStream_t s);")
            w(f"void launch_dp1_{tag}(const EriArgs &a, const int32_t *, int nseg, hipStream_t s)")
            w("{")
            for q in range(nparts):
                w(f"    launch_dp1_{tag}p{q}(a, nseg, s);")
            w("}")
        w("")
        w("}  // namespace hgp")
        srcs[p] = "\n".join(out) + "\n"
    info = {"tag": tag, "cap": cap, "waves": waves, "chunks": len(chunks), "parts": nparts, "nodes": nodes,
            "recompute": round(nodes / len(P.g.nodes), 3), "max_peak_live": maxpl, "n_acc": len(P.acc_index)}
    return srcs, info
