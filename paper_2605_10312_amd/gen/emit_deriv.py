"""First-derivative integrals d/dR (ab|cd) as op tables for the
wave-cooperative interpreter (csrc/hgp_t3.hip), the adjacent step of the
method for nuclear gradients (the paper's Sec. IV counts first-derivative
kernel variants; Sec. VII names derivative integrals as the next step).

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
quartet from the primitive pair records (ACC_W ops).

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


def build_deriv_tables(la, lb, lc, ld, rule="ket_zyx", bundle=BUNDLE):
    ls = (la, lb, lc, ld)
    L = sum(ls) + 1
    pieces = deriv_pieces(*ls)
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
    targets = sorted({key for (w, key) in acc_index}, key=lambda t: (sum(t[0]), t[0], sum(t[1]), t[1]))
    g = TargetGraph(targets, L, rule)
    sched, pl, order = vrrmod.best_order(g)
    # weight slots after the base values: 2 alpha, 2 beta, 2 gamma
    wslot = {"a": L + 1, "b": L + 2, "g": L + 3, "0": None}
    acc0 = L + 4
    tid = {t: g.target_ids[k] for k, t in enumerate(g.targets)}
    accs = {}
    for (w, key), k in acc_index.items():
        accs.setdefault(tid[key], []).append((k, wslot[w]))
    # ---- Phase 2: per shifted class the Cartesian HRR, then per centre the
    # combination and the four transforms
    ops = []
    cart = {}                     # (centre, sign) -> {(a, b, c, d) cart tuples: name}
    for n, (r, w, sl, sgn) in enumerate(pieces):
        p2 = p2mod.Phase2(*sl, hname=lambda e, f, w=w: f"h{acc_index[(w, (e, f))]}", prefix=f"s{n}_",
                          spherical=False)
        ops.extend(p2.ops)
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
        return d

    C0 = [comps(x) for x in ls]
    T = [tmatrix(x) for x in ls]
    na, nb, nc, nd = (nsph(x) for x in ls)
    sph_out = {}
    for r in range(3):
        for i in range(3):
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
    for i in range(3):
        sph_out[(3, i)] = {k: lin([(-1.0, sph_out[(r, i)][k]) for r in range(3)], "dd")
                           for k in sph_out[(0, i)]}
    out_names = [sph_out[(r, i)][(mu, nu, lam, sig)] for r in range(4) for i in range(3) for mu in range(na)
                 for nu in range(nb) for lam in range(nc) for sig in range(nd)]
    # (an output may repeat or be an accumulator itself, where s and p
    # shells make the transforms and a combination identities: the output
    # slots are then shared or kept, never freed)
    flops = 0
    for o in ops:
        flops += 2 if o[1] == "hrr" else 2 * len(o[2]) - 1
    n_acc = len(acc_index)
    # per primitive quartet: the VRR nodes, one add per unweighted and one FMA
    # (2 FLOP) per weighted accumulation
    vrr_flops = g.flops() - len(g.targets) + sum(1 if w == "0" else 2 for (w, _) in acc_index)
    return assemble_tables(g, order, sched, pl, L, acc0, n_acc, accs, ops, out_names, vrr_flops, flops, bundle,
                           f"d{la}{lb}{lc}{ld}")


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


def emit_deriv_table(classes):
    """The descriptor table of the derivative classes built into the library."""
    out = ["// Generated: the first-derivative classes of the library.", '#include "hgp_t3.h"', "",
           "#if !defined(__HIP_DEVICE_COMPILE__)", "namespace hgp {"]
    for ls in classes:
        out.append(f"extern const T3Class t3_d{''.join(str(x) for x in ls)};")
    out.append("extern const DerivClass g_deriv_table[] = {")
    for ls in classes:
        out.append(f"    {{{ls[0]}, {ls[1]}, {ls[2]}, {ls[3]}, &t3_d{''.join(str(x) for x in ls)}}},")
    if not classes:
        out.append("    {0, 0, 0, 0, nullptr},")
    out.append("};")
    out.append(f"extern const int g_num_deriv = {len(classes)};")
    out.append("}  // namespace hgp")
    out.append("#endif")
    return "\n".join(out) + "\n"
