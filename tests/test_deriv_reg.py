"""The register form of the first-derivative classes (gen/emit_deriv.py),
run on the CPU.  The generator's own statements -- the weighted
accumulation inside the primitive loop, the centre-ordered Cartesian HRR,
combination and transforms, the stores and the running sums that give centre
D -- are executed by Python (each C statement is also a Python one) over every
primitive quartet of contracted shells, and the 12 blocks are compared with
the oracle's derivative integrals, which are pinned to finite differences and
translational invariance (tests/test_oracle_deriv.py).  The Boys values come
from scipy's 1F1, independent of both sides."""
import re

import numpy as np
import pytest
from scipy.special import hyp1f1

import oracle
import workloads
from paper_2605_10312_amd.gen import emit_deriv


def _py(lines):
    out = []
    for ln in lines:
        s = ln.strip()
        assert s.endswith(";"), s
        s = re.sub(r"^(const )?double ", "", s[:-1])
        out.append(s)
    return compile("\n".join(out), "<emitted>", "exec")


def run_reg(ls, basis):
    """The emitted program on shells 0..3 of `basis` (canonical order)."""
    P = emit_deriv.deriv_program(*ls)
    vrr = _py(emit_deriv._vrr_weighted(P, ""))
    p2 = _py(emit_deriv._phase2_stores(P, ""))
    env = {"fma": lambda a, b, c: a * b + c}
    for k in range(len(P.acc_index)):
        env[f"h{k}"] = 0.0
    off = np.concatenate([[0], np.cumsum(basis.nprim)])
    ex = [basis.exps[off[s]:off[s + 1]] for s in range(4)]
    co = [oracle.norm_coefs(int(basis.l[s]), ex[s], basis.coefs[off[s]:off[s + 1]]) for s in range(4)]
    A, B, C, D = (basis.centers[s] for s in range(4))
    for i, a in enumerate(ex[0]):
        for j, b in enumerate(ex[1]):
            zeta = a + b
            Pc = (a * A + b * B) / zeta
            Kb = co[0][i] * co[1][j] * np.exp(-a * b / zeta * np.sum((A - B) ** 2)) * np.sqrt(2) * np.pi ** 1.25 / zeta
            for k, c in enumerate(ex[2]):
                for m, d in enumerate(ex[3]):
                    eta = c + d
                    Q = (c * C + d * D) / eta
                    Kk = co[2][k] * co[3][m] * np.exp(-c * d / eta * np.sum((C - D) ** 2)) * np.sqrt(2) * np.pi ** 1.25 / eta
                    ze = zeta + eta
                    rz, re_ = eta / ze, zeta / ze
                    PQ = Pc - Q
                    T = zeta * rz * np.sum(PQ ** 2)
                    env.update(base=Kb * Kk / np.sqrt(ze), o2z=0.5 / zeta, o2e=0.5 / eta, o2ze=0.5 / ze, rz=rz, re=re_,
                               F=[hyp1f1(n + 0.5, n + 1.5, -T) / (2 * n + 1) for n in range(P.L + 1)],
                               wa=2 * a, wb=2 * b, wg=2 * c)
                    for ax, n in enumerate("xyz"):
                        env.update({f"PA{n}": (Pc - A)[ax], f"QC{n}": (Q - C)[ax], f"WP{n}": -rz * PQ[ax],
                                    f"WQ{n}": re_ * PQ[ax]})
                    exec(vrr, env)
    na, nb, nc, nd = P.nsph
    out = np.full((4, 3, na, nb, nc, nd), np.nan)
    seen = np.zeros(out.shape, bool)

    def store(r, ax, mu, nu, lam, sig, v):
        assert not seen[r, ax, mu, nu, lam, sig]
        seen[r, ax, mu, nu, lam, sig] = True
        out[r, ax, mu, nu, lam, sig] = v

    for ax, n in enumerate("xyz"):
        env[f"AB{n}"] = (A - B)[ax]
        env[f"CD{n}"] = (C - D)[ax]
    env.update(HGP_DSTORE=store, o0=0, o1=1, o2=2, o3=3)
    exec(p2, env)
    assert seen.all()
    return out


def _basis(ls, nprim, seed):
    rng = np.random.default_rng(seed)
    cen = rng.uniform(0.0, 1.6, (4, 3))
    exps = np.exp(rng.uniform(np.log(0.3), np.log(4.0), sum(nprim)))
    return workloads.Basis(l=np.array(ls, np.int32), nprim=np.array(nprim, np.int32), centers=cen, exps=exps,
                           coefs=rng.uniform(0.1, 1.0, sum(nprim)), atom=np.arange(4, dtype=np.int32), atoms=cen)


REG = [(0, 0, 0, 0), (1, 0, 0, 0), (1, 0, 1, 0), (1, 1, 0, 0), (2, 0, 0, 0), (2, 0, 1, 0), (2, 1, 0, 0),
       (1, 1, 1, 0), (2, 2, 0, 0)]


def test_register_classes_are_the_small_ones():
    got = [ls for ls in REG if emit_deriv.reg_eligible(ls)]
    assert got == REG
    assert not emit_deriv.reg_eligible((2, 0, 2, 0)) and not emit_deriv.reg_eligible((1, 1, 1, 1))


@pytest.mark.parametrize("ls", REG)
def test_register_form_matches_oracle(ls):
    b = _basis(ls, (2, 1, 3, 2), seed=90 + sum(ls))
    got = run_reg(ls, b)
    ref = oracle.eri_deriv_shell_quartet(b, 0, 1, 2, 3, precision="long double")
    scale = np.abs(ref).max()
    err = np.abs(got - ref).max()
    assert err <= 1e-12 * scale + 1e-14, (ls, err, scale)


def test_register_source_declares_what_it_uses():
    src = emit_deriv.emit_deriv_reg(2, 1, 0, 0)
    assert "void launch_dreg_2100(const EriArgs &a, const int32_t *code, int, hipStream_t s)" in src
    assert "__launch_bounds__(128) void dreg_2100(EriArgs a, const int32_t *__restrict__ code)" in src
    assert src.count("HGP_DSTORE(o3, ") == 3 * 5 * 3      # centre D: 3 axes x 15 elements
    table = emit_deriv.emit_deriv_table([(2, 1, 0, 0), (2, 2, 2, 2)], ["2100"])
    assert "&t3_d2100, launch_dreg_2100, nullptr, 0}" in table and "&t3_d2222, nullptr, nullptr, 0}" in table


def _prim_env(ls, seed):
    """Per-primitive VRR inputs of one random primitive quartet (the
    same quantities the kernels form from the pair records)."""
    rng = np.random.default_rng(seed)
    A, B, C, D = rng.uniform(0.0, 1.6, (4, 3))
    a, b, c, d = np.exp(rng.uniform(np.log(0.3), np.log(4.0), 4))
    zeta, eta = a + b, c + d
    Pc, Q = (a * A + b * B) / zeta, (c * C + d * D) / eta
    ze = zeta + eta
    rz, re_ = eta / ze, zeta / ze
    PQ = Pc - Q
    T = zeta * rz * np.sum(PQ ** 2)
    env = {"fma": lambda x, y, z: x * y + z, "base": 0.7, "o2z": 0.5 / zeta, "o2e": 0.5 / eta, "o2ze": 0.5 / ze,
           "rz": rz, "re": re_, "wa": 2 * a, "wb": 2 * b, "wg": 2 * c,
           "F": [hyp1f1(n + 0.5, n + 1.5, -T) / (2 * n + 1) for n in range(sum(ls) + 2)]}
    for ax, n in enumerate("xyz"):
        env.update({f"PA{n}": (Pc - A)[ax], f"QC{n}": (Q - C)[ax], f"WP{n}": -rz * PQ[ax], f"WQ{n}": re_ * PQ[ax]})
    return env


@pytest.mark.parametrize("ls,cap", [((1, 1, 1, 0), 96), ((2, 2, 0, 0), 40), ((2, 1, 2, 1), 96), ((2, 2, 1, 1), 64),
                                    ((2, 2, 2, 2), 96)])
def test_staged_chunks_cover_every_accumulator(ls, cap):
    """Each accumulator is stored by exactly one chunk, with the value the
    whole-class program (checked against the oracle above) gives it, over two
    primitive quartets (so the accumulation, not only one term, is compared)."""
    P = emit_deriv.deriv_program(*ls)
    full = _py(emit_deriv._vrr_weighted(P, ""))
    ref = {f"h{k}": 0.0 for k in range(len(P.acc_index))}
    envs = [_prim_env(ls, 7), _prim_env(ls, 8)]
    for e in envs:
        ref.update(e)
        exec(full, ref)
    stored = {}
    chunks = emit_deriv.stage_chunks(P, cap)
    assert max(sum(len(P.accs[P.g.target_ids[P.g.targets.index(t)]]) for t in ch) for ch in chunks) <= cap
    for ch in chunks:
        lines, ks, _, _ = emit_deriv.chunk_vrr(P, ch)
        env = {f"h{k}": 0.0 for k in ks}
        code = _py(lines)
        for e in envs:
            env.update(e)
            exec(code, env)
        for k in ks:
            assert k not in stored
            stored[k] = env[f"h{k}"]
    assert sorted(stored) == list(range(len(P.acc_index)))
    for k, v in stored.items():
        assert abs(v - ref[f"h{k}"]) <= 1e-14 * max(1.0, abs(ref[f"h{k}"])), k


def test_staged_source_shape():
    srcs, info = emit_deriv.emit_deriv_staged(2, 1, 2, 1, cap=96)
    assert info["parts"] == len(srcs) == (info["chunks"] + emit_deriv.STAGE_PART - 1) // emit_deriv.STAGE_PART
    assert "void launch_dp1_2121(const EriArgs &a, const int32_t *, int nseg, hipStream_t s)" in srcs[0]
    assert all(f"launch_dp1_2121p{p}(a, nseg, s);" in srcs[0] for p in srcs)
    n_store = sum(src.count(" * a.stride] = h") for src in srcs.values())
    assert n_store == info["n_acc"]
    assert all("double *__restrict__ S = a.scratch + (int64_t)s * 1548 * a.stride + i;" in src for src in srcs.values())
    table = emit_deriv.emit_deriv_table([(2, 1, 2, 1), (1, 0, 0, 0)], ["1000"], {"2121": 16})
    assert "&t3_d2121, nullptr, launch_dp1_2121, 16}" in table and "&t3_d1000, launch_dreg_1000, nullptr, 0}" in table


def test_segments_partition_the_primitive_loop():
    """The loop prelude's segment bounds (segment s of nseg covers t in
    [ntot s / nseg, ntot (s + 1) / nseg) of the flattened bra x ket
    primitive quartets) tile [0, ntot) in order, and the first record of
    every segment is in range; run on the emitted expressions (integer
    division, non-negative operands)."""
    from paper_2605_10312_amd.gen import emit
    lines = emit.loop_prelude(2, "", "late", weights=True, seg=True)
    seg = [ln.strip() for ln in lines if "t_lo =" in ln or "ip0 =" in ln]
    assert len(seg) == 2
    stmts = []
    for ln in seg:
        body = ln.split(";")[0].replace("const int ", "").replace("(int64_t)", "").replace("(int)", "")
        stmts.extend(x.strip().replace("/", "//") for x in body.split(", "))
    code = compile("\n".join(stmts), "<seg>", "exec")
    for nb in range(1, 7):
        for nkp in range(1, 7):
            ntot = nb * nkp
            for nseg in range(1, 17):
                covered = []
                for s_ in range(nseg):
                    env = {"ntot": ntot, "s": s_, "nseg": nseg, "nkp": nkp}
                    exec(code, env)
                    assert 0 <= env["t_lo"] <= env["t_hi"] <= ntot and env["t_lo"] < ntot
                    assert env["ip0"] < nb and env["jp0"] < nkp and env["ip0"] * nkp + env["jp0"] == env["t_lo"]
                    covered.extend(range(env["t_lo"], env["t_hi"]))
                assert covered == list(range(ntot))
