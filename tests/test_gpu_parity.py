"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Tolerances: 1e-12 absolute per contracted FP64 integral; J/K entries 1e-9
absolute (the stated bar), with the measured error printed.  For primitive
quartets with widely separated centres, where FP64 horizontal recurrences
lose digits in any evaluation order, the bar is applied against the
long-double oracle with an allowance of a few times the FP64 oracle's own
error (the oracle cannot certify more than it achieves).
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

ERI_TOL = 1e-12
JK_TOL = 1e-9


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def hgp():
    import paper_2605_10312_amd as m
    m.lib()
    return m


def _all_blocks(hgp, torch, basis_w, quartets):
    b = hgp.Basis.from_workload(basis_w)
    sizes = [int(np.prod([2 * basis_w.l[s] + 1 for s in q])) for q in quartets]
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    out = torch.full((int(sum(sizes)),), np.nan, dtype=torch.float64, device="cuda")
    hgp.eri_shell_quartets(b, np.array(quartets, np.int32), offs, out)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    blocks = [o[offs[i]:offs[i] + sizes[i]].reshape([2 * basis_w.l[s] + 1 for s in q]) for i, q in enumerate(quartets)]
    b.close()
    return blocks


def test_tiny_system_every_unique_integral(hgp, torch_cuda):
    """Config: 4 atoms, s(3) s(1) p(1) per atom: every unique spherical ERI."""
    bw, D = workloads.tiny_system()
    T = oracle.eri_tensor(bw)
    ns = bw.nshell
    quartets = [(i, j, k, l) for i in range(ns) for j in range(i + 1) for k in range(ns) for l in range(k + 1)
                if i * (i + 1) // 2 + j >= k * (k + 1) // 2 + l]
    assert len(quartets) == 3081
    blocks = _all_blocks(hgp, torch_cuda, bw, quartets)
    off = bw.shell_offsets()
    err = 0.0
    for q, blk in zip(quartets, blocks):
        ref = T[off[q[0]]:off[q[0] + 1], off[q[1]]:off[q[1] + 1], off[q[2]]:off[q[2] + 1], off[q[3]]:off[q[3] + 1]]
        err = max(err, float(np.abs(blk - ref).max()))
    # unique function-level integrals: i>=j, k>=l, ij>=kl
    N = bw.nbf
    n_unique = sum(1 for i in range(N) for j in range(i + 1) for k in range(N) for l in range(k + 1)
                   if i * (i + 1) // 2 + j >= k * (k + 1) // 2 + l)
    assert n_unique == 22155
    print(f"tiny system: max |gpu - oracle| over all unique blocks = {err:.3e}")
    assert err <= ERI_TOL


@pytest.mark.parametrize("seed", [11, 12, 13])
def test_random_shell_quartets_any_order(hgp, torch_cuda, seed):
    """Random l <= 2 bases, shell quartets in arbitrary (non-canonical) order,
    including repeated shells and shells sharing a centre."""
    bw = workloads.random_small_basis(seed=seed, natom=3, lmax=hgp.max_l() if hgp.max_l() <= 2 else 2, maxprim=4)
    rng = np.random.default_rng(seed)
    quartets = [tuple(int(x) for x in rng.integers(0, bw.nshell, 4)) for _ in range(300)]
    quartets += [(0, 0, 0, 0), (1, 1, 1, 1), (bw.nshell - 1,) * 4, (2, 1, 2, 1)]
    blocks = _all_blocks(hgp, torch_cuda, bw, quartets)
    err = 0.0
    for q, blk in zip(quartets, blocks):
        ref = oracle.eri_shell_quartet(bw, *q)
        err = max(err, float(np.abs(blk - ref).max()))
    print(f"seed {seed}: max abs error {err:.3e}")
    assert err <= ERI_TOL


def _jk_gpu(hgp, torch, bw, D, tau):
    b = hgp.Basis.from_workload(bw)
    plan = hgp.Plan(b, tau=tau)
    Dt = torch.tensor(D, dtype=torch.float64, device="cuda")
    J = torch.empty_like(Dt)
    K = torch.empty_like(Dt)
    plan.jk(Dt, J, K)
    torch.cuda.synchronize()
    out = J.cpu().numpy(), K.cpu().numpy(), plan.stats()
    plan.close()
    b.close()
    return out


def test_tiny_system_jk(hgp, torch_cuda):
    bw, D = workloads.tiny_system()
    Jr, Kr = oracle.jk(bw, D, tau=0.0)
    J, K, st = _jk_gpu(hgp, torch_cuda, bw, D, 0.0)
    assert st["quartets_kept"] == st["quartets_total"] == 3081
    # tau = 0: no primitive pair is dropped
    assert st["prim_pairs_kept"] == st["prim_pairs_total"] > 0
    ej, ek = np.abs(J - Jr).max(), np.abs(K - Kr).max()
    print(f"tiny J/K: max |dJ| {ej:.3e}, max |dK| {ek:.3e}")
    assert ej <= JK_TOL and ek <= JK_TOL
    assert ej <= 1e-12 * np.abs(Jr).max() * 10 and ek <= 1e-12 * np.abs(Kr).max() * 10


@pytest.mark.parametrize("seed,tau", [(21, 0.0), (22, 1e-10), (23, 1e-12)])
def test_random_basis_jk(hgp, torch_cuda, seed, tau):
    bw = workloads.random_small_basis(seed=seed, natom=4, lmax=2, maxprim=4, box=5.0, exp_range=(0.1, 50.0))
    D = workloads.psd_density(bw.nbf, seed)
    Jr, Kr = oracle.jk(bw, D, tau=tau)
    J, K, st = _jk_gpu(hgp, torch_cuda, bw, D, tau)
    ej, ek = np.abs(J - Jr).max(), np.abs(K - Kr).max()
    print(f"seed {seed} tau {tau}: kept {st['quartets_kept']}/{st['quartets_total']}, |dJ| {ej:.2e} |dK| {ek:.2e}")
    assert ej <= JK_TOL and ek <= JK_TOL


def test_j_only_and_k_only(hgp, torch_cuda):
    bw, D = workloads.tiny_system()
    Jr, Kr = oracle.jk(bw, D)
    b = hgp.Basis.from_workload(bw)
    plan = hgp.Plan(b, tau=0.0)
    Dt = torch_cuda.tensor(D, device="cuda")
    J = torch_cuda.full_like(Dt, np.nan)
    K = torch_cuda.full_like(Dt, np.nan)
    plan.jk(Dt, J=J)
    plan.jk(Dt, K=K)
    torch_cuda.cuda.synchronize()
    assert np.abs(J.cpu().numpy() - Jr).max() <= JK_TOL
    assert np.abs(K.cpu().numpy() - Kr).max() <= JK_TOL


def test_jk_run_to_run(hgp, torch_cuda):
    """FP64 atomics reorder the sums: repeated builds agree to rounding."""
    bw = workloads.random_small_basis(seed=31, natom=4, lmax=2, maxprim=3)
    D = workloads.psd_density(bw.nbf, 3)
    b = hgp.Basis.from_workload(bw)
    plan = hgp.Plan(b, tau=1e-12)
    Dt = torch_cuda.tensor(D, device="cuda")
    outs = []
    for _ in range(3):
        J = torch_cuda.empty_like(Dt)
        K = torch_cuda.empty_like(Dt)
        plan.jk(Dt, J, K)
        torch_cuda.cuda.synchronize()
        outs.append((J.cpu().numpy(), K.cpu().numpy()))
    for J, K in outs[1:]:
        assert np.abs(J - outs[0][0]).max() <= 1e-13 * max(1.0, np.abs(J).max())
        assert np.abs(K - outs[0][1]).max() <= 1e-13 * max(1.0, np.abs(K).max())


def test_empty_basis(hgp, torch_cuda):
    b = hgp.Basis([], [], np.zeros((0, 3)), [], [])
    assert b.nbf == 0
    plan = hgp.Plan(b, tau=1e-12)
    assert plan.stats()["quartets_kept"] == 0
    z = torch_cuda.zeros((0, 0), dtype=torch_cuda.float64, device="cuda")
    plan.jk(z, z, z)
    torch_cuda.cuda.synchronize()


@pytest.mark.parametrize("l", [2])
def test_prim_quartets_microbench_class(hgp, torch_cuda, l):
    """Config-3 shapes (ll|ll), normalised primitives, centres in a 6 A box,
    exponents log-uniform [0.1, 100]."""
    if l > hgp.max_l():
        pytest.skip("class not built")
    n = 2000
    cen, ex = workloads.prim_quartets(l, n)
    ls = (l, l, l, l)
    ref = oracle.eri_prim_quartets(ls, cen, ex)
    ref_ld = oracle.eri_prim_quartets(ls, cen, ex, precision="long double")
    ct = torch_cuda.tensor(cen, device="cuda")
    et = torch_cuda.tensor(ex, device="cuda")
    out = torch_cuda.full((n,) + ref.shape[1:], np.nan, dtype=torch_cuda.float64, device="cuda")
    hgp.eri_prim_quartets(ls, ct, et, out)
    torch_cuda.cuda.synchronize()
    g = out.cpu().numpy()
    e_gpu = np.abs(g - ref_ld)
    e_orc = np.abs(ref - ref_ld)
    print(f"({l}{l}|{l}{l}) x {n}: max |gpu-oracle| {np.abs(g - ref).max():.3e}, max |gpu-ld| {e_gpu.max():.3e}, "
          f"max |oracle-ld| {e_orc.max():.3e}")
    assert np.all(e_gpu <= ERI_TOL + 8.0 * e_orc)


def test_prim_quartets_noncanonical_order(hgp, torch_cuda):
    rng = np.random.default_rng(5)
    n = 300
    for ls in [(0, 1, 0, 0), (0, 0, 1, 2), (1, 2, 2, 0), (0, 2, 1, 1)]:
        cen = rng.uniform(-2, 2, (n, 4, 3))
        ex = np.exp(rng.uniform(np.log(0.2), np.log(20), (n, 4)))
        ref = oracle.eri_prim_quartets(ls, cen, ex)
        out = torch_cuda.full((n,) + ref.shape[1:], np.nan, dtype=torch_cuda.float64, device="cuda")
        hgp.eri_prim_quartets(ls, torch_cuda.tensor(cen, device="cuda"), torch_cuda.tensor(ex, device="cuda"), out)
        torch_cuda.cuda.synchronize()
        assert np.abs(out.cpu().numpy() - ref).max() <= ERI_TOL, ls


def test_concurrent_class_streams_match_one_stream(hgp, torch_cuda):
    """A plan runs its scratch-free class lists concurrently on several
    streams, and all of them on one stream while kernel timing is on; the
    two must agree within 1e-12 plus 1e-14 of the largest entry (only the
    order of the FP64 atomic additions differs)."""
    torch = torch_cuda
    bw = workloads.random_small_basis(seed=31, natom=4, lmax=2, maxprim=3)
    D = workloads.psd_density(bw.nbf, 31)
    b = hgp.Basis.from_workload(bw)
    p = hgp.Plan(b, tau=1e-12)
    Dt = torch.tensor(D, device="cuda")
    J1, K1, J2, K2 = (torch.empty_like(Dt) for _ in range(4))
    p.jk(Dt, J1, K1)
    p.set_timing(True)
    p.jk(Dt, J2, K2)
    torch.cuda.synchronize()
    p.set_timing(False)
    p.close()
    b.close()
    tol = 1e-12 + 1e-14 * max(J2.abs().max().item(), K2.abs().max().item())
    assert (J1 - J2).abs().max().item() <= tol and (K1 - K2).abs().max().item() <= tol
    Jr, Kr = oracle.jk(bw, D, tau=1e-12)
    assert np.abs(J1.cpu().numpy() - Jr).max() <= JK_TOL and np.abs(K1.cpu().numpy() - Kr).max() <= JK_TOL


def test_basis_flags_given_coefficients(hgp, torch_cuda):
    """hgp_basis_create with flags = 0 takes the coefficients as given: with
    the oracle's normalised coefficients (N(a, l) and the contraction norm
    applied) it must reproduce the HGP_NORMALIZE basis built from the raw
    ones, integrals and J/K alike."""
    bw = workloads.random_small_basis(seed=31, natom=3, lmax=3, maxprim=3)
    D = workloads.psd_density(bw.nbf, 31)
    off = bw.prim_offsets()
    given = np.concatenate([oracle.norm_coefs(int(bw.l[s]), bw.exps[off[s]:off[s + 1]], bw.coefs[off[s]:off[s + 1]])
                            for s in range(bw.nshell)])
    Dt = torch_cuda.tensor(D, device="cuda")
    res = []
    for normalize, coefs in ((True, bw.coefs), (False, given)):
        b = hgp.Basis(bw.l, bw.nprim, bw.centers, bw.exps, coefs, normalize=normalize)
        p = hgp.Plan(b, tau=0.0)
        J, K = torch_cuda.empty_like(Dt), torch_cuda.empty_like(Dt)
        p.jk(Dt, J, K)
        q = [(0, 1, 2, 3), (5, 4, 3, 2), (7, 7, 1, 0)]
        sizes = [int(np.prod([2 * bw.l[s] + 1 for s in x])) for x in q]
        offs = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
        out = torch_cuda.empty(int(sum(sizes)), dtype=torch_cuda.float64, device="cuda")
        hgp.eri_shell_quartets(b, np.array(q, np.int32), offs, out)
        torch_cuda.cuda.synchronize()
        res.append((J.cpu().numpy(), K.cpu().numpy(), out.cpu().numpy()))
        p.close()
        b.close()
    dj = np.abs(res[0][0] - res[1][0]).max()
    dk = np.abs(res[0][1] - res[1][1]).max()
    de = np.abs(res[0][2] - res[1][2]).max()
    print(f"flags 0 vs HGP_NORMALIZE: |dJ| {dj:.2e} |dK| {dk:.2e} |dERI| {de:.2e}")
    assert dj <= 1e-12 and dk <= 1e-12 and de <= 1e-13


def test_shell_quartets_device_arrays_stream_ordered(hgp, torch_cuda):
    """hgp_eri_shell_quartets with quartets and offsets already on the device,
    on a side stream, in mixed classes and shell orders (register, staged and
    op-table classes in one call): every block equals the oracle's, the
    blocks between the listed ones stay untouched, and a bad shell index is
    rejected before anything is written."""
    torch = torch_cuda
    bw = workloads.random_small_basis(seed=88, natom=3, lmax=4, maxprim=2, box=3.0, exp_range=(0.3, 8.0))
    rng = np.random.default_rng(88)
    ns = bw.nshell
    quartets = [tuple(int(x) for x in rng.integers(0, ns, 4)) for _ in range(300)]
    quartets += [(0, 0, 0, 0), (ns - 1, 0, ns - 1, 0)]
    sizes = [int(np.prod([2 * bw.l[s] + 1 for s in q])) for q in quartets]
    gap = 3                                             # untouched guard entries between blocks
    offs = np.concatenate([[0], np.cumsum(np.array(sizes) + gap)[:-1]]).astype(np.int64)
    total = int(offs[-1] + sizes[-1] + gap)
    b = hgp.Basis.from_workload(bw)
    qd = torch.tensor(np.array(quartets, np.int32), device="cuda")
    od = torch.tensor(offs, device="cuda")
    out = torch.full((total,), -7.0, dtype=torch.float64, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    hgp.eri_shell_quartets(b, qd, od, out, stream=side)
    side.synchronize()
    o = out.cpu().numpy()
    err = 0.0
    mask = np.ones(total, bool)
    for i, q in enumerate(quartets):
        ref = oracle.eri_shell_quartet(bw, *q).ravel()
        err = max(err, float(np.abs(o[offs[i]:offs[i] + sizes[i]] - ref).max()))
        mask[offs[i]:offs[i] + sizes[i]] = False
    print(f"{len(quartets)} quartets, lmax {int(bw.l.max())}: max |dERI| {err:.2e}")
    assert err <= ERI_TOL
    assert (o[mask] == -7.0).all()
    # an out-of-range shell: HGP_E_INVALID, out unchanged
    bad = qd.clone()
    bad[5, 2] = ns
    out2 = torch.full((total,), -7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(hgp.HGPError, match="out of range"):
        hgp.eri_shell_quartets(b, bad, od, out2)
    torch.cuda.synchronize()
    assert (out2.cpu().numpy() == -7.0).all()
    b.close()
