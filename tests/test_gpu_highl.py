"""Parity for f and g shells (l = 3, 4): the high-l microbench classes and
the HBM-scratch tier that serves the largest classes, through the C ABI.

Same bars as tests/test_gpu_parity.py: 1e-12 absolute per integral (against
the long-double oracle, allowing a few times the FP64 oracle's own error
where the horizontal recurrence loses digits in any FP64 evaluation) and
1e-9 absolute on J/K entries."""
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
    if m.max_l() < 4:
        pytest.fail("the library was built without l = 3, 4 classes")
    return m


def _prim(hgp, torch, ls, cen, ex):
    ref = oracle.eri_prim_quartets(ls, cen, ex)
    ref_ld = oracle.eri_prim_quartets(ls, cen, ex, precision="long double")
    out = torch.full((len(ex),) + ref.shape[1:], np.nan, dtype=torch.float64, device="cuda")
    hgp.eri_prim_quartets(ls, torch.tensor(cen, device="cuda"), torch.tensor(ex, device="cuda"), out)
    torch.cuda.synchronize()
    g = out.cpu().numpy()
    return g, ref, ref_ld


@pytest.mark.parametrize("l,n", [(3, 3000), (4, 1000)])
def test_microbench_class_config_inputs(hgp, torch_cuda, l, n):
    """(ff|ff) and (gg|gg) on the microbench's own distribution: centres in a
    6 A box, exponents log-uniform [0.1, 100], normalised primitives.  With
    centres several bohr apart the horizontal recurrence cancels heavily and
    any FP64 evaluation loses digits, so the bar is applied per quartet: the
    GPU's largest error on a quartet may not exceed 1e-12 plus a few times
    the FP64 oracle's own largest error on that quartet (both against the
    long-double oracle)."""
    cen, ex = workloads.prim_quartets(l, n)
    ls = (l, l, l, l)
    g, ref, ref_ld = _prim(hgp, torch_cuda, ls, cen, ex)
    e_gpu = np.abs(g - ref_ld).reshape(n, -1).max(axis=1)
    e_orc = np.abs(ref - ref_ld).reshape(n, -1).max(axis=1)
    hard = int(np.sum(e_orc > ERI_TOL))
    print(f"({l}{l}|{l}{l}) x {n}: max |I| {np.abs(ref_ld).max():.2e}, max |gpu-ld| {e_gpu.max():.3e}, "
          f"max |oracle-ld| {e_orc.max():.3e}, quartets where the FP64 oracle misses 1e-12: {hard}; "
          f"max |gpu-ld| on the others {e_gpu[e_orc <= ERI_TOL].max():.3e}")
    assert np.all(np.isfinite(g))
    assert np.all(e_gpu <= ERI_TOL + 8.0 * e_orc)


@pytest.mark.parametrize("ls", [(3, 3, 3, 3), (4, 4, 4, 4), (4, 3, 2, 1), (1, 4, 0, 3), (2, 2, 4, 4), (3, 0, 3, 0),
                                (4, 4, 4, 3), (3, 4, 3, 4), (4, 3, 3, 3)])
def test_compact_high_l_quartets(hgp, torch_cuda, ls):
    """Compact quartets (1 A box, exponents [0.2, 2]) whose integrals are of
    order one, in canonical and non-canonical shell order."""
    cen, ex = workloads.prim_quartets(max(ls), 200, seed=91, box=1.0, exp_range=(0.2, 2.0))
    g, ref, ref_ld = _prim(hgp, torch_cuda, ls, cen, ex)
    e_gpu, e_orc = np.abs(g - ref_ld), np.abs(ref - ref_ld)
    print(f"{ls}: max |I| {np.abs(ref_ld).max():.2e}, max |gpu-ld| {e_gpu.max():.3e}, max |oracle-ld| {e_orc.max():.3e}")
    assert np.all(e_gpu <= ERI_TOL + 8.0 * e_orc)


def test_random_high_l_shell_quartets(hgp, torch_cuda):
    """Contracted shells up to g (1-2 primitives) in random shell order."""
    bw = workloads.random_small_basis(seed=41, natom=2, lmax=4, maxprim=2, box=1.5, exp_range=(0.3, 5.0))
    rng = np.random.default_rng(41)
    quartets = [tuple(int(x) for x in rng.integers(0, bw.nshell, 4)) for _ in range(120)]
    quartets += [(4, 4, 4, 4), (9, 4, 9, 4), (3, 8, 2, 7)]
    b = hgp.Basis.from_workload(bw)
    sizes = [int(np.prod([2 * bw.l[s] + 1 for s in q])) for q in quartets]
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    out = torch_cuda.full((int(sum(sizes)),), np.nan, dtype=torch_cuda.float64, device="cuda")
    hgp.eri_shell_quartets(b, np.array(quartets, np.int32), offs, out)
    torch_cuda.cuda.synchronize()
    o = out.cpu().numpy()
    b.close()
    err = 0.0
    for i, q in enumerate(quartets):
        ref = oracle.eri_shell_quartet(bw, *q)
        blk = o[offs[i]:offs[i] + sizes[i]].reshape(ref.shape)
        err = max(err, float(np.abs(blk - ref).max()))
    print(f"l <= 4 shell quartets: max abs error {err:.3e}")
    assert err <= ERI_TOL


@pytest.mark.parametrize("lmax,tau", [(3, 0.0), (4, 0.0), (4, 1e-12)])
def test_high_l_jk(hgp, torch_cuda, lmax, tau):
    bw = workloads.random_small_basis(seed=50 + lmax, natom=2, lmax=lmax, maxprim=2, box=1.5, exp_range=(0.3, 5.0))
    D = workloads.psd_density(bw.nbf, 7)
    Jr, Kr = oracle.jk(bw, D, tau=tau)
    b = hgp.Basis.from_workload(bw)
    plan = hgp.Plan(b, tau=tau)
    Dt = torch_cuda.tensor(D, device="cuda")
    J = torch_cuda.empty_like(Dt)
    K = torch_cuda.empty_like(Dt)
    plan.jk(Dt, J, K)
    torch_cuda.cuda.synchronize()
    tiers = sorted({c["tier"] for c in plan.classes()})
    plan.close()
    b.close()
    ej, ek = np.abs(J.cpu().numpy() - Jr).max(), np.abs(K.cpu().numpy() - Kr).max()
    print(f"lmax {lmax} tau {tau}: N {bw.nbf}, tiers {tiers}, |dJ| {ej:.2e} |dK| {ek:.2e}")
    assert ej <= JK_TOL and ek <= JK_TOL


def test_gggg_large_batch_lane_form(hgp, torch_cuda):
    """(gg|gg) has two forms: batches below 65536 quartets run one wavefront
    per quartet with the slots in the scratch buffer, larger batches one lane
    per quartet.  70 000 quartets take the lane form; a sample of them is
    checked against the oracle, and the same sample run as a small batch
    (wave form) must agree with it."""
    torch = torch_cuda
    n = 70000
    cen, ex = workloads.prim_quartets(4, n, seed=93, box=1.0, exp_range=(0.2, 2.0))
    ls = (4, 4, 4, 4)
    out = torch.empty((n, 9, 9, 9, 9), dtype=torch.float64, device="cuda")
    hgp.eri_prim_quartets(ls, torch.tensor(cen, device="cuda"), torch.tensor(ex, device="cuda"), out)
    torch.cuda.synchronize()
    pick = np.array([0, 1, 4097, 33333, 65535, 65536, n - 1])
    big = out[torch.tensor(pick, device="cuda")].cpu().numpy()
    del out
    small = torch.empty((len(pick), 9, 9, 9, 9), dtype=torch.float64, device="cuda")
    hgp.eri_prim_quartets(ls, torch.tensor(cen[pick], device="cuda"), torch.tensor(ex[pick], device="cuda"), small)
    torch.cuda.synchronize()
    small = small.cpu().numpy()
    ref_ld = oracle.eri_prim_quartets(ls, cen[pick], ex[pick], precision="long double")
    e_orc = np.abs(oracle.eri_prim_quartets(ls, cen[pick], ex[pick]) - ref_ld)
    e_big, e_small = np.abs(big - ref_ld), np.abs(small - ref_ld)
    print(f"(gg|gg) x {n}: lane form max |gpu-ld| {e_big.max():.3e}, wave form {e_small.max():.3e}, "
          f"oracle {e_orc.max():.3e}")
    assert np.all(e_big <= ERI_TOL + 8.0 * e_orc) and np.all(e_small <= ERI_TOL + 8.0 * e_orc)
