"""Batched J/K over several systems of uneven size, captured as one HIP graph
(hgp_batch_*): every replay must give each system what its own plan gives
alone, the replays must follow the current densities, and eager work between
replays must not disturb them.

Bars: 1e-12 absolute plus 1e-14 of the largest entry between the batched
and the per-system results of the same plans (only the order of the FP64
atomic additions differs), 1e-9 absolute against the oracle on the systems
small enough for it."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

SAME_TOL = 1e-12
JK_TOL = 1e-9


def same_tol(results):
    """Bar for the same terms summed in another order: 1e-12 absolute plus
    1e-14 of the largest entry (a plan runs its classes concurrently, so the
    FP64 atomic additions land in a different order from run to run)."""
    big = max(max(np.abs(r[0]).max(), np.abs(r[1]).max()) for r in results)
    return SAME_TOL + 1e-14 * big


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


def _setup(hgp, torch, systems, tau, theta=0.0):
    bases, plans, Ds, Js, Ks = [], [], [], [], []
    for bw, D in systems:
        b = hgp.Basis.from_workload(bw)
        bases.append(b)
        plans.append(hgp.Plan(b, tau=tau, theta=theta))
        Dt = torch.tensor(D, device="cuda")
        Ds.append(Dt)
        Js.append(torch.full_like(Dt, np.nan))
        Ks.append(torch.full_like(Dt, np.nan))
    return bases, plans, Ds, Js, Ks


def _alone(torch, plans, Ds):
    out = []
    for p, D in zip(plans, Ds):
        J, K = torch.empty_like(D), torch.empty_like(D)
        p.jk(D, J, K)
        torch.cuda.synchronize()
        out.append((J.cpu().numpy(), K.cpu().numpy()))
    return out


def _close(objs):
    for o in objs:
        o.close()


@pytest.mark.parametrize("lmax,tau", [(2, 0.0), (3, 1e-12)])
def test_batch_matches_each_system_alone(hgp, torch_cuda, lmax, tau):
    """Nine systems of 1-4 atoms (uneven sizes, more systems than branches)."""
    systems = workloads.batch_systems(seed=1004, n=9, natom=(1, 4), lmax=lmax, nprim=(1, 2))
    bases, plans, Ds, Js, Ks = _setup(hgp, torch_cuda, systems, tau)
    ref = _alone(torch_cuda, plans, Ds)
    batch = hgp.Batch(plans, Ds, Js, Ks)
    batch.run()
    torch_cuda.cuda.synchronize()
    worst = 0.0
    for i, (J, K) in enumerate(zip(Js, Ks)):
        worst = max(worst, np.abs(J.cpu().numpy() - ref[i][0]).max(), np.abs(K.cpu().numpy() - ref[i][1]).max())
    # the smallest system also against the oracle
    small = int(np.argmin([bw.nbf for bw, _ in systems]))
    Jr, Kr = oracle.jk(systems[small][0], systems[small][1], tau=tau)
    ej = np.abs(Js[small].cpu().numpy() - Jr).max()
    ek = np.abs(Ks[small].cpu().numpy() - Kr).max()
    print(f"lmax {lmax}: N = {[bw.nbf for bw, _ in systems]}, max |batch - alone| {worst:.2e}, "
          f"system {small} vs oracle |dJ| {ej:.2e} |dK| {ek:.2e}")
    batch.close()
    _close(plans + bases)
    assert worst <= same_tol(ref)
    assert ej <= JK_TOL and ek <= JK_TOL


def test_batch_replays_follow_density_and_survive_eager_work(hgp, torch_cuda):
    torch = torch_cuda
    systems = workloads.batch_systems(seed=7, n=5, natom=(1, 3), lmax=2, nprim=(1, 3))
    bases, plans, Ds, Js, Ks = _setup(hgp, torch, systems, 1e-12)
    ref = _alone(torch, plans, Ds)
    batch = hgp.Batch(plans, Ds, Js[:3] + [None, None], [None] + Ks[1:])
    scale = [1.0, -0.5, 3.0]
    prev = 1.0
    for r, sc in enumerate(scale):
        for D in Ds:                       # eager work on the stream between replays
            D.mul_(sc / prev)
        prev = sc
        noise = torch.randn(256, 256, device="cuda", dtype=torch.float64)
        _ = (noise @ noise).sum().item()
        for J in Js[3:]:
            J.fill_(7.0)                   # J not requested for these systems: must stay untouched
        for K in Ks[:1]:
            K.fill_(7.0)
        batch.run()
        torch.cuda.synchronize()
        worst = 0.0
        for i in range(len(systems)):
            if i < 3:
                worst = max(worst, np.abs(Js[i].cpu().numpy() - sc * ref[i][0]).max())
            else:
                assert np.all(Js[i].cpu().numpy() == 7.0)
            if i >= 1:
                worst = max(worst, np.abs(Ks[i].cpu().numpy() - sc * ref[i][1]).max())
            else:
                assert np.all(Ks[i].cpu().numpy() == 7.0)
        print(f"replay {r} (D x {sc}): max |batch - scaled alone| {worst:.2e}")
        assert worst <= same_tol(ref) * max(1.0, abs(sc))
    # a plan of the batch still runs alone between replays, with the same result
    for D in Ds:
        D.div_(prev)
    again = _alone(torch, plans, Ds)
    for a, b in zip(again, ref):
        assert np.abs(a[0] - b[0]).max() <= same_tol(ref) and np.abs(a[1] - b[1]).max() <= same_tol(ref)
    batch.close()
    _close(plans + bases)


def test_batch_mixed_precision_plans(hgp, torch_cuda):
    systems = workloads.batch_systems(seed=11, n=4, natom=(2, 4), lmax=2, nprim=(1, 3))
    bases, plans, Ds, Js, Ks = _setup(hgp, torch_cuda, systems, 1e-12, theta=1e-6)
    ref = _alone(torch_cuda, plans, Ds)
    batch = hgp.Batch(plans, Ds, Js, Ks)
    for _ in range(2):
        batch.run()
        torch_cuda.cuda.synchronize()
        worst = max(max(np.abs(J.cpu().numpy() - r[0]).max(), np.abs(K.cpu().numpy() - r[1]).max())
                    for J, K, r in zip(Js, Ks, ref))
        assert worst <= same_tol(ref)
    batch.close()
    _close(plans + bases)


def test_batch_rejects_bad_arguments(hgp, torch_cuda):
    systems = workloads.batch_systems(seed=3, n=2, natom=(1, 2), lmax=2, nprim=(1, 1))
    bases, plans, Ds, Js, Ks = _setup(hgp, torch_cuda, systems, 0.0)
    with pytest.raises(hgp.HGPError, match="twice"):
        hgp.Batch([plans[0], plans[0]], Ds[:1] * 2, Js[:1] * 2, Ks[:1] * 2)
    plans[1].set_timing(True)
    with pytest.raises(hgp.HGPError, match="timing"):
        hgp.Batch(plans, Ds, Js, Ks)
    plans[1].set_timing(False)
    with pytest.raises(hgp.HGPError, match="no D or no output"):
        hgp.Batch(plans, Ds, [None, None], [None, None])
    b = hgp.Batch(plans, Ds, Js, Ks)       # still fine afterwards
    b.run()
    torch_cuda.cuda.synchronize()
    b.close()
    _close(plans + bases)
