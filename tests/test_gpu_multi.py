"""Several systems in one plan (hgp_plan_create_multi / hgp_jk_multi): each
class runs once over the quartets of every system.  Screening (primitive
pairs included) is decided per system, so the plan evaluates exactly the
quartets and primitive pairs of the systems' own plans: every system's J/K
must equal its own plan's within 1e-12 plus 1e-14 of the largest entry (only
the order of the FP64 atomic additions differs), the counts must add up, and quartets never cross
systems."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

SAME_TOL = 1e-12
JK_TOL = 1e-9


def same_tol(results):
    """Bar for the same terms summed in another order: 1e-12 absolute plus
    1e-14 of the largest entry (the classes run concurrently and the FP64
    atomic additions land in a different order)."""
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


def _alone(hgp, torch, bw, D, tau):
    b = hgp.Basis.from_workload(bw)
    p = hgp.Plan(b, tau=tau)
    Dt = torch.tensor(D, device="cuda")
    J, K = torch.empty_like(Dt), torch.empty_like(Dt)
    p.jk(Dt, J, K)
    torch.cuda.synchronize()
    st = p.stats()
    p.close()
    b.close()
    return J.cpu().numpy(), K.cpu().numpy(), st


@pytest.mark.parametrize("lmax,tau", [(2, 0.0), (3, 0.0), (4, 0.0), (3, 1e-12)])
def test_multi_plan_equals_each_system(hgp, torch_cuda, lmax, tau):
    torch = torch_cuda
    systems = workloads.batch_systems(seed=2000 + lmax, n=5, natom=(1, 4), lmax=lmax, nprim=(1, 2))
    alone = [_alone(hgp, torch, bw, D, tau) for bw, D in systems]
    bases = [hgp.Basis.from_workload(bw) for bw, _ in systems]
    plan = hgp.Plan.multi(bases, tau=tau)
    for b in bases:                       # the plan holds its own copy of the shells
        b.close()
    Ds = [torch.tensor(D, device="cuda") for _, D in systems]
    Js = [torch.full_like(D, np.nan) for D in Ds]
    Ks = [torch.full_like(D, np.nan) for D in Ds]
    for rep in range(2):                  # the second call must not see the first's accumulators
        plan.jk_multi(Ds, Js, Ks)
        torch.cuda.synchronize()
    st = plan.stats()
    worst = max(max(np.abs(J.cpu().numpy() - a[0]).max(), np.abs(K.cpu().numpy() - a[1]).max())
                for J, K, a in zip(Js, Ks, alone))
    tol = same_tol(alone)
    print(f"lmax {lmax} tau {tau}: N = {[bw.nbf for bw, _ in systems]}, kept {st['quartets_kept']} "
          f"(alone {sum(a[2]['quartets_kept'] for a in alone)}), max |multi - alone| {worst:.2e}")
    assert st["quartets_total"] == sum(a[2]["quartets_total"] for a in alone)
    assert st["quartets_kept"] == sum(a[2]["quartets_kept"] for a in alone)
    assert st["prim_pairs_kept"] == sum(a[2]["prim_pairs_kept"] for a in alone)
    assert worst <= tol
    small = int(np.argmin([bw.nbf for bw, _ in systems]))
    Jr, Kr = oracle.jk(systems[small][0], systems[small][1], tau=tau)
    assert np.abs(Js[small].cpu().numpy() - Jr).max() <= JK_TOL
    assert np.abs(Ks[small].cpu().numpy() - Kr).max() <= JK_TOL
    # only J, then only K
    Jo = [torch.full_like(D, np.nan) for D in Ds]
    plan.jk_multi(Ds, Jo, None)
    Ko = [torch.full_like(D, np.nan) for D in Ds]
    plan.jk_multi(Ds, None, Ko)
    torch.cuda.synchronize()
    for a, b in zip(Jo, Js):
        assert (a - b).abs().max().item() <= tol
    for a, b in zip(Ko, Ks):
        assert (a - b).abs().max().item() <= tol
    plan.close()


def test_multi_plan_errors(hgp, torch_cuda):
    torch = torch_cuda
    systems = workloads.batch_systems(seed=2100, n=2, natom=(1, 2), lmax=2, nprim=(1, 1))
    bases = [hgp.Basis.from_workload(bw) for bw, _ in systems]
    plan = hgp.Plan.multi(bases, tau=0.0)
    D = torch.tensor(systems[0][1], device="cuda")
    with pytest.raises(hgp.HGPError, match="hgp_jk_multi"):
        plan.jk(D, torch.empty_like(D))
    plan.close()
    one = hgp.Plan.multi(bases[:1], tau=0.0)          # one system: the plain path
    J1 = torch.empty_like(D)
    one.jk_multi([D], [J1], None)
    ref = _alone(hgp, torch, systems[0][0], systems[0][1], 0.0)
    torch.cuda.synchronize()
    assert np.abs(J1.cpu().numpy() - ref[0]).max() <= same_tol([ref])
    one.close()
    for b in bases:
        b.close()
