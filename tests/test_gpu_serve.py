"""Serving (continuous batching on several streams, plans reused across
closed-loop density updates, HBM-budget admission): every served J/K must
equal what the same plan gives for that density alone, 1e-12 absolute plus
1e-14 of the largest entry (only the order of FP64 atomic additions
differs); for mixed plans also within 1e-9 of the FP64 plan alone."""
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


def _requests(serve, n, nupd, lmax, theta, seed):
    systems = workloads.batch_systems(seed=seed, n=n, natom=(1, 3), lmax=lmax, nprim=(1, 2))
    arrivals = serve.poisson_arrivals(400.0, n, seed)
    reqs = []
    for i, (bw, D) in enumerate(systems):
        dens = [D] + [workloads.psd_density(bw.nbf, seed + 100 * i + k) for k in range(1, nupd)]
        reqs.append(serve.Request(i, float(arrivals[i]), bw, dens, tau=1e-12, theta=theta))
    return reqs


def _alone(hgp, torch, r, theta):
    """Each update of request r through its own plan, one at a time; also the
    bytes the server charges for it."""
    b = hgp.Basis.from_workload(r.basis)
    p = hgp.Plan(b, tau=r.tau, theta=theta)
    out = []
    for D in r.densities:
        Dt = torch.tensor(D, device="cuda")
        J, K = torch.empty_like(Dt), torch.empty_like(Dt)
        p.jk(Dt, J, K)
        torch.cuda.synchronize()
        out.append((J.cpu().numpy(), K.cpu().numpy()))
    n = r.basis.nbf
    nbytes = p.stats()["device_bytes"] + 8 * n * n * (len(r.densities) + 2)
    p.close()
    b.close()
    return out, nbytes


@pytest.mark.parametrize("theta,worker", [(0.0, False), (1e-10, False), (0.0, True)])
def test_served_equals_alone(hgp, torch_cuda, theta, worker):
    from paper_2605_10312_amd import serve
    reqs = _requests(serve, 8, 3, lmax=4, theta=theta, seed=1005)
    alone = [_alone(hgp, torch_cuda, r, theta) for r in reqs]
    sizes = sorted(a[1] for a in alone)
    budget = sizes[-1] + sizes[-2]                  # the two largest plans fit together, not three
    ex = serve.GpuExecutor(slots=4, keep=True, worker=worker)
    srv = serve.Server(ex, hbm_budget=budget, max_active=4, slots=4)
    recs, ups = srv.run(reqs)
    ex.close()
    assert all(r.rejected is None for r in recs) and len(ups) == 24
    assert srv.peak_bytes <= budget
    worst = 0.0
    for r, (res, _) in zip(reqs, alone):
        for k in range(3):
            J, K = ex.results[(r.rid, k)]
            worst = max(worst, np.abs(J - res[k][0]).max(), np.abs(K - res[k][1]).max())
    s = serve.summarize(recs, ups, max(u.done for u in ups))
    tol = same_tol([x for a in alone for x in a[0]])
    print(f"theta {theta} worker {worker}: N = {[r.basis.nbf for r in reqs]}, peak active {srv.peak_active}, "
          f"max |served - alone| {worst:.2e}, update p50/p99 {s['update_p50_ms']:.2f}/{s['update_p99_ms']:.2f} ms")
    assert worst <= tol
    if theta > 0:
        # the mixed results against the FP64 plan alone, and the smallest system against the oracle
        err = 0.0
        for r in reqs[:3]:
            ref, _ = _alone(hgp, torch_cuda, r, 0.0)
            J, K = ex.results[(r.rid, 2)]
            err = max(err, np.abs(J - ref[2][0]).max(), np.abs(K - ref[2][1]).max())
        print(f"mixed vs FP64: {err:.2e}")
        assert err <= JK_TOL
    small = min(reqs, key=lambda r: r.basis.nbf)
    Jr, Kr = oracle.jk(small.basis, small.densities[1], tau=small.tau)
    J, K = ex.results[(small.rid, 1)]
    assert np.abs(J - Jr).max() <= JK_TOL and np.abs(K - Kr).max() <= JK_TOL


def test_iteration_served_equals_alone(hgp, torch_cuda):
    """Iteration-level batching: every step one multi-system plan over the
    active requests; each served J/K equals its own plan alone (1e-12)."""
    from paper_2605_10312_amd import serve
    reqs = _requests(serve, 8, 3, lmax=4, theta=0.0, seed=1006)
    for r in reqs[::3]:
        r.densities = r.densities[:2]                 # uneven update counts: the active set changes
    alone = [_alone(hgp, torch_cuda, r, 0.0) for r in reqs]
    ex = serve.GpuMultiExecutor(keep=True)
    srv = serve.IterationServer(ex, hbm_budget=8 << 30, max_active=4)
    recs, ups = srv.run(reqs)
    ex.close()
    assert all(r.rejected is None for r in recs)
    assert len(ups) == sum(len(r.densities) for r in reqs)
    worst = 0.0
    for r, (res, _) in zip(reqs, alone):
        for k in range(len(r.densities)):
            J, K = ex.results[(r.rid, k)]
            worst = max(worst, np.abs(J - res[k][0]).max(), np.abs(K - res[k][1]).max())
    print(f"iteration server: peak active {srv.peak_active}, rebuilds {srv.rebuilds}, max |served - alone| {worst:.2e}")
    assert worst <= same_tol([x for a in alone for x in a[0]]) and srv.peak_active == 4


def _multi_need(hgp, reqs):
    """Bytes GpuMultiExecutor charges for one multi-system plan over reqs:
    the plan's device bytes plus each request's densities and J, K."""
    bases = [hgp.Basis.from_workload(r.basis) for r in reqs]
    p = hgp.Plan.multi(bases, tau=reqs[0].tau)
    need = p.stats()["device_bytes"] + sum(8 * r.basis.nbf ** 2 * (len(r.densities) + 2) for r in reqs)
    p.close()
    for b in bases:
        b.close()
    return need


def test_iteration_budget_pushes_back_and_rejects(hgp, torch_cuda):
    """Iteration-level batching under a budget that holds each small request
    alone but not all of them together, and not the one large request even
    alone: the large request is rejected (its device data freed), requests
    that do not fit beside the others are sent back to the queue and run
    later, and every served result equals its own plan alone."""
    from paper_2605_10312_amd import serve
    systems = workloads.batch_systems(seed=1007, n=5, natom=(1, 2), lmax=3, nprim=(1, 2))
    systems += workloads.batch_systems(seed=1008, n=1, natom=(6, 6), lmax=3, nprim=(2, 2))
    reqs = [serve.Request(i, 0.0, bw, [D, workloads.psd_density(bw.nbf, 77 + i)], tau=1e-12, theta=0.0)
            for i, (bw, D) in enumerate(systems)]
    alone = [_alone(hgp, torch_cuda, r, 0.0) for r in reqs]
    big = len(reqs) - 1
    single = max(_multi_need(hgp, [r]) for r in reqs[:big])
    all_small = _multi_need(hgp, reqs[:big])
    budget = int(single * 1.05)
    assert all_small > budget and _multi_need(hgp, [reqs[big]]) > budget
    ex = serve.GpuMultiExecutor(keep=True)
    srv = serve.IterationServer(ex, hbm_budget=budget, max_active=6)
    recs, ups = srv.run(reqs)
    assert ex.dev == {}                               # finished, pushed-back and rejected data all freed
    ex.close()
    assert recs[big].rejected is not None
    assert all(r.rejected is None for i, r in enumerate(recs) if i != big)
    assert srv.peak_active < 5                        # not every request fitted at once
    worst = 0.0
    for i, (r, (res, _)) in enumerate(zip(reqs, alone)):
        if i == big:
            continue
        for k in range(2):
            J, K = ex.results[(r.rid, k)]
            worst = max(worst, np.abs(J - res[k][0]).max(), np.abs(K - res[k][1]).max())
    print(f"budget {budget / 2**20:.1f} MiB (all five small together {all_small / 2**20:.1f} MiB): rejected "
          f"request {big}, peak active {srv.peak_active}, rebuilds {srv.rebuilds}, max |served - alone| {worst:.2e}")
    assert worst <= same_tol([x for i, a in enumerate(alone) if i != big for x in a[0]])
