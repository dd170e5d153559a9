"""Streamed class lists: a plan whose quartet lists do not fit its HBM budget
keeps per bra row the offset of its first kept quartet and re-screens the
rows chunk by chunk into one buffer on every build.  The same quartets run
in the same order, so J/K equal the stored-list plan's (the FP64 atomics'
order aside: 1e-12) and the oracle's (1e-9), eagerly, repeatedly and in a
captured graph; and a budget below one chunk of the longest row is refused."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu
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


def _run(hgp, torch, plan, D):
    Dt = torch.tensor(D, device="cuda")
    J, K = torch.empty_like(Dt), torch.empty_like(Dt)
    plan.jk(Dt, J, K)
    torch.cuda.synchronize()
    return J.cpu().numpy(), K.cpu().numpy()


@pytest.mark.parametrize("seed,natom,lmax,tau", [(301, 8, 2, 1e-12), (302, 6, 3, 0.0)])
def test_streamed_plan_matches_stored(hgp, torch_cuda, seed, natom, lmax, tau):
    bw = workloads.random_small_basis(seed=seed, natom=natom, lmax=lmax, maxprim=3, box=5.0, exp_range=(0.2, 20.0))
    D = workloads.psd_density(bw.nbf, seed)
    b = hgp.Basis.from_workload(bw)
    full = hgp.Plan(b, tau=tau)
    st = full.stats()
    assert st["quartets_streamed"] == 0 and st["chunk_capacity"] == 0
    J0, K0 = _run(hgp, torch_cuda, full, D)
    nonlist = st["device_bytes"] - 8 * st["quartets_kept"]
    # room for a tenth of the lists: the smallest stored, the rest streamed in chunks
    budget = nonlist + 8 * (st["quartets_kept"] // 10)
    sp = hgp.Plan(b, tau=tau, hbm_budget=budget)
    ss = sp.stats()
    print(f"seed {seed}: kept {st['quartets_kept']}, streamed {ss['quartets_streamed']} in {ss['stream_chunks']} "
          f"chunks of <= {ss['chunk_capacity']}, bytes {ss['device_bytes']} <= budget {budget}")
    assert ss["quartets_kept"] == st["quartets_kept"]
    assert ss["quartets_streamed"] > st["quartets_kept"] // 2 and ss["stream_chunks"] > 3
    assert ss["device_bytes"] <= budget
    for rep in range(2):
        J, K = _run(hgp, torch_cuda, sp, D)
        assert np.abs(J - J0).max() <= 1e-12 and np.abs(K - K0).max() <= 1e-12, rep
    Jr, Kr = oracle.jk(bw, D, tau=tau)
    assert np.abs(J - Jr).max() <= JK_TOL and np.abs(K - Kr).max() <= JK_TOL
    # the streamed plan in a captured graph, replayed twice
    torch = torch_cuda
    Dt = torch.tensor(D, device="cuda")
    Jg, Kg = torch.empty_like(Dt), torch.empty_like(Dt)
    g = hgp.Batch([sp], [Dt], [Jg], [Kg])
    for rep in range(2):
        Jg.fill_(7.0)
        g.run()
        torch.cuda.synchronize()
        assert np.abs(Jg.cpu().numpy() - J0).max() <= 1e-12 and np.abs(Kg.cpu().numpy() - K0).max() <= 1e-12, rep
    g.close()
    sp.close()
    full.close()
    # below the non-list bytes plus one row's chunk: refused
    with pytest.raises(hgp.HGPError, match="budget"):
        hgp.Plan(b, tau=tau, hbm_budget=nonlist + 64)
    b.close()
