"""First-derivative integrals on the GPU (hgp_eri_deriv_shell_quartets)
against the oracle's derivative integrals, which are pinned to finite
differences and translational invariance (tests/test_oracle_deriv.py).
Tolerance, against the long-double oracle: 1e-12 of the largest derivative
in the sample (a block whose exact value is zero, e.g. four shells on one
centre, is a cancellation of terms of that magnitude) plus 8 times the FP64
oracle's own error on the block (contracted (dd|dd) derivatives cancel
enough to cost the FP64 oracle about 1e-12), as for the integrals."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


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


def _run(hgp, torch, bw, quartets, stream=None):
    b = hgp.Basis.from_workload(bw)
    sizes = [12 * int(np.prod([2 * bw.l[s] + 1 for s in q])) for q in quartets]
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    out = torch.full((int(sum(sizes)),), np.nan, dtype=torch.float64, device="cuda")
    hgp.eri_shell_quartets(b, np.array(quartets, np.int32), offs, out, deriv=True, stream=stream)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    b.close()
    return [o[offs[i]:offs[i] + sizes[i]].reshape([4, 3] + [2 * bw.l[s] + 1 for s in q])
            for i, q in enumerate(quartets)]


@pytest.mark.parametrize("seed,maxprim", [(401, 1), (402, 3)])
def test_deriv_random_quartets_any_order(hgp, torch_cuda, seed, maxprim):
    """Random shell quartets of an l <= 2 basis, in any shell order and with
    repeated shells, contracted shells up to three primitives."""
    assert hgp.deriv_max_l() >= 2
    bw = workloads.random_small_basis(seed=seed, natom=3, lmax=2, maxprim=maxprim, box=3.0, exp_range=(0.2, 8.0))
    rng = np.random.default_rng(seed)
    ns = bw.nshell
    quartets = [tuple(int(x) for x in rng.integers(0, ns, 4)) for _ in range(60)]
    quartets += [(0, 0, 0, 0), (ns - 1, ns - 1, ns - 1, ns - 1), (2, 5, 2, 5)]
    got = _run(hgp, torch_cuda, bw, quartets)
    refs = [oracle.eri_deriv_shell_quartet(bw, *q, precision="long double") for q in quartets]
    scale = max(np.abs(r).max() for r in refs)
    worst = 0.0
    for q, g, ref in zip(quartets, got, refs):
        e_orc = np.abs(oracle.eri_deriv_shell_quartet(bw, *q) - ref).max()
        err = np.abs(g - ref).max()
        worst = max(worst, err)
        assert err <= 1e-12 * scale + 8 * e_orc, (q, err, scale, e_orc)
        # translational invariance holds on the GPU's own values too
        assert np.abs(g.sum(axis=0)).max() <= 1e-12 * scale
    print(f"seed {seed}: {len(quartets)} quartets, max |d| {scale:.2e}, worst |d - oracle| {worst:.2e}")


def test_deriv_rejects_g_and_bad_index(hgp, torch_cuda):
    bw = workloads.random_small_basis(seed=403, natom=2, lmax=3, maxprim=1, box=2.0)
    f_shell = int(np.nonzero(bw.l == 3)[0][0])
    with pytest.raises(hgp.HGPError, match="derivative integrals are built"):
        _run(hgp, torch_cuda, bw, [(f_shell, 0, 0, 0)])
    b = hgp.Basis.from_workload(bw)
    out = torch_cuda.full((12 * 7 ** 4,), -3.0, dtype=torch_cuda.float64, device="cuda")
    with pytest.raises(hgp.HGPError, match="out of range"):
        hgp.eri_shell_quartets(b, np.array([(0, 0, 0, bw.nshell)], np.int32), np.zeros(1, np.int64), out, deriv=True)
    torch_cuda.cuda.synchronize()
    assert (out.cpu().numpy() == -3.0).all()                # nothing written
    b.close()


def test_deriv_register_and_staged_forms_agree_at_scale(hgp, torch_cuda):
    """A class with both forms runs the register form from 65 536 quartets on
    and the staged form (segmented primitive loops) below: 40 distinct
    quartets of four register-form classes, repeated to 68 000 and to 750
    quartets of each class, give the oracle's blocks in every copy."""
    bw = workloads.random_small_basis(seed=404, natom=3, lmax=2, maxprim=3, box=3.0, exp_range=(0.2, 8.0))
    rng = np.random.default_rng(404)
    L = np.asarray(bw.l)
    s_sh, p_sh, d_sh = (np.nonzero(L == l)[0] for l in range(3))
    pick = lambda a: int(rng.choice(a))
    # (ps|ps), (ds|ps), (dp|ss) and (ps|ss) in shuffled shell orders
    base = []
    for _ in range(10):
        base += [(pick(p_sh), pick(s_sh), pick(p_sh), pick(s_sh)), (pick(s_sh), pick(d_sh), pick(p_sh), pick(s_sh)),
                 (pick(d_sh), pick(p_sh), pick(s_sh), pick(s_sh)), (pick(s_sh), pick(s_sh), pick(s_sh), pick(p_sh))]
    refs = [oracle.eri_deriv_shell_quartet(bw, *q, precision="long double") for q in base]
    scale = max(np.abs(r).max() for r in refs)
    for copies in (1700, 75):
        quartets = base * copies
        got = _run(hgp, torch_cuda, bw, quartets)
        worst = 0.0
        for i, g in enumerate(got):
            worst = max(worst, np.abs(g - refs[i % len(base)]).max())
        assert worst <= 1e-12 * scale, (copies, worst, scale)
        print(f"{len(quartets)} quartets: worst |d - oracle| {worst:.2e} (max |d| {scale:.2e})")


def test_deriv_full_size_sample(hgp, torch_cuda):
    """The timed derivative workload at its full size and launch shape: 400 000
    uniformly drawn screened unique shell quartets of the 30-atom 3s2p1d
    molecule (tau 1e-12) in one call, device arrays.  64 sampled quartets
    against the long-double oracle (1e-12 of the sample's largest derivative
    plus 8 times the FP64 oracle's own error), translational invariance on
    4 000 sampled blocks, and every value finite."""
    torch = torch_cuda
    bw, _ = workloads.molecule_3s2p1d()
    Q = oracle.schwarz(bw)
    ns = bw.nshell
    rng = np.random.default_rng(2005)
    want, picked = 400000, []
    while len(picked) < want:
        q = rng.integers(0, ns, (4 * want, 4))
        i, j, k, l = q.T
        keep = (i >= j) & (k >= l) & (i * (i + 1) // 2 + j >= k * (k + 1) // 2 + l) & (Q[i, j] * Q[k, l] >= 1e-12)
        picked.extend(map(tuple, q[keep][: want - len(picked)]))
    quartets = np.array(picked, np.int32)
    L = np.asarray(bw.l)
    sizes = 12 * np.prod(2 * L[quartets] + 1, axis=1).astype(np.int64)
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    b = hgp.Basis.from_workload(bw)
    out = torch.full((int(sizes.sum()),), np.nan, dtype=torch.float64, device="cuda")
    hgp.eri_shell_quartets(b, torch.tensor(quartets, device="cuda"), torch.tensor(offs, device="cuda"), out,
                           deriv=True)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(out).all())
    o = out.cpu().numpy()
    b.close()
    chk = rng.choice(len(quartets), 64, replace=False)
    refs = [oracle.eri_deriv_shell_quartet(bw, *quartets[i], precision="long double") for i in chk]
    scale = max(np.abs(r).max() for r in refs)
    worst, at = 0.0, None
    for i, ref in zip(chk, refs):
        g = o[offs[i]:offs[i] + sizes[i]].reshape(ref.shape)
        e_orc = np.abs(oracle.eri_deriv_shell_quartet(bw, *quartets[i]) - ref).max()
        err = np.abs(g - ref).max()
        if err > worst:
            worst, at = err, (tuple(int(x) for x in quartets[i]), [int(L[x]) for x in quartets[i]], e_orc,
                              float(np.abs(ref).max()))
        assert err <= 1e-12 * scale + 8 * e_orc, (tuple(quartets[i]), err, scale, e_orc)
    inv = 0.0
    for i in rng.choice(len(quartets), 4000, replace=False):
        g = o[offs[i]:offs[i] + sizes[i]].reshape(4, -1)
        inv = max(inv, np.abs(g.sum(axis=0)).max())
    assert inv <= 1e-12 * max(scale, np.abs(o).max())
    print(f"400 000 quartets: worst |d - oracle| {worst:.2e} over 64 (max |d| {scale:.2e}) at quartet {at[0]} "
          f"(l {at[1]}, its max |d| {at[3]:.2e}, the FP64 oracle's own error there {at[2]:.2e}), "
          f"max |sum over centres| {inv:.2e} over 4 000")
