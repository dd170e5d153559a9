"""Mixed precision (FP32 VRR and primitive contraction for quartets whose
Schwarz bound is below theta; FP64 Boys, pair quantities, HRR, transforms and
J/K accumulation): J/K within the 1e-9 bar of the oracle, the FP32 lists
present where they should be, the full-size workload against both the
oracle's sampled blocks and the plan's own FP64 result, and the integrals-out
entry with HGP_MIXED against the oracle per class."""
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


def _jk(hgp, torch, bw, D, tau, theta):
    b = hgp.Basis.from_workload(bw)
    plan = hgp.Plan(b, tau=tau, theta=theta)
    Dt = torch.tensor(D, device="cuda")
    J = torch.empty_like(Dt)
    K = torch.empty_like(Dt)
    plan.jk(Dt, J, K)
    torch.cuda.synchronize()
    cls = plan.classes()
    plan.close()
    b.close()
    return J.cpu().numpy(), K.cpu().numpy(), cls


@pytest.mark.parametrize("seed,tau,theta", [(61, 0.0, 1e-6), (62, 1e-12, 1e-6), (63, 1e-12, 1e-5)])
def test_mixed_random_basis(hgp, torch_cuda, seed, tau, theta):
    bw = workloads.random_small_basis(seed=seed, natom=4, lmax=2, maxprim=4, box=5.0, exp_range=(0.1, 50.0))
    D = workloads.psd_density(bw.nbf, seed)
    Jr, Kr = oracle.jk(bw, D, tau=tau)
    J, K, cls = _jk(hgp, torch_cuda, bw, D, tau, theta)
    n32 = sum(c["quartets"] for c in cls if c["bits"] == 32)
    n64 = sum(c["quartets"] for c in cls if c["bits"] == 64)
    ej, ek = np.abs(J - Jr).max(), np.abs(K - Kr).max()
    print(f"seed {seed} tau {tau} theta {theta}: {n32} FP32 / {n64} FP64 quartets, |dJ| {ej:.2e} |dK| {ek:.2e}")
    assert n32 > 0
    assert all(c["tier"] == 0 for c in cls if c["bits"] == 32)
    assert ej <= JK_TOL and ek <= JK_TOL


def test_mixed_error_grows_with_theta(hgp, torch_cuda):
    """The FP32 part really runs and its error follows the threshold: the
    deviation from FP64 grows with theta and stays within FP32's relative
    precision of the largest Schwarz bound it covers."""
    bw = workloads.random_small_basis(seed=64, natom=4, lmax=2, maxprim=4, box=5.0, exp_range=(0.1, 50.0))
    D = workloads.psd_density(bw.nbf, 64)
    J0, K0, _ = _jk(hgp, torch_cuda, bw, D, 0.0, 0.0)
    errs = []
    for theta in (1e-8, 1e-6, 1e-4, 1e-2):
        J, K, cls = _jk(hgp, torch_cuda, bw, D, 0.0, theta)
        e = max(np.abs(J - J0).max(), np.abs(K - K0).max())
        errs.append(e)
        print(f"theta {theta:g}: FP32 quartets {sum(c['quartets'] for c in cls if c['bits'] == 32)}, "
              f"max |JK_mixed - JK_fp64| {e:.2e}")
    assert errs[-1] > errs[0]
    assert errs[-1] <= 1e-2 * 1e-3 * bw.nbf


def test_theta_below_tau_is_fp64(hgp, torch_cuda):
    bw, D = workloads.tiny_system()
    J, K, cls = _jk(hgp, torch_cuda, bw, D, 1e-10, 1e-11)
    assert all(c["bits"] == 64 for c in cls)


def test_mixed_full_size(hgp, torch_cuda):
    """The 30-atom 3s2p1d workload at the library's default theta: sampled
    blocks against the oracle and every entry against the FP64 plan."""
    bw, D = workloads.molecule_3s2p1d()
    J64, K64, _ = _jk(hgp, torch_cuda, bw, D, 1e-12, 0.0)
    Jm, Km, cls = _jk(hgp, torch_cuda, bw, D, 1e-12, hgp.MIXED_THETA_DEFAULT)
    frac = sum(c["quartets"] for c in cls if c["bits"] == 32) / sum(c["quartets"] for c in cls)
    dj, dk = np.abs(Jm - J64).max(), np.abs(Km - K64).max()
    print(f"default theta {hgp.MIXED_THETA_DEFAULT}: FP32 share {frac:.3f}, max |J_mixed - J_fp64| {dj:.2e}, "
          f"max |K_mixed - K_fp64| {dk:.2e}")
    assert dj <= JK_TOL and dk <= JK_TOL
    from tests.test_gpu_fullsize import compare_blocks, load_golden_blocks
    rows, rms = compare_blocks(bw, Jm, Km, load_golden_blocks())
    print(f"mixed vs oracle over {len(rows)} blocks: max |dJ| {max(r[2] for r in rows):.2e}, "
          f"max |dK| {max(r[3] for r in rows):.2e}, RMS {rms:.2e}")
    for pr, ls, ej, ek, eo in rows:
        assert ej <= JK_TOL and ek <= JK_TOL, (pr, ls, ej, ek)


def test_mixed_plans_keep_row_form_classes_fp64(hgp, torch_cuda):
    """A d-rich basis has (dd|dd)-type lists in the staged row form, which has
    an FP32 Phase 1 for the integrals-out entry; a mixed J/K plan still runs
    them in FP64 (their HRR cancellation lifts the FP32 error past what the
    Schwarz bound controls) and stays within the bar."""
    bw = workloads.random_small_basis(seed=66, natom=3, lmax=2, maxprim=3, box=4.0, exp_range=(0.2, 20.0))
    D = workloads.psd_density(bw.nbf, 66)
    Jr, Kr = oracle.jk(bw, D, tau=0.0)
    J, K, cls = _jk(hgp, torch_cuda, bw, D, 0.0, 1e-6)
    assert any(c["tier"] == 1 and hgp.class_has_fp32(c["ls"]) for c in cls)
    assert all(c["tier"] == 0 for c in cls if c["bits"] == 32) and any(c["bits"] == 32 for c in cls)
    ej, ek = np.abs(J - Jr).max(), np.abs(K - Kr).max()
    print(f"|dJ| {ej:.2e} |dK| {ek:.2e}")
    assert ej <= JK_TOL and ek <= JK_TOL


# HGP_MIXED runs the same recurrences as the FP64 path with the VRR values
# rounded to FP32: its error is the FP64 path's own rounding error scaled by
# the ratio of the unit roundoffs, 2^-24 / 2^-53 = 2^29, whatever the
# cancellation the class's HRR brings.  Both errors are taken against the
# long-double oracle; the bar allows a factor 10 over that scaling, and the
# FP64 error is floored at one FP64 rounding of the largest integral.
EPS_RATIO = 2.0 ** 29


@pytest.mark.parametrize("ls", [(0, 0, 0, 0), (1, 1, 1, 1), (2, 1, 1, 0), (2, 2, 1, 1), (2, 2, 2, 1), (2, 2, 2, 2),
                                (3, 2, 1, 0), (3, 3, 3, 3), (4, 4, 4, 4)])
def test_prim_quartets_mixed(hgp, torch_cuda, ls):
    torch = torch_cuda
    n = 200
    cen, ex = workloads.prim_quartets(max(ls), n, seed=77 + sum(ls))
    ct, et = torch.tensor(cen, device="cuda"), torch.tensor(ex, device="cuda")
    nsph = int(np.prod([2 * x + 1 for x in ls]))
    o64 = torch.empty((n, nsph), dtype=torch.float64, device="cuda")
    o32 = torch.empty_like(o64)
    hgp.eri_prim_quartets(ls, ct, et, o64, precision=hgp.HGP_FP64)
    hgp.eri_prim_quartets(ls, ct, et, o32, precision=hgp.HGP_MIXED)
    torch.cuda.synchronize()
    g64, g32 = o64.cpu().numpy(), o32.cpu().numpy()
    ref = oracle.eri_prim_quartets(ls, cen, ex).reshape(n, -1)
    ref_ld = oracle.eri_prim_quartets(ls, cen, ex, precision="long double").reshape(n, -1)
    scale = np.abs(ref_ld).max()
    e_orc = np.abs(ref - ref_ld).max()
    e64, e32 = np.abs(g64 - ref_ld).max(), np.abs(g32 - ref_ld).max()
    rms = float(np.sqrt(np.mean((g32 - ref) ** 2)))
    tier, f32 = hgp.class_form(ls)
    print(f"{ls} tier {tier} fp32 form {f32}: scale {scale:.2e}, FP64 err {e64:.2e} (oracle {e_orc:.2e}), "
          f"mixed err {e32:.2e} ({e32 / scale:.2e} of scale, {e32 / max(e64, 2.0 ** -53 * scale):.2e} x FP64), "
          f"RMS vs oracle {rms:.2e}")
    assert e64 <= 1e-12 * scale + 8 * e_orc
    if f32:
        assert e32 <= 10 * EPS_RATIO * max(e64, 2.0 ** -53 * scale)
        assert e32 > e64                       # the FP32 form really ran
    else:
        assert np.array_equal(g32, g64)        # no FP32 form: the FP64 kernels, bit for bit
