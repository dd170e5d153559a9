"""Pins for the CPU oracle against things other than itself.

- primitive Cartesian integrals (vertical + horizontal recurrences, Eqs. vrr
  and hrr of Sec. II-A) vs brute-force quadrature of the Coulomb operator;
- contraction and shell normalisation vs numerically integrated overlaps;
- the Cartesian -> pure spherical matrices (Sec. III-B, Eq. cart2sph) vs
  scipy's spherical harmonics on the unit sphere, harmonicity and the sign
  convention;
- (ss|ss) vs the electrostatics of Gaussian charge distributions;
- a textbook worked example (H2 / STO-3G);
- invariances of the exact integrals: 8-fold permutational symmetry,
  translation and rotation invariance, the Schwarz inequality;
- J/K digestion from unique quartets vs the full tensor contracted with
  einsum, symmetry, linearity and positivity for a PSD density.
"""
import math
import os

import numpy as np
import pytest
import scipy.special

import workloads
from tests import quadrature as qd

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _cart_list(l):
    return [(x, y, l - x - y) for x in range(l, -1, -1) for y in range(l - x, -1, -1)]


# ---------------------------------------------------------------- primitive integrals

CLASSES = [(0, 0, 0, 0), (1, 0, 0, 0), (0, 1, 0, 0), (0, 0, 1, 0), (0, 0, 0, 1), (1, 1, 0, 0), (0, 0, 1, 1),
           (1, 0, 1, 0), (1, 1, 1, 1), (2, 0, 0, 0), (0, 0, 2, 0), (2, 1, 1, 0), (0, 2, 1, 1), (2, 2, 1, 1),
           (1, 2, 2, 1), (2, 2, 2, 2), (3, 1, 0, 2), (0, 3, 2, 1), (4, 0, 1, 0), (1, 1, 0, 4)]


@pytest.mark.parametrize("ls", CLASSES)
def test_prim_cart_vs_quadrature(oracle_lib, ls):
    rng = np.random.default_rng(100 + sum(k * 7 ** i for i, k in enumerate(ls)))
    for trial in range(3):
        cen = rng.uniform(-1.5, 1.5, (4, 3))
        if trial == 1:
            cen[1] = cen[0]            # A = B: horizontal recurrence factor vanishes
        al = np.exp(rng.uniform(math.log(0.25), math.log(6.0), 4))
        ref = qd.prim_cart_eri(ls, cen, al)
        got = oracle_lib.prim_cart_eri(ls, cen, al)
        scale = np.abs(ref).max()
        assert np.abs(got - ref).max() <= 1e-12 * scale + 1e-16, (ls, trial)


def test_prim_cart_large_T(oracle_lib):
    # distant pairs: T well above the series/asymptotic switch of the Boys function
    rng = np.random.default_rng(7)
    for ls in [(1, 1, 1, 0), (2, 0, 2, 1)]:
        cen = rng.uniform(-0.5, 0.5, (4, 3))
        cen[2:] += np.array([4.0, 1.0, -2.0])
        al = np.array([2.5, 3.0, 4.0, 1.5])
        ref = qd.prim_cart_eri(ls, cen, al)
        got = oracle_lib.prim_cart_eri(ls, cen, al)
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


# ---------------------------------------------------------------- normalisation + shell transform

def _shell_overlap(oracle_lib, l, exps, coefs):
    """<phi_mu|phi_nu> for the spherical functions of one contracted shell,
    each primitive integral done by Gauss-Hermite moments."""
    c = oracle_lib.norm_coefs(l, exps, coefs)
    t = oracle_lib.sph_matrix(l)
    cl = _cart_list(l)
    n = len(cl)
    S = np.zeros((n, n))
    for k, ak in enumerate(exps):
        for q, aq in enumerate(exps):
            beta = ak + aq
            for i, ci in enumerate(cl):
                for j, cj in enumerate(cl):
                    S[i, j] += c[k] * c[q] * math.prod(qd.gauss_moment(ci[ax] + cj[ax], beta) for ax in range(3))
    return t @ S @ t.T


@pytest.mark.parametrize("l", [0, 1, 2, 3, 4])
def test_contracted_spherical_shell_is_orthonormal(oracle_lib, l):
    rng = np.random.default_rng(l)
    for nprim in (1, 3, 6):
        exps = np.exp(rng.uniform(math.log(0.05), math.log(5e3), nprim))
        coefs = rng.uniform(0.1, 1.0, nprim)
        S = _shell_overlap(oracle_lib, l, exps, coefs)
        assert np.abs(S - np.eye(2 * l + 1)).max() < 1e-12


def _real_ylm(l, m, theta, phi):
    # real spherical harmonics from scipy's complex ones (phase-free magnitude check)
    y = scipy.special.sph_harm_y(l, abs(m), theta, phi)
    if m > 0:
        return math.sqrt(2) * y.real
    if m < 0:
        return math.sqrt(2) * y.imag
    return y.real


@pytest.mark.parametrize("l", [2, 3, 4])
def test_sph_rows_are_real_harmonics(oracle_lib, l):
    t = oracle_lib.sph_matrix(l)
    cl = _cart_list(l)
    rng = np.random.default_rng(10 + l)
    pts = rng.normal(size=(64, 3))
    pts /= np.linalg.norm(pts, axis=1, keepdims=True)
    theta = np.arccos(pts[:, 2])
    phi = np.arctan2(pts[:, 1], pts[:, 0])
    mono = np.stack([pts[:, 0] ** c[0] * pts[:, 1] ** c[1] * pts[:, 2] ** c[2] for c in cl], axis=1)
    ratios = []
    for row in range(2 * l + 1):
        m = row - l
        s = mono @ t[row]
        y = np.array([_real_ylm(l, m, th, ph) for th, ph in zip(theta, phi)])
        r = s / y
        # a solid harmonic of degree l and order m is a fixed multiple of Y_lm on the sphere
        assert np.std(r) < 1e-10 * np.abs(np.mean(r)), (l, m)
        ratios.append(abs(np.mean(r)))
    # unit norm in the Gaussian basis makes that multiple the same for every m
    assert np.ptp(ratios) < 1e-10 * ratios[0]


@pytest.mark.parametrize("l", [2, 3, 4])
def test_sph_rows_harmonic_and_sign(oracle_lib, l):
    t = oracle_lib.sph_matrix(l)
    cl = _cart_list(l)
    idx = {c: i for i, c in enumerate(cl)}
    for row in range(2 * l + 1):
        m = row - l
        lap = {}
        for c, v in zip(cl, t[row]):
            for ax in range(3):
                if c[ax] >= 2:
                    d = list(c)
                    d[ax] -= 2
                    lap[tuple(d)] = lap.get(tuple(d), 0.0) + v * c[ax] * (c[ax] - 1)
        assert max((abs(v) for v in lap.values()), default=0.0) < 1e-12
        am = abs(m)
        lead = (am, 0, l - am) if m >= 0 else (am - 1, 1, l - am)
        assert t[row, idx[lead]] > 0


def test_n_cart_and_n_sph_counts():
    # Sec. III-B: 6 -> 5 at l = 2, 15 -> 9 at l = 4, 15^4 / 9^4 = 7.7
    assert [len(_cart_list(l)) for l in range(5)] == [1, 3, 6, 10, 15]
    assert round(15 ** 4 / 9 ** 4, 1) == 7.7


# ---------------------------------------------------------------- closed forms and a worked example

def _one_prim_basis(ls, centers, exps):
    return workloads.Basis(np.array(ls, np.int32), np.ones(len(ls), np.int32), np.array(centers, float).reshape(-1, 3),
                           np.array(exps, float), np.ones(len(ls)), np.zeros(len(ls), np.int32),
                           np.zeros((1, 3)))


def test_ssss_gaussian_electrostatics(oracle_lib):
    # s_a1 s_a2 on A is a Gaussian charge of exponent p = a1 + a2 and total charge
    # S_A = N1 N2 (pi/p)^{3/2}; two such charges interact as S_A S_B erf(sqrt(mu) R)/R,
    # mu = p q / (p + q), and 2 S_A S_B sqrt(mu/pi) at R = 0.
    rng = np.random.default_rng(3)
    for R in (0.0, 0.3, 1.7, 6.0):
        a = np.exp(rng.uniform(-1.5, 2.0, 4))
        A = np.zeros(3)
        B = np.array([0.0, 0.0, R])
        b = _one_prim_basis([0, 0, 0, 0], [A, A, B, B], a)
        got = oracle_lib.eri_shell_quartet(b, 0, 1, 2, 3)[0, 0, 0, 0]
        N = (2 * a / math.pi) ** 0.75
        p, q = a[0] + a[1], a[2] + a[3]
        SA = N[0] * N[1] * (math.pi / p) ** 1.5
        SB = N[2] * N[3] * (math.pi / q) ** 1.5
        mu = p * q / (p + q)
        ref = SA * SB * (2 * math.sqrt(mu / math.pi) if R == 0 else math.erf(math.sqrt(mu) * R) / R)
        assert abs(got - ref) <= 2e-15 * abs(ref)


def test_one_centre_equal_exponent_ssss(oracle_lib):
    for alpha in (0.1, 1.0, 37.0):
        b = _one_prim_basis([0, 0, 0, 0], [np.zeros(3)] * 4, [alpha] * 4)
        got = oracle_lib.eri_shell_quartet(b, 0, 1, 2, 3)[0, 0, 0, 0]
        assert abs(got - 2 * math.sqrt(alpha / math.pi)) <= 1e-15 * got


def test_h2_sto3g_textbook_values(oracle_lib):
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, "h2_sto3g_szabo_ostlund.txt")) if ln.strip() and ln[0] != "#"]
    ex = np.array([float(x) for x in rows[0][1:]])
    co = np.array([float(x) for x in rows[1][1:]])
    R = float(rows[2][1])
    b = workloads.Basis(np.zeros(2, np.int32), np.array([3, 3], np.int32), np.array([[0, 0, 0], [0, 0, R]], float),
                        np.concatenate([ex, ex]), np.concatenate([co, co]), np.zeros(2, np.int32), np.zeros((1, 3)))
    for r in rows[3:]:
        i, j, k, l = (int(x) for x in r[1:5])
        got = oracle_lib.eri_shell_quartet(b, i, j, k, l)[0, 0, 0, 0]
        assert abs(got - float(r[5])) <= 6e-5, (r, got)


# ---------------------------------------------------------------- invariances of the exact integrals

@pytest.fixture(scope="module")
def small_basis():
    return workloads.random_small_basis(seed=11, natom=3, lmax=2, maxprim=3)


def test_eightfold_symmetry(oracle_lib, small_basis):
    b = small_basis
    rng = np.random.default_rng(1)
    for _ in range(25):
        i, j, k, l = (int(x) for x in rng.integers(0, b.nshell, 4))
        ref = oracle_lib.eri_shell_quartet(b, i, j, k, l)
        perms = {(j, i, k, l): (1, 0, 2, 3), (i, j, l, k): (0, 1, 3, 2), (j, i, l, k): (1, 0, 3, 2),
                 (k, l, i, j): (2, 3, 0, 1), (l, k, i, j): (3, 2, 0, 1), (k, l, j, i): (2, 3, 1, 0),
                 (l, k, j, i): (3, 2, 1, 0)}
        for sh, ax in perms.items():
            got = oracle_lib.eri_shell_quartet(b, *sh)
            assert np.abs(np.transpose(got, np.argsort(ax)) - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())


def test_translation_invariance(oracle_lib, small_basis):
    b = small_basis
    shifted = workloads.Basis(b.l, b.nprim, b.centers + np.array([3.3, -1.2, 7.9]), b.exps, b.coefs, b.atom, b.atoms)
    rng = np.random.default_rng(2)
    for _ in range(12):
        q = [int(x) for x in rng.integers(0, b.nshell, 4)]
        a = oracle_lib.eri_shell_quartet(b, *q)
        c = oracle_lib.eri_shell_quartet(shifted, *q)
        assert np.abs(a - c).max() <= 1e-13 * max(1.0, np.abs(a).max())


def _rotation(rng):
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q *= np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


@pytest.mark.parametrize("lmax", [2, 4])
def test_rotation_invariants(oracle_lib, lmax):
    # under a rigid rotation each shell's spherical functions mix orthogonally, so the
    # Frobenius norm of every block and the singular values of its (ab) x (cd)
    # unfolding are unchanged
    b = workloads.random_small_basis(seed=20 + lmax, natom=2, lmax=lmax, maxprim=2)
    rng = np.random.default_rng(9)
    Rm = _rotation(rng)
    rot = workloads.Basis(b.l, b.nprim, b.centers @ Rm.T, b.exps, b.coefs, b.atom, b.atoms)
    for _ in range(8 if lmax == 2 else 4):
        q = [int(x) for x in rng.integers(0, b.nshell, 4)]
        x = oracle_lib.eri_shell_quartet(b, *q)
        y = oracle_lib.eri_shell_quartet(rot, *q)
        scale = max(1.0, np.linalg.norm(x))
        assert abs(np.linalg.norm(x) - np.linalg.norm(y)) <= 1e-12 * scale
        sx = np.linalg.svd(x.reshape(x.shape[0] * x.shape[1], -1), compute_uv=False)
        sy = np.linalg.svd(y.reshape(y.shape[0] * y.shape[1], -1), compute_uv=False)
        assert np.abs(sx - sy).max() <= 1e-12 * scale


def test_schwarz_inequality(oracle_lib, small_basis):
    b = small_basis
    T = oracle_lib.eri_tensor(b)
    N = b.nbf
    diag = np.einsum("ijij->ij", T)
    bound = np.sqrt(np.abs(diag)[:, :, None, None] * np.abs(diag)[None, None, :, :])
    # equality holds for (ab|ba) vs (ab|ab); the two sides come from different horizontal-
    # recurrence directions, whose FP64 rounding differs by a few 1e-12 relative
    assert np.all(np.abs(T) <= bound * (1 + 1e-11) + 1e-14)
    Q = oracle_lib.schwarz(b)
    off = b.shell_offsets()
    for s in range(b.nshell):
        for t in range(b.nshell):
            blk = diag[off[s]:off[s + 1], off[t]:off[t + 1]]
            assert abs(Q[s, t] - math.sqrt(np.abs(blk).max())) <= 1e-12 * max(1.0, Q[s, t])


def test_long_double_build_agrees(oracle_lib):
    b = workloads.random_small_basis(seed=31, natom=2, lmax=3, maxprim=3)
    rng = np.random.default_rng(4)
    for _ in range(6):
        q = [int(x) for x in rng.integers(0, b.nshell, 4)]
        x = oracle_lib.eri_shell_quartet(b, *q)
        y = oracle_lib.eri_shell_quartet(b, *q, precision="long double")
        assert np.abs(x - y).max() <= 1e-13 * max(1.0, np.abs(y).max())


# ---------------------------------------------------------------- J / K

@pytest.fixture(scope="module")
def tiny():
    return workloads.tiny_system()


def test_tiny_system_shape(tiny):
    b, D = tiny
    assert b.nshell == 12 and b.nbf == 20 and D.shape == (20, 20)
    assert np.allclose(D, D.T) and np.linalg.eigvalsh(D).min() > -1e-12


def test_jk_unique_quartets_vs_full_tensor(oracle_lib, tiny):
    b, D = tiny
    T = oracle_lib.eri_tensor(b)
    J, K = oracle_lib.jk(b, D)
    Jr = np.einsum("ijkl,kl->ij", T, D)
    Kr = np.einsum("ikjl,kl->ij", T, D)
    assert np.abs(J - Jr).max() <= 1e-12 * np.abs(Jr).max()
    assert np.abs(K - Kr).max() <= 1e-12 * np.abs(Kr).max()


def test_jk_nonsymmetric_density_vs_full_tensor(oracle_lib, small_basis):
    # the unique-quartet digestion must not silently assume a symmetric D
    b = small_basis
    D = np.random.default_rng(8).normal(size=(b.nbf, b.nbf))
    T = oracle_lib.eri_tensor(b)
    J, K = oracle_lib.jk(b, D)
    assert np.abs(J - np.einsum("ijkl,kl->ij", T, D)).max() <= 1e-12 * np.abs(J).max()
    assert np.abs(K - np.einsum("ikjl,kl->ij", T, D)).max() <= 1e-12 * np.abs(K).max()


def test_jk_symmetric_linear_positive(oracle_lib, tiny):
    b, D = tiny
    J, K = oracle_lib.jk(b, D)
    assert np.abs(J - J.T).max() <= 1e-13 * np.abs(J).max()
    assert np.abs(K - K.T).max() <= 1e-13 * np.abs(K).max()
    D2 = workloads.psd_density(b.nbf, 77)
    J2, K2 = oracle_lib.jk(b, D2)
    J3, K3 = oracle_lib.jk(b, 2.0 * D - 0.5 * D2)
    assert np.abs(J3 - (2 * J - 0.5 * J2)).max() <= 1e-12 * np.abs(J3).max()
    assert np.abs(K3 - (2 * K - 0.5 * K2)).max() <= 1e-12 * np.abs(K3).max()
    # the Coulomb kernel is positive definite: tr(DJ), tr(DK) >= 0 for PSD D
    assert np.trace(D @ J) > 0 and np.trace(D @ K) > 0


def test_jk_blocks_match_digestion(oracle_lib, tiny):
    b, D = tiny
    J, K = oracle_lib.jk(b, D)
    off = b.shell_offsets()
    pairs = [(0, 0), (2, 1), (5, 8), (11, 3)]
    Js, Ks = oracle_lib.jk_blocks(b, D, pairs)
    for (p, q), jb, kb in zip(pairs, Js, Ks):
        assert np.abs(jb - J[off[p]:off[p + 1], off[q]:off[q + 1]]).max() <= 1e-12 * np.abs(J).max()
        assert np.abs(kb - K[off[p]:off[p + 1], off[q]:off[q + 1]]).max() <= 1e-12 * np.abs(K).max()


def test_screening_error_is_bounded(oracle_lib):
    b = workloads.random_small_basis(seed=41, natom=4, lmax=1, maxprim=2, box=12.0, exp_range=(2.0, 30.0))
    D = workloads.psd_density(b.nbf, 5)
    J0, K0 = oracle_lib.jk(b, D, tau=0.0)
    tau = 1e-8
    J1, K1 = oracle_lib.jk(b, D, tau=tau)
    Q = oracle_lib.schwarz(b)
    skipped = (Q.reshape(-1)[:, None] * Q.reshape(-1)[None, :] < tau).sum()
    assert skipped > 0
    # each skipped ordered quartet changes an entry by at most tau * max|D|
    bound = tau * np.abs(D).max() * skipped
    assert np.abs(J1 - J0).max() <= bound and np.abs(K1 - K0).max() <= bound


def test_oracle_rejects_bad_input(oracle_lib):
    b = _one_prim_basis([5, 0, 0, 0], [np.zeros(3)] * 4, [1.0] * 4)
    with pytest.raises(ValueError):
        oracle_lib.eri_shell_quartet(b, 0, 1, 2, 3)
    b = _one_prim_basis([0, 0, 0, 0], [np.zeros(3)] * 4, [1.0, -1.0, 1.0, 1.0])
    with pytest.raises(ValueError):
        oracle_lib.eri_shell_quartet(b, 0, 1, 2, 3)
