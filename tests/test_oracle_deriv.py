"""Pins for the oracle's first-derivative integrals d/dR (ij|kl) (the method's
adjacent step for nuclear gradients), against things other than the
derivative code itself:

- finite differences: the integrals of the long-double oracle at displaced
  shell centres, central differences at steps h and h/2 combined by
  Richardson extrapolation (error O(h^4));
- translational invariance: moving all four centres together leaves the
  integral unchanged, so the four centre derivatives sum to zero along
  every axis;
- index symmetry: the derivative with respect to shell i's centre of (ij|kl)
  equals the one with respect to the same shell in (ji|lk) and (kl|ij),
  with the block transposed.
"""
import copy

import numpy as np
import pytest

import workloads


def _basis(seed, ls, nprim=2, box=1.6):
    rng = np.random.default_rng(seed)
    n = len(ls)
    npr = np.full(n, nprim, np.int32)
    return workloads.Basis(l=np.array(ls, np.int32), nprim=npr, centers=rng.uniform(-box / 2, box / 2, (n, 3)),
                           exps=np.exp(rng.uniform(np.log(0.4), np.log(4.0), n * nprim)),
                           coefs=rng.uniform(0.3, 1.0, n * nprim), atom=np.arange(n, dtype=np.int32),
                           atoms=np.zeros((n, 3)))


def _fd(oracle_lib, b, q, shell_pos, axis, h):
    """Richardson-extrapolated central difference of (q) in the centre of shell q[shell_pos]."""
    def val(step):
        bb = copy.deepcopy(b)
        bb.centers = np.array(b.centers, dtype=float)
        bb.centers[q[shell_pos], axis] += step
        return oracle_lib.eri_shell_quartet(bb, *q, precision="long double")
    d1 = (val(h) - val(-h)) / (2 * h)
    d2 = (val(h / 2) - val(-h / 2)) / h
    return (4 * d2 - d1) / 3


CLASSES = [(0, 0, 0, 0), (1, 0, 0, 0), (1, 1, 1, 1), (2, 1, 0, 1), (2, 2, 1, 0), (3, 1, 2, 0), (2, 2, 2, 2),
           (4, 0, 1, 1), (3, 3, 1, 0), (0, 2, 4, 1)]


@pytest.mark.parametrize("ls", CLASSES)
def test_deriv_vs_finite_differences(oracle_lib, ls):
    b = _basis(500 + sum(k * 7 ** i for i, k in enumerate(ls)), ls)
    q = (0, 1, 2, 3)
    got = oracle_lib.eri_deriv_shell_quartet(b, *q)
    scale = np.abs(got).max()
    for r in range(4):
        for t in range(3):
            fd = _fd(oracle_lib, b, q, r, t, 1e-3)
            err = np.abs(got[r, t] - fd).max()
            assert err <= 1e-9 * scale + 1e-14, (ls, r, t, err, scale)


@pytest.mark.parametrize("ls", CLASSES + [(4, 4, 3, 2), (4, 3, 4, 4)])
def test_deriv_translational_invariance(oracle_lib, ls):
    b = _basis(700 + sum(k * 7 ** i for i, k in enumerate(ls)), ls, nprim=1 if max(ls) == 4 else 2)
    got = oracle_lib.eri_deriv_shell_quartet(b, 0, 1, 2, 3)
    total = got.sum(axis=0)                          # sum over the four centres, per axis
    assert np.abs(total).max() <= 1e-12 * np.abs(got).max()


def test_deriv_shared_centre_and_symmetry(oracle_lib):
    # two shells on one centre: the derivative in that centre is the sum of both shells' parts
    ls = (2, 1, 1, 0)
    b = _basis(901, ls)
    b.centers[1] = b.centers[0]
    g = oracle_lib.eri_deriv_shell_quartet(b, 0, 1, 2, 3)
    h = 1e-3

    def moved(step, t):
        bb = copy.deepcopy(b)
        bb.centers = np.array(b.centers, dtype=float)
        bb.centers[0, t] += step
        bb.centers[1, t] += step
        return oracle_lib.eri_shell_quartet(bb, 0, 1, 2, 3, precision="long double")
    for t in range(3):
        fd = (4 * (moved(h / 2, t) - moved(-h / 2, t)) / h - (moved(h, t) - moved(-h, t)) / (2 * h)) / 3
        assert np.abs(g[0, t] + g[1, t] - fd).max() <= 1e-9 * np.abs(g).max()
    # (ji|lk): centres 1, 0, 3, 2 and blocks transposed accordingly
    g2 = oracle_lib.eri_deriv_shell_quartet(b, 1, 0, 3, 2)
    for r, r2 in ((0, 1), (1, 0), (2, 3), (3, 2)):
        assert np.allclose(g2[r2], g[r].transpose(0, 2, 1, 4, 3), rtol=0, atol=1e-12 * np.abs(g).max())
    g3 = oracle_lib.eri_deriv_shell_quartet(b, 2, 3, 0, 1)
    for r, r3 in ((0, 2), (1, 3), (2, 0), (3, 1)):
        assert np.allclose(g3[r3], g[r].transpose(0, 3, 4, 1, 2), rtol=0, atol=1e-12 * np.abs(g).max())


def test_deriv_double_vs_long_double(oracle_lib):
    b = _basis(77, (3, 2, 2, 1), nprim=3)
    gd = oracle_lib.eri_deriv_shell_quartet(b, 0, 1, 2, 3)
    gl = oracle_lib.eri_deriv_shell_quartet(b, 0, 1, 2, 3, precision="long double")
    assert np.abs(gd - gl).max() <= 1e-12 * np.abs(gl).max()
