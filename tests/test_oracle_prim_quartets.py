"""Pins for the oracle's batched primitive-quartet entry (the high-l
microbench's reference): its own plumbing -- centres [n][4][3], exponents
[n][4], unit coefficients turned into N(a, l), output blocks
[n][nsph(la)][nsph(lb)][nsph(lc)][nsph(ld)] in the order the classes are
given -- checked against things that do not go through that plumbing.

- For l <= 2: brute-force quadrature of the Coulomb operator (tests/quadrature.py,
  no recurrences) times the primitive normalisation written out here from its
  closed form, N(a, l) = (2a/pi)^(3/4) (4a)^(l/2) / sqrt((2l-1)!!), and the
  Cartesian -> spherical rows (pinned separately against scipy's Y_lm).
- For every class up to (gg|gg): the single-shell-quartet entry on a basis of
  four one-primitive shells (itself pinned by electrostatics, the H2/STO-3G
  worked example and the invariances), element by element.
- (ss|ss): the electrostatic energy of two Gaussian charge distributions.
"""
import math

import numpy as np
import pytest
import scipy.special

import workloads
from tests import quadrature as qd

BOHR = 0.529177210903


def _norm(a, l):
    dfact = 1.0
    for k in range(2 * l - 1, 0, -2):
        dfact *= k
    return (2 * a / math.pi) ** 0.75 * (4 * a) ** (l / 2) / math.sqrt(dfact)


def _draw(rng, n, box=6.0, lo=0.1, hi=100.0):
    """Microbench-shaped quartets: centres uniform in a box (angstrom -> bohr),
    exponents log-uniform."""
    cen = rng.uniform(0.0, box, (n, 4, 3)) / BOHR
    ex = np.exp(rng.uniform(math.log(lo), math.log(hi), (n, 4)))
    return cen, ex


def _one_prim_basis(ls, cen, ex):
    return workloads.Basis(l=np.array(ls, np.int32), nprim=np.ones(4, np.int32), centers=np.asarray(cen, float),
                           exps=np.asarray(ex, float), coefs=np.ones(4), atom=np.arange(4, dtype=np.int32),
                           atoms=np.asarray(cen, float))


LOW = [(0, 0, 0, 0), (1, 0, 0, 0), (0, 1, 0, 0), (1, 1, 0, 0), (1, 0, 1, 0), (0, 1, 0, 1), (1, 1, 1, 1),
       (2, 0, 0, 0), (0, 0, 0, 2), (2, 1, 0, 1), (1, 2, 2, 0), (2, 2, 1, 1), (2, 2, 2, 2)]


@pytest.mark.parametrize("ls", LOW)
def test_prim_quartets_vs_quadrature(oracle_lib, ls):
    rng = np.random.default_rng(3000 + sum(k * 5 ** i for i, k in enumerate(ls)))
    # compact quartets (quadrature converges), one of them with A = B and C = D
    n = 3
    cen = rng.uniform(-1.2, 1.2, (n, 4, 3))
    cen[1, 1] = cen[1, 0]
    cen[1, 3] = cen[1, 2]
    ex = np.exp(rng.uniform(math.log(0.3), math.log(5.0), (n, 4)))
    got = oracle_lib.eri_prim_quartets(ls, cen, ex)
    assert got.shape == (n,) + tuple(2 * l + 1 for l in ls)
    T = [oracle_lib.sph_matrix(l) for l in ls]
    for q in range(n):
        cart = qd.prim_cart_eri(ls, cen[q], ex[q])
        nrm = np.prod([_norm(ex[q, r], ls[r]) for r in range(4)])
        ref = nrm * np.einsum("ai,bj,ck,dl,ijkl->abcd", T[0], T[1], T[2], T[3], cart)
        scale = np.abs(ref).max()
        assert np.abs(got[q] - ref).max() <= 1e-12 * scale + 1e-16, (ls, q)


HIGH = [(3, 3, 3, 3), (4, 4, 4, 4), (4, 3, 2, 1), (1, 2, 3, 4), (0, 4, 4, 0), (3, 0, 0, 4), (4, 4, 0, 0),
        (2, 2, 2, 2), (3, 2, 3, 2)]


@pytest.mark.parametrize("ls", HIGH)
@pytest.mark.parametrize("shape", ["microbench", "compact"])
def test_prim_quartets_vs_shell_quartet(oracle_lib, ls, shape):
    rng = np.random.default_rng(4000 + sum(k * 5 ** i for i, k in enumerate(ls)) + (shape == "compact"))
    n = 4 if max(ls) == 4 else 6
    if shape == "microbench":
        cen, ex = _draw(rng, n)
    else:
        cen, ex = _draw(rng, n, box=1.0, lo=0.5, hi=3.0)
    got = oracle_lib.eri_prim_quartets(ls, cen, ex)
    for q in range(n):
        ref = oracle_lib.eri_shell_quartet(_one_prim_basis(ls, cen[q], ex[q]), 0, 1, 2, 3)
        scale = np.abs(ref).max()
        # same arithmetic by a different route into it: agreement to rounding
        assert np.abs(got[q] - ref).max() <= 1e-14 * scale + 1e-300, (ls, shape, q)


def test_prim_quartets_ssss_electrostatics(oracle_lib):
    # (ss|ss) of normalised primitives = interaction of the charge distributions
    # phi_a phi_b and phi_c phi_d: S_ab S_cd erf(sqrt(mu) R) / R, with each
    # product a Gaussian of exponent p (q) and weight S_ab (S_cd), mu = pq/(p+q)
    rng = np.random.default_rng(5)
    cen, ex = _draw(rng, 32)
    got = oracle_lib.eri_prim_quartets((0, 0, 0, 0), cen, ex)[:, 0, 0, 0, 0]
    for k in range(32):
        a, b, c, d = ex[k]
        A, B, C, D = cen[k]
        p, q = a + b, c + d
        P, Q = (a * A + b * B) / p, (c * C + d * D) / q
        Sab = _norm(a, 0) * _norm(b, 0) * (math.pi / p) ** 1.5 * math.exp(-a * b / p * np.sum((A - B) ** 2))
        Scd = _norm(c, 0) * _norm(d, 0) * (math.pi / q) ** 1.5 * math.exp(-c * d / q * np.sum((C - D) ** 2))
        mu = p * q / (p + q)
        R = math.sqrt(np.sum((P - Q) ** 2))
        v = Sab * Scd * (2 * math.sqrt(mu / math.pi) if R < 1e-12 else scipy.special.erf(math.sqrt(mu) * R) / R)
        assert abs(got[k] - v) <= 1e-13 * abs(v) + 1e-300, (k, got[k], v)


def test_prim_quartets_block_layout(oracle_lib):
    # a permuted class must give the permuted block: (ab|cd) -> (ba|dc) and (cd|ab)
    rng = np.random.default_rng(9)
    cen, ex = _draw(rng, 3, box=2.0, lo=0.3, hi=5.0)
    ls = (3, 1, 2, 0)
    g = oracle_lib.eri_prim_quartets(ls, cen, ex)
    perm = [1, 0, 3, 2]
    g2 = oracle_lib.eri_prim_quartets(tuple(ls[i] for i in perm), cen[:, perm], ex[:, perm])
    # the permuted evaluation runs the recurrences from other centres, so the
    # blocks agree to rounding relative to the block's largest element
    scale = np.abs(g).max(axis=(1, 2, 3, 4), keepdims=True)
    assert (np.abs(g2 - g.transpose(0, 2, 1, 4, 3)) <= 1e-12 * scale).all()
    perm = [2, 3, 0, 1]
    g3 = oracle_lib.eri_prim_quartets(tuple(ls[i] for i in perm), cen[:, perm], ex[:, perm])
    assert (np.abs(g3 - g.transpose(0, 3, 4, 1, 2)) <= 1e-12 * scale).all()


def test_prim_quartets_rejects(oracle_lib):
    with pytest.raises(ValueError):
        oracle_lib.eri_prim_quartets((5, 0, 0, 0), np.zeros((1, 4, 3)), np.ones((1, 4)))
