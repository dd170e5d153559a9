"""Pins for the oracle's Boys function F_m(T) = int_0^1 t^{2m} exp(-T t^2) dt
(the base values of the vertical recurrence, Sec. II-A, Eq. vrr).

Independent references: mpmath's confluent hypergeometric function at 40
digits, F_m(T) = 1F1(m+1/2; m+3/2; -T)/(2m+1); the closed form of F_0 through
erf; F_m(0) = 1/(2m+1); the large-T asymptote."""
import math

import mpmath
import numpy as np
import pytest

T_GRID = [0.0, 1e-14, 1e-8, 1e-3, 0.1, 0.5, 1.0, 2.5, 5.0, 9.99, 15.0, 24.5, 30.0, 35.0, 39.999, 40.0,
          40.001, 55.0, 100.0, 1234.5, 1e5, 1e8]


def _boys_mp(m, T):
    mpmath.mp.dps = 40
    return mpmath.hyp1f1(m + mpmath.mpf(1) / 2, m + mpmath.mpf(3) / 2, -mpmath.mpf(T)) / (2 * m + 1)


@pytest.mark.parametrize("T", T_GRID)
def test_boys_vs_hypergeometric(oracle_lib, T):
    F = oracle_lib.boys(20, T)
    for m in range(21):
        ref = float(_boys_mp(m, T))
        assert abs(F[m] - ref) <= 2e-15 * ref, (m, T, F[m], ref)


def test_boys_zero_exact(oracle_lib):
    F = oracle_lib.boys(20, 0.0)
    assert all(F[m] == 1.0 / (2 * m + 1) for m in range(21))


def test_boys_f0_erf(oracle_lib):
    rng = np.random.default_rng(5)
    for T in np.concatenate([rng.uniform(1e-6, 60, 200), [1e-10, 39.9999, 40.0]]):
        ref = 0.5 * math.sqrt(math.pi / T) * math.erf(math.sqrt(T))
        # the double-precision erf reference itself carries a few ulps
        assert abs(oracle_lib.boys(0, T)[0] - ref) <= 2e-15 * ref + 1e-17


def test_boys_recurrence_identity(oracle_lib):
    # 2T F_{m+1} = (2m+1) F_m - exp(-T), an identity of the integral (integration by parts)
    for T in [0.3, 7.0, 33.0, 45.0]:
        F = oracle_lib.boys(16, T)
        for m in range(16):
            lhs = 2 * T * F[m + 1]
            rhs = (2 * m + 1) * F[m] - math.exp(-T)
            assert abs(lhs - rhs) <= 1e-14 * abs(rhs) + 1e-300


def test_boys_large_T_asymptote(oracle_lib):
    # F_m(T) -> (2m-1)!! / 2^{m+1} sqrt(pi / T^{2m+1}) as T -> infinity
    T = 1e6
    F = oracle_lib.boys(12, T)
    for m in range(13):
        dfm = math.prod(range(2 * m - 1, 0, -2)) if m > 0 else 1
        ref = dfm / 2 ** (m + 1) * math.sqrt(math.pi / T ** (2 * m + 1))
        assert abs(F[m] - ref) <= 1e-14 * ref


def test_boys_long_double_agrees(oracle_lib):
    for T in T_GRID:
        a = oracle_lib.boys(16, T)
        b = oracle_lib.boys(16, T, precision="long double")
        assert np.all(np.abs(a - b) <= 2e-15 * np.abs(b))
