"""Pins for the oracle's K_ν and Matérn covariance (Sec. 2.2 Eq. (2)).

The oracle integrates K_ν(x) = ∫_0^∞ exp(-x cosh t) cosh(νt) dt with the
trapezoidal rule, and the Matérn covariance from the same integral with x^ν
taken inside.  It is pinned here against sources that share nothing with
that method: mpmath's arbitrary-precision besselk, scipy's Amos-based kv, the
three-term recurrence in ν, the x → 0 limit, and the elementary closed forms
the paper lists for special smoothness values.
"""
import math

import mpmath
import numpy as np
import pytest
import scipy.special as sp

import oracle

mpmath.mp.dps = 40

NUS = [0.05, 0.25, 0.5, 0.77, 1.0, 1.3, 1.5, 2.0, 2.5, 3.3, 5.0]
XS = [1e-8, 1e-5, 1e-3, 0.02, 0.1, 0.5, 1.0, 1.9, 2.0, 2.1, 3.0, 5.0, 10.0, 30.0, 100.0, 300.0, 700.0]


@pytest.mark.parametrize("nu", NUS)
def test_scaled_bessel_k_vs_mpmath(nu):
    worst = 0.0
    for x in XS:
        ref = float(mpmath.besselk(nu, x) * mpmath.exp(x))
        got = oracle.bessel_k_scaled(nu, x)
        worst = max(worst, abs(got - ref) / ref)
    assert worst < 2e-14, worst


@pytest.mark.parametrize("nu", [0.1, 0.5, 1.0, 1.7, 2.5])
def test_bessel_k_vs_scipy(nu):
    for x in [1e-6, 0.01, 0.3, 1.0, 4.0, 20.0, 200.0]:
        ref = sp.kv(nu, x)
        got = oracle.bessel_k(nu, x)
        assert abs(got - ref) <= 1e-13 * ref, (nu, x, got, ref)


@pytest.mark.parametrize("nu", [0.3, 1.0, 1.5, 2.2])
def test_bessel_recurrence(nu):
    # DLMF 10.29.1: K_{ν+1}(x) = K_{ν-1}(x) + (2ν/x) K_ν(x); all terms positive.
    for x in [0.05, 0.7, 2.0, 9.0, 60.0]:
        lhs = oracle.bessel_k_scaled(nu + 1, x)
        rhs = oracle.bessel_k_scaled(abs(nu - 1), x) + (2 * nu / x) * oracle.bessel_k_scaled(nu, x)
        assert abs(lhs - rhs) <= 4e-15 * lhs


@pytest.mark.parametrize("nu", [0.5, 1.0, 1.5, 2.5])
def test_small_argument_limit(nu):
    # x^ν K_ν(x) → 2^(ν-1) Γ(ν) as x → 0 (DLMF 10.30.2); the next term is
    # O(x^min(2ν, 2) log x), far below the tolerance at x = 1e-9 for ν >= 1/2.
    x = 1e-9
    got = x ** nu * oracle.bessel_k(nu, x)
    ref = 2 ** (nu - 1) * math.gamma(nu)
    assert abs(got - ref) <= 1e-6 * ref


@pytest.mark.parametrize("nu", [0.1, 0.2, 0.35])
def test_small_argument_two_terms(nu):
    # For 0 < ν < 1, K_ν = π/2 (I_{-ν} - I_ν)/sin(νπ) (DLMF 10.27.4) and
    # I_{±ν}(x) = (x/2)^{±ν}/Γ(1±ν) (1 + O(x²)), so
    # x^ν K_ν(x) = π/(2 sin νπ) [2^ν/Γ(1-ν) - 2^-ν x^{2ν}/Γ(1+ν)] + O(x²).
    for x in [1e-9, 1e-7]:
        got = x ** nu * oracle.bessel_k(nu, x)
        ref = math.pi / (2 * math.sin(nu * math.pi)) * (
            2 ** nu / math.gamma(1 - nu) - 2 ** -nu * x ** (2 * nu) / math.gamma(1 + nu))
        assert abs(got - ref) <= 1e-12 * ref, (nu, x, got, ref)


def test_half_integer_closed_form():
    # K_{n+1/2}(x) = sqrt(π/(2x)) e^{-x} Σ_k (n+k)! / (k! (n-k)! (2x)^k)  (DLMF 10.49.12)
    for n in range(0, 4):
        for x in [0.01, 0.4, 3.0, 40.0]:
            s = sum(math.factorial(n + k) / (math.factorial(k) * math.factorial(n - k) * (2 * x) ** k)
                    for k in range(n + 1))
            ref = math.sqrt(math.pi / (2 * x)) * s
            got = oracle.bessel_k_scaled(n + 0.5, x)
            assert abs(got - ref) <= 4e-15 * ref, (n, x)


THETAS = [(1.0, 0.1), (2.3, 0.03), (0.7, 0.3)]
RS = [1e-7, 1e-4, 0.003, 0.02, 0.1, 0.25, 0.6, 1.0, 1.4]


@pytest.mark.parametrize("t1,t2", THETAS)
def test_matern_exponential(t1, t2):
    # Sec. 2.2: θ3 = 1/2 reduces to θ1 exp(-r/θ2)
    for r in RS:
        ref = t1 * math.exp(-r / t2)
        got = oracle.matern(r, (t1, t2, 0.5))
        assert abs(got - ref) <= 4e-15 * max(ref, 1e-300), (r, got, ref)


@pytest.mark.parametrize("t1,t2", THETAS)
def test_matern_three_halves_and_five_halves(t1, t2):
    for r in RS:
        x = r / t2
        ref32 = t1 * (1 + x) * math.exp(-x)
        ref52 = t1 * (1 + x + x * x / 3) * math.exp(-x)
        assert abs(oracle.matern(r, (t1, t2, 1.5)) - ref32) <= 5e-15 * max(ref32, 1e-300)
        assert abs(oracle.matern(r, (t1, t2, 2.5)) - ref52) <= 5e-15 * max(ref52, 1e-300)


@pytest.mark.parametrize("t1,t2", THETAS)
def test_matern_whittle(t1, t2):
    # Sec. 2.2: θ3 = 1 gives the Whittle model θ1 (r/θ2) K_1(r/θ2); scipy's k1 is Cephes.
    for r in RS:
        x = r / t2
        ref = t1 * x * sp.k1(x)
        got = oracle.matern(r, (t1, t2, 1.0))
        assert abs(got - ref) <= 1e-13 * max(ref, 1e-300), (r, got, ref)


def test_matern_general_nu_vs_mpmath():
    for nu in [0.3, 0.77, 1.2, 2.0, 3.1]:
        for r in [1e-5, 0.01, 0.07, 0.3, 0.9]:
            t1, t2 = 1.7, 0.08
            x = mpmath.mpf(r) / t2
            ref = float(t1 / (mpmath.mpf(2) ** (nu - 1) * mpmath.gamma(nu)) * x ** nu * mpmath.besselk(nu, x))
            got = oracle.matern(r, (t1, t2, nu))
            assert abs(got - ref) <= 3e-14 * ref, (nu, r)


@pytest.mark.parametrize("nu", [0.05, 0.3, 0.77, 1.0, 1.3, 2.2, 3.2, 10.0, 25.0, 45.0, 50.0])
def test_matern_wide_range_vs_mpmath(nu):
    """x = r/θ2 over [1e-8, 745] (both sides of x = 2, up to where x^ν e^-x
    leaves the binary64 range), including large ν at small x, where x^ν
    underflows and K_ν overflows on their own: 2e-13 relative wherever the
    value is a normal number, within a few subnormal steps elsewhere."""
    xs = list(np.geomspace(1e-8, 745.0, 61)) + [1.999999999, 2.0, 2.000000001, 700.0, 740.0, 745.0]
    for x in xs:
        ref = float(mpmath.mpf(2) ** (1 - nu) / mpmath.gamma(nu) * mpmath.mpf(x) ** nu * mpmath.besselk(nu, x))
        got = oracle.matern(x, (1.0, 1.0, nu))
        if ref >= 2.2250738585072014e-308:
            assert abs(got - ref) <= 2e-13 * ref, (nu, x, got, ref)
        else:
            assert abs(got - ref) <= 64 * 5e-324, (nu, x, got, ref)


def test_matern_at_zero_is_variance():
    for theta in [(1.0, 0.1, 0.5), (2.5, 0.3, 1.7), (0.5, 0.02, 2.5)]:
        assert oracle.matern(0.0, theta) == theta[0]


def test_matern_far_field_underflows_to_zero():
    assert oracle.matern(1.0, (1.0, 1e-3, 0.5)) == 0.0
    assert oracle.matern(1.0, (1.0, 1e-3, 1.3)) == 0.0


def test_cov_matrix_matches_scalar():
    rng = np.random.default_rng(3)
    x1, y1 = rng.random(7), rng.random(7)
    x2, y2 = rng.random(5), rng.random(5)
    th = (1.3, 0.2, 1.1)
    c = oracle.cov_matrix(x1, y1, x2, y2, th)
    for i in range(7):
        for j in range(5):
            dx, dy = x1[i] - x2[j], y1[i] - y2[j]
            r = math.sqrt(dx * dx + dy * dy)
            assert c[i, j] == oracle.matern(r, th)
    s = oracle.cov_symmetric(x1, y1, th)
    assert np.array_equal(s, s.T)
    assert np.all(np.diag(s) == 1.3)
