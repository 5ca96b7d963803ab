"""Pins for the oracle's l(θ) (Sec. 2 Eq. (1), Alg. 2), kriging (Eq. (5),
Alg. 3) and data generator (Alg. 1).

Each pin comes from outside the oracle's own code path: closed forms for
n = 1 and n = 2, eigendecomposition brute force, mpmath at 30 digits, exact
algebraic identities (θ1 scaling, permutation invariance), the near-diagonal
limit where Σ = θ1·I exactly, and the interpolation property of kriging.
"""
import math

import mpmath
import numpy as np
import pytest

import geoinputs
import oracle

LOG2PI = math.log(2 * math.pi)


def test_n1_closed_form():
    for theta in [(1.0, 0.1, 0.5), (2.7, 0.3, 1.3)]:
        z = 0.83
        l, ld, q, info = oracle.loglik([0.4], [0.6], [z], theta)
        assert info == 0
        ref = -0.5 * math.log(2 * math.pi * theta[0]) - z * z / (2 * theta[0])
        assert abs(l - ref) <= 1e-15 * abs(ref)
        assert abs(ld - math.log(theta[0])) <= 1e-15


def test_n2_closed_form():
    for theta in [(1.0, 0.1, 0.5), (1.8, 0.25, 1.5)]:
        x, y = [0.1, 0.17], [0.2, 0.13]
        z1, z2 = 0.5, -1.2
        r = math.hypot(0.07, 0.07)
        t1, t2, _ = theta
        rho = oracle.matern(r, theta) / t1
        if theta[2] == 0.5:
            assert abs(rho - math.exp(-r / t2)) < 1e-15
        det = t1 * t1 * (1 - rho * rho)
        quad = (z1 * z1 - 2 * rho * z1 * z2 + z2 * z2) / (t1 * (1 - rho * rho))
        ref = -LOG2PI - 0.5 * math.log(det) - 0.5 * quad
        l, ld, q, info = oracle.loglik(x, y, [z1, z2], theta)
        assert abs(ld - math.log(det)) <= 1e-13
        assert abs(q - quad) <= 1e-13 * quad
        assert abs(l - ref) <= 1e-13 * abs(ref)


@pytest.mark.parametrize("n,theta", [(16, (1.0, 0.1, 0.5)), (40, (1.5, 0.2, 1.5)),
                                     (64, (0.8, 0.05, 1.0)), (64, (1.0, 0.3, 2.5))])
def test_vs_eigendecomposition(n, theta):
    x, y = geoinputs.jittered_grid(n, 7)
    z = geoinputs.normal_vector(n, 7)
    a = oracle.cov_symmetric(x, y, theta)
    lam, u = np.linalg.eigh(a)
    assert lam.min() > 0
    logdet = float(np.sum(np.log(lam)))
    quad = float(np.sum((u.T @ z) ** 2 / lam))
    ref = -0.5 * n * LOG2PI - 0.5 * logdet - 0.5 * quad
    l, ld, q, info = oracle.loglik(x, y, z, theta)
    cond = lam.max() / lam.min()
    tol = 1e-14 * cond
    assert abs(ld - logdet) <= tol * max(1.0, abs(logdet))
    assert abs(q - quad) <= tol * quad
    assert abs(l - ref) <= tol * abs(ref)


def test_vs_mpmath_high_precision():
    n = 10
    theta = (1.3, 0.2, 0.5)
    x, y = geoinputs.jittered_grid(n, 11)
    z = geoinputs.normal_vector(n, 11)
    mpmath.mp.dps = 30
    # build Σ in 30-digit arithmetic from the exponential closed form
    a = mpmath.matrix(n, n)
    for i in range(n):
        for j in range(n):
            r = mpmath.sqrt((mpmath.mpf(x[i]) - x[j]) ** 2 + (mpmath.mpf(y[i]) - y[j]) ** 2)
            a[i, j] = theta[0] * mpmath.exp(-r / theta[1])
    L = mpmath.cholesky(a)
    w = mpmath.lu_solve(L, mpmath.matrix(list(z)))
    logdet = 2 * sum(mpmath.log(L[i, i]) for i in range(n))
    quad = sum(w[i] ** 2 for i in range(n))
    ref = float(-n / 2 * mpmath.log(2 * mpmath.pi) - logdet / 2 - quad / 2)
    l, ld, q, info = oracle.loglik(x, y, z, theta)
    assert abs(l - ref) <= 1e-13 * abs(ref)
    assert abs(ld - float(logdet)) <= 1e-13 * abs(float(logdet))


@pytest.mark.parametrize("theta", [(1.0, 0.1, 0.5), (1.0, 0.05, 1.5), (1.0, 0.1, 0.8)])
def test_theta1_scaling(theta):
    # Σ(θ1, θ2, θ3) = θ1 Σ(1, θ2, θ3) exactly in real arithmetic, hence
    # l = -n/2 log 2π - n/2 log θ1 - ½ logdet₁ - q₁ / (2 θ1).
    n = 300
    x, y = geoinputs.jittered_grid(n, 5)
    z = geoinputs.normal_vector(n, 5)
    _, ld1, q1, _ = oracle.loglik(x, y, z, (1.0, theta[1], theta[2]))
    for t1 in [0.3, 2.0, 7.5]:
        l, ld, q, _ = oracle.loglik(x, y, z, (t1, theta[1], theta[2]))
        ref = -0.5 * n * LOG2PI - 0.5 * n * math.log(t1) - 0.5 * ld1 - q1 / (2 * t1)
        assert abs(l - ref) <= 1e-12 * abs(ref)


def test_near_diagonal_limit():
    # θ2 so small that every off-diagonal exp(-r/θ2) underflows: Σ = θ1 I exactly.
    n = 400
    x, y = geoinputs.jittered_grid(n, 3)
    z = geoinputs.normal_vector(n, 3)
    for theta in [(1.0, 1e-6, 0.5), (2.5, 1e-6, 1.5), (0.7, 1e-6, 1.1)]:
        l, ld, q, info = oracle.loglik(x, y, z, theta)
        ref_ld = n * math.log(theta[0])
        ref_q = float(np.sum(z * z)) / theta[0]
        ref = -0.5 * n * math.log(2 * math.pi * theta[0]) - 0.5 * ref_q
        assert abs(ld - ref_ld) <= 1e-14 * abs(ref_ld) + 1e-12
        assert abs(q - ref_q) <= 1e-14 * ref_q
        assert abs(l - ref) <= 1e-14 * abs(ref)


def test_permutation_invariance():
    n = 250
    x, y = geoinputs.jittered_grid(n, 9)
    z = geoinputs.normal_vector(n, 9)
    perm = np.random.default_rng(4).permutation(n)
    for theta in [(1.0, 0.1, 0.5), (1.0, 0.05, 1.5)]:
        a = oracle.loglik(x, y, z, theta)
        b = oracle.loglik(x[perm], y[perm], z[perm], theta)
        assert abs(a[0] - b[0]) <= 1e-12 * abs(a[0])


def test_not_spd_reports_info():
    # Two identical locations make Σ singular: the second pivot is exactly 0
    # for the exponential model (θ3 = 1/2, r = 0 → θ1 on both rows).
    x = np.array([0.1, 0.1, 0.5])
    y = np.array([0.2, 0.2, 0.7])
    l, ld, q, info = oracle.loglik(x, y, [1.0, 2.0, 3.0], (1.0, 0.1, 0.5))
    assert info == 2
    assert l == -math.inf


def test_krige_vs_dense_solve_and_interpolation():
    n = 60
    theta = (1.2, 0.15, 1.5)
    x, y = geoinputs.jittered_grid(n, 21)
    z = geoinputs.normal_vector(n, 21)
    xn, yn = geoinputs.uniform_points(5, 21)
    # held-out points include two observed locations: kriging interpolates exactly there
    xn = np.concatenate([xn, x[[3, 40]]])
    yn = np.concatenate([yn, y[[3, 40]]])
    got, info = oracle.krige(x, y, z, xn, yn, theta)
    assert info == 0
    s22 = oracle.cov_symmetric(x, y, theta)
    s12 = oracle.cov_matrix(xn, yn, x, y, theta)
    ref = s12 @ np.linalg.solve(s22, z)
    cond = np.linalg.cond(s22)
    assert np.allclose(got, ref, rtol=0, atol=1e-15 * cond * np.abs(z).max() * 10)
    assert abs(got[5] - z[3]) <= 1e-15 * cond
    assert abs(got[6] - z[40]) <= 1e-15 * cond


def test_krige_far_points_vanish():
    x, y = geoinputs.jittered_grid(30, 2)
    z = geoinputs.normal_vector(30, 2)
    got, _ = oracle.krige(x, y, z, [500.0, -400.0], [500.0, 800.0], (1.0, 0.1, 0.5))
    assert np.all(got == 0.0)


def test_synth_is_factor_times_e():
    n = 100
    theta = (1.0, 0.1, 0.5)
    x, y = geoinputs.jittered_grid(n, 13)
    e = geoinputs.normal_vector(n, 13)
    z, info = oracle.synth(x, y, e, theta)
    assert info == 0
    a = oracle.cov_symmetric(x, y, theta)
    import scipy.linalg as sla
    ref = sla.cholesky(a, lower=True) @ e
    assert np.allclose(z, ref, rtol=1e-12, atol=1e-12)
    # quad at the generating θ equals ||e||² (Z = L e ⇒ L⁻¹ Z = e)
    _, _, q, _ = oracle.loglik(x, y, z, theta)
    assert abs(q - float(e @ e)) <= 1e-10 * float(e @ e)
