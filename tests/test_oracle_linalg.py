"""Pins for the oracle's dense kernels: Cholesky, triangular solves, TRMV.

Pinned against LAPACK through scipy (an independent implementation), against
exact results (θ1·I), against the backward-error bound of Cholesky, and
against LAPACK's info convention for a matrix that is not positive definite.
"""
import numpy as np
import pytest
import scipy.linalg as sla
from scipy.linalg import lapack

import geoinputs
import oracle

EPS = np.finfo(np.float64).eps


def _sigma(n, theta, seed=0):
    x, y = geoinputs.jittered_grid(n, seed)
    return oracle.cov_symmetric(x, y, theta)


@pytest.mark.parametrize("n,theta", [(50, (1.0, 0.1, 0.5)), (120, (1.0, 0.03, 1.5)),
                                     (200, (2.0, 0.2, 1.0)), (64, (1.0, 0.3, 2.5))])
def test_cholesky_matches_lapack_and_residual(n, theta):
    a = _sigma(n, theta)
    l, info = oracle.cholesky(a)
    assert info == 0
    assert np.all(np.triu(l, 1) == 0.0)
    ref = sla.cholesky(a, lower=True)
    # forward error of two backward-stable factorisations: bounded by cond · eps
    cond = np.linalg.cond(a)
    assert np.max(np.abs(l - ref)) <= 50 * n * EPS * cond * np.max(np.abs(ref))
    res = np.linalg.norm(l @ l.T - a) / np.linalg.norm(a)
    assert res <= 4 * n * EPS


def test_cholesky_scaled_identity_exact():
    a = 2.25 * np.eye(9)
    l, info = oracle.cholesky(a)
    assert info == 0
    assert np.array_equal(l, 1.5 * np.eye(9))


@pytest.mark.parametrize("bad", [0, 3, 7])
def test_cholesky_not_spd_info_matches_lapack(bad):
    rng = np.random.default_rng(bad)
    q = np.linalg.qr(rng.standard_normal((10, 10)))[0]
    ev = np.linspace(1.0, 3.0, 10)
    a = (q * ev) @ q.T
    a = (a + a.T) / 2
    # make the leading (bad+1)×(bad+1) block indefinite
    a[bad, bad] = -1.0 + (a[bad, :bad] @ np.linalg.solve(a[:bad, :bad], a[:bad, bad]) if bad else 0.0)
    _, info = oracle.cholesky(a)
    _, linfo = lapack.dpotrf(a, lower=1)
    assert info == linfo == bad + 1


def test_triangular_solves_and_trmv():
    a = _sigma(150, (1.0, 0.1, 0.5))
    l, _ = oracle.cholesky(a)
    rng = np.random.default_rng(1)
    z = rng.standard_normal(150)
    w = oracle.forward(l, z)
    assert np.allclose(w, sla.solve_triangular(l, z, lower=True), rtol=1e-12, atol=1e-12)
    v = oracle.backward(l, w)
    assert np.allclose(v, sla.solve_triangular(l.T, w, lower=False), rtol=1e-12, atol=1e-12)
    assert np.allclose(v, np.linalg.solve(a, z), rtol=1e-9, atol=1e-9)
    e = rng.standard_normal(150)
    assert np.allclose(oracle.trmv(l, e), l @ e, rtol=1e-13, atol=1e-13)


def test_logdet_and_dot():
    a = _sigma(80, (1.0, 0.1, 0.5))
    l, _ = oracle.cholesky(a)
    sign, ld = np.linalg.slogdet(a)
    assert sign > 0
    assert abs(oracle.logdet(l) - ld) <= 1e-11 * abs(ld)
    w = np.random.default_rng(2).standard_normal(1000)
    assert abs(oracle.dot(w) - float(np.dot(w, w))) <= 1e-13 * np.dot(w, w)
