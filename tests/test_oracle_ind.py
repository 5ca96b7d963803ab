"""Pins of the oracle's independent-blocks (IND) approximation (Sec. 6.8):
off-diagonal blocks of Σ annihilated, diagonal blocks of consecutive
locations kept.  Checked against the masked dense covariance by
eigendecomposition, the closed form for blocks of one location, the exact l
when one block holds every location, and additivity over blocks."""
import math

import numpy as np
import pytest

import geoinputs
import oracle


def masked_loglik(x, y, z, theta, block):
    """Gaussian log-density of z under Σ with every entry between different
    blocks set to zero, by eigendecomposition of the whole masked matrix."""
    n = x.size
    a = oracle.cov_symmetric(x, y, theta)
    blk = np.arange(n) // block
    a = np.where(blk[:, None] == blk[None, :], a, 0.0)
    lam, u = np.linalg.eigh(a)
    return -0.5 * n * math.log(2 * math.pi) - 0.5 * np.sum(np.log(lam)) - 0.5 * np.sum((u.T @ z) ** 2 / lam)


@pytest.mark.parametrize("n,block", [(90, 32), (100, 25), (77, 10), (64, 64)])
@pytest.mark.parametrize("theta", [(1.0, 0.1, 0.5), (1.4, 0.2, 1.5)])
def test_ind_vs_masked_dense(n, block, theta):
    x, y = geoinputs.jittered_grid(n, 21)
    z = geoinputs.normal_vector(n, 21)
    l, ld, q, info = oracle.loglik_ind(x, y, z, theta, block)
    assert info == 0
    assert l == pytest.approx(masked_loglik(x, y, z, theta, block), rel=1e-10)


def test_ind_single_location_blocks_closed_form():
    x, y = geoinputs.jittered_grid(50, 4)
    z = geoinputs.normal_vector(50, 4)
    theta = (1.7, 0.1, 0.5)
    l, ld, q, info = oracle.loglik_ind(x, y, z, theta, 1)
    want = sum(-0.5 * math.log(2 * math.pi) - 0.5 * math.log(theta[0]) - 0.5 * zi * zi / theta[0] for zi in z)
    assert info == 0 and l == pytest.approx(want, rel=1e-13)
    assert ld == pytest.approx(50 * math.log(theta[0]), rel=1e-13)


def test_ind_one_block_is_exact_and_blocks_add():
    n = 120
    x, y = geoinputs.jittered_grid(n, 5)
    z = geoinputs.normal_vector(n, 5)
    theta = (1.0, 0.15, 1.0)
    exact = oracle.loglik(x, y, z, theta)
    assert oracle.loglik_ind(x, y, z, theta, n)[0] == exact[0]
    assert oracle.loglik_ind(x, y, z, theta, 10 * n)[0] == exact[0]
    parts = [oracle.loglik(x[s:s + 40], y[s:s + 40], z[s:s + 40], theta)[0] for s in range(0, n, 40)]
    assert oracle.loglik_ind(x, y, z, theta, 40)[0] == pytest.approx(sum(parts), rel=1e-14)


def test_ind_reports_first_failing_column():
    x, y = geoinputs.jittered_grid(60, 6)
    x[45], y[45] = x[44], y[44]  # duplicate inside the second block of 30
    z = geoinputs.normal_vector(60, 6)
    l, ld, q, info = oracle.loglik_ind(x, y, z, (1.0, 0.1, 0.5), 30)
    assert info == 46 and l == -math.inf


# ------------------------------------------------ kriging under IND (Eq. 5) --

def masked_conditional_mean(x, y, z, miss, theta, block):
    """E[Z_M | Z_O] under the covariance of all locations with every entry
    between different blocks set to zero, by a dense LU solve (numpy) on the
    whole masked matrix — independent of the oracle's per-block Cholesky."""
    n = x.size
    a = oracle.cov_symmetric(x, y, theta)
    blk = np.arange(n) // block
    a = np.where(blk[:, None] == blk[None, :], a, 0.0)
    o, m = ~miss.astype(bool), miss.astype(bool)
    return a[np.ix_(m, o)] @ np.linalg.solve(a[np.ix_(o, o)], z[o])


def _miss(n, k, seed):
    return (np.random.Generator(np.random.PCG64(seed)).permutation(np.arange(n) % k) == 0).astype(np.int32)


@pytest.mark.parametrize("n,block", [(90, 32), (100, 25), (64, 7)])
@pytest.mark.parametrize("theta", [(1.0, 0.1, 0.5), (1.4, 0.2, 1.5)])
def test_krige_ind_vs_masked_dense(n, block, theta):
    x, y = geoinputs.jittered_grid(n, 31)
    z = geoinputs.normal_vector(n, 31)
    miss = _miss(n, 5, 32)
    got, info = oracle.krige_ind(x, y, z, miss, theta, block)
    assert info == 0
    want = masked_conditional_mean(x, y, z, miss, theta, block)
    assert np.max(np.abs(got - want)) <= 1e-10 * np.max(np.abs(want))


def test_krige_ind_single_location_blocks_predict_the_mean():
    """Blocks of one location: a held-out value has no observed neighbour in
    its block, so it is predicted by the zero mean."""
    x, y = geoinputs.jittered_grid(40, 33)
    z = geoinputs.normal_vector(40, 33)
    miss = _miss(40, 4, 34)
    got, info = oracle.krige_ind(x, y, z, miss, (1.6, 0.12, 0.5), 1)
    assert info == 0 and got.size == int(miss.sum()) and np.all(got == 0.0)


def test_krige_ind_one_block_is_exact():
    n = 110
    x, y = geoinputs.jittered_grid(n, 35)
    z = geoinputs.normal_vector(n, 35)
    miss = _miss(n, 6, 36)
    theta = (1.0, 0.15, 1.0)
    o, m = miss == 0, miss != 0
    exact, info = oracle.krige(x[o], y[o], z[o], x[m], y[m], theta)
    assert info == 0
    for block in (n, 3 * n):
        got, info = oracle.krige_ind(x, y, z, miss, theta, block)
        assert info == 0 and np.array_equal(got, exact)


def test_krige_ind_reports_first_failing_location():
    x, y = geoinputs.jittered_grid(60, 37)
    x[45], y[45] = x[44], y[44]
    z = geoinputs.normal_vector(60, 37)
    miss = np.zeros(60, dtype=np.int32)
    miss[[3, 50]] = 1
    _, info = oracle.krige_ind(x, y, z, miss, (1.0, 0.1, 0.5), 30)
    assert info == 46
