"""Pins of the oracle's great-circle distance (Sec. 7.4, haversine formula) and
prediction variance (Sec. 2.3, Eq. 4), each against something other than the
oracle's own formula: exact arcs, the 3-D chord identity, closed forms for
one observed point, dense linear algebra, and limits."""
import math

import numpy as np
import pytest

import geoinputs
import oracle

R = oracle.EARTH_RADIUS_KM
GC = oracle.GREAT_CIRCLE


def chord_distance(l1, p1, l2, p2, radius=R):
    """Great-circle distance from the chord between the two unit vectors,
    d = 2 ρ asin(|u1 - u2| / 2): a different route to the same arc."""
    def unit(lon, lat):
        lo, la = math.radians(lon), math.radians(lat)
        return np.array([math.cos(la) * math.cos(lo), math.cos(la) * math.sin(lo), math.sin(la)])
    c = np.linalg.norm(unit(l1, p1) - unit(l2, p2))
    return 2.0 * radius * math.asin(min(1.0, c / 2.0))


def region_points(n, seed):
    """Jittered grid mapped to a 15° x 15° longitude/latitude box."""
    x, y = geoinputs.jittered_grid(n, seed)
    return -100.0 + 15.0 * x, 30.0 + 15.0 * y


@pytest.mark.parametrize("l1,l2", [(0.0, 90.0), (-100.0, -85.0), (170.0, -170.0)])
def test_gcd_equator_arc(l1, l2):
    dl = abs((l2 - l1 + 180.0) % 360.0 - 180.0)
    assert oracle.distance(l1, 0.0, l2, 0.0, GC, R) == pytest.approx(R * math.radians(dl), rel=1e-13)


@pytest.mark.parametrize("p1,p2", [(-30.0, 45.0), (10.0, 11.0), (-89.0, 89.0)])
def test_gcd_meridian_arc(p1, p2):
    assert oracle.distance(-95.0, p1, -95.0, p2, GC, R) == pytest.approx(R * math.radians(abs(p2 - p1)), rel=1e-13)


def test_gcd_special_arcs():
    assert oracle.distance(12.0, 90.0, 77.0, 0.0, GC, R) == pytest.approx(R * math.pi / 2, rel=1e-13)
    assert oracle.distance(-60.0, 20.0, 120.0, -20.0, GC, R) == pytest.approx(R * math.pi, rel=1e-12)
    assert oracle.distance(-91.3, 37.2, -91.3, 37.2, GC, R) == 0.0
    assert oracle.distance(0.0, 0.0, 1.0, 0.0, GC, 1.0) == pytest.approx(math.radians(1.0), rel=1e-13)


def test_gcd_matches_chord_and_is_a_metric():
    rng = np.random.Generator(np.random.PCG64(4))
    pts = np.column_stack([rng.uniform(-180, 180, 60), rng.uniform(-89, 89, 60)])
    d = np.array([[oracle.distance(*pts[i], *pts[j], GC, R) for j in range(60)] for i in range(60)])
    for i in range(0, 60, 7):
        for j in range(60):
            want = chord_distance(*pts[i], *pts[j])
            assert abs(d[i, j] - want) <= 1e-9 * max(want, 1.0)
    assert np.array_equal(d, d.T)
    assert np.all(d <= math.pi * R * (1 + 1e-15))
    for i, j, k in rng.integers(0, 60, size=(300, 3)):
        assert d[i, k] <= d[i, j] + d[j, k] + 1e-9


def test_gcd_small_scale_is_planar():
    """Over 100 m the sphere is flat: d ≈ ρ sqrt(Δφ² + cos²φ Δλ²)."""
    lat = 38.0
    dlon, dlat = 5e-4, 7e-4
    planar = R * math.hypot(math.radians(dlat), math.cos(math.radians(lat + dlat / 2)) * math.radians(dlon))
    got = oracle.distance(-90.0, lat, -90.0 + dlon, lat + dlat, GC, R)
    assert got == pytest.approx(planar, rel=1e-8)


def test_cov_with_gcd_uses_the_arc():
    x, y = region_points(30, 3)
    theta = (1.0, 150.0, 0.5)
    c = oracle.cov_matrix(x, y, x[:5], y[:5], theta, GC, R)
    for i in range(30):
        for j in range(5):
            want = theta[0] * math.exp(-chord_distance(x[i], y[i], x[j], y[j]) / theta[1])
            assert abs(c[i, j] - want) <= 1e-12


def test_loglik_gcd_vs_eigendecomposition():
    n = 60
    theta = (1.2, 200.0, 1.5)
    x, y = region_points(n, 5)
    z = geoinputs.normal_vector(n, 5)
    a = np.empty((n, n))
    for i in range(n):
        for j in range(n):
            r = chord_distance(x[i], y[i], x[j], y[j]) / theta[1]
            a[i, j] = theta[0] * (1 + r) * math.exp(-r)
    lam, u = np.linalg.eigh(a)
    ref = -0.5 * n * math.log(2 * math.pi) - 0.5 * np.sum(np.log(lam)) - 0.5 * np.sum((u.T @ z) ** 2 / lam)
    l, ld, q, info = oracle.loglik(x, y, z, theta, metric=GC, radius=R)
    assert info == 0
    assert l == pytest.approx(ref, rel=1e-10)


def test_variance_one_observation_closed_form():
    """n = 1: var = θ1 - C(r)² / θ1, prediction = C(r) z / θ1."""
    theta = (1.7, 0.2, 0.5)
    xo, yo, zo = np.array([0.3]), np.array([0.4]), np.array([0.9])
    xn, yn = np.array([0.3, 0.5, 2.0]), np.array([0.4, 0.1, 2.0])
    pred, var, info = oracle.krige(xo, yo, zo, xn, yn, theta, return_variance=True)
    assert info == 0
    for k in range(3):
        c = theta[0] * math.exp(-math.hypot(xn[k] - 0.3, yn[k] - 0.4) / theta[1])
        assert var[k] == pytest.approx(theta[0] - c * c / theta[0], abs=1e-14)
        assert pred[k] == pytest.approx(c * 0.9 / theta[0], abs=1e-14)


@pytest.mark.parametrize("metric", [0, 1])
def test_variance_vs_dense_and_limits(metric):
    n, m = 80, 12
    if metric == 0:
        x, y = geoinputs.jittered_grid(n, 6)
        xn, yn = geoinputs.uniform_points(m, 6)
        theta = (1.3, 0.12, 1.0)
        far = (50.0, 50.0)
    else:
        x, y = region_points(n, 6)
        xn, yn = geoinputs.uniform_points(m, 6)
        xn, yn = -100.0 + 15.0 * xn, 30.0 + 15.0 * yn
        theta = (1.3, 180.0, 1.0)
        far = (80.0, -30.0)
    z = geoinputs.normal_vector(n, 6)
    # observed points and one far point appended
    xq = np.concatenate([xn, x[:3], [far[0]]])
    yq = np.concatenate([yn, y[:3], [far[1]]])
    pred, var, info = oracle.krige(x, y, z, xq, yq, theta, return_variance=True, metric=metric, radius=R)
    assert info == 0
    # dense route with numpy on covariances from scipy's Bessel function
    from scipy.special import kv, gamma

    def cov(r):
        r = np.asarray(r, dtype=float)
        out = np.full(r.shape, theta[0])
        nz = r > 0
        s = r[nz] / theta[1]
        out[nz] = theta[0] / (2 ** (theta[2] - 1) * gamma(theta[2])) * s ** theta[2] * kv(theta[2], s)
        return out

    def dist(a, b, c, d):
        return chord_distance(a, b, c, d) if metric else math.hypot(a - c, b - d)

    s22 = cov(np.array([[dist(x[i], y[i], x[j], y[j]) for j in range(n)] for i in range(n)]))
    s12 = cov(np.array([[dist(xq[k], yq[k], x[j], y[j]) for j in range(n)] for k in range(xq.size)]))
    dense_var = theta[0] - np.einsum("kj,jk->k", s12, np.linalg.solve(s22, s12.T))
    dense_pred = s12 @ np.linalg.solve(s22, z)
    assert np.allclose(var, dense_var, rtol=1e-7, atol=1e-9)
    assert np.allclose(pred, dense_pred, rtol=1e-7, atol=1e-9)
    assert np.all(var[:m] > 0) and np.all(var[:m] < theta[0])
    assert np.all(np.abs(var[m:m + 3]) <= 1e-9)           # at observed points
    assert np.allclose(pred[m:m + 3], z[:3], atol=1e-8)
    assert var[-1] == pytest.approx(theta[0], abs=1e-12)   # far from every observation
