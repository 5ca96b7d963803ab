"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

Element-wise parity where the oracle can afford the size (several tiles and a
ragged tail), scalar parity of l(θ), log|Σ| and ZᵀΣ⁻¹Z, and the degenerate
cases (n = 1, n below one tile, a singular Σ).  Tolerances:

* Σ(θ) entries: 1e-12 relative (+1e-300 absolute).  Both sides evaluate
  x^ν e^-x through an exponential whose argument reaches ~745 in magnitude, so
  each carries up to ~745 ulp of relative rounding there; elsewhere they agree
  to a few ulp.
* l(θ): 1e-10 relative (the stated FP64 bound) when Σ is well conditioned;
  for ill-conditioned θ the bound is 4 × the noise floor of binary64 itself:
  the largest distance from the oracle of other correct FP64 evaluations of
  the same l (the oracle on reordered locations, LAPACK's Cholesky, the tiled
  right-looking order, and LAPACK on Σ with ±1 ulp moved into each entry,
  i.e. a different correctly rounded Eq. (2)), floored at 1e-10.
"""
import math

import numpy as np
import pytest

import geoinputs
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def g():
    import paper_1708_02835_amd as pkg
    pkg.lib()  # fails loudly when the library is missing
    return pkg


@pytest.fixture(scope="module")
def ctx(g):
    c = g.Context(0)
    yield c
    c.close()


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def _tiled_loglik(S, z, b):
    """Right-looking tile Cholesky with LAPACK tile kernels (the same blocking
    as the device path), then the Alg. 2 scalars — one more correct FP64
    evaluation order of the same l."""
    import scipy.linalg as sla
    n = S.shape[0]
    nt = -(-n // b)
    A = np.eye(nt * b)
    A[:n, :n] = S
    for k in range(nt):
        ks = slice(k * b, (k + 1) * b)
        A[ks, ks] = np.linalg.cholesky(A[ks, ks])
        for i in range(k + 1, nt):
            isl = slice(i * b, (i + 1) * b)
            A[isl, ks] = sla.solve_triangular(A[ks, ks], A[isl, ks].T, lower=True).T
        for j in range(k + 1, nt):
            js = slice(j * b, (j + 1) * b)
            A[j * b:, js] -= A[j * b:, ks] @ A[js, ks].T
    L = np.tril(A)[:n, :n]
    w = sla.solve_triangular(L, z, lower=True)
    return -0.5 * w @ w - np.sum(np.log(np.diag(L))) - 0.5 * n * math.log(2 * math.pi)


def noise_floor(x, y, z, theta, reps=3):
    """Spread of correct binary64 evaluations of one l: the largest relative
    distance from the oracle's value of (a) the oracle on reordered locations
    (exact arithmetic leaves l unchanged), (b) LAPACK's Cholesky on the
    oracle's Σ, (c) the tiled right-looking order at tiles 128, 256, 512,
    (d) LAPACK on Σ with every entry moved by a random -1/0/+1 ulp, which is
    how far two correctly rounded evaluations of Eq. (2) may differ."""
    import scipy.linalg as sla
    a = oracle.loglik(x, y, z, theta)[0]
    worst = 0.0
    for seed in range(reps):
        perm = np.random.default_rng(seed).permutation(x.size)
        worst = max(worst, rel(oracle.loglik(x[perm], y[perm], z[perm], theta)[0], a))
    S = oracle.cov_symmetric(x, y, theta)
    L = np.linalg.cholesky(S)
    w = sla.solve_triangular(L, z, lower=True)
    lap = -0.5 * w @ w - np.sum(np.log(np.diag(L))) - 0.5 * x.size * math.log(2 * math.pi)
    worst = max(worst, rel(lap, a))
    for b in (128, 256, 512):
        worst = max(worst, rel(_tiled_loglik(S, z, b), a))
    rng = np.random.default_rng(1)
    for _ in range(reps):
        p = np.triu(rng.integers(-1, 2, size=S.shape), 1)
        p = p + p.T
        Sp = np.where(p > 0, np.nextafter(S, np.inf), np.where(p < 0, np.nextafter(S, -np.inf), S))
        Lp = np.linalg.cholesky(Sp)
        wp = sla.solve_triangular(Lp, z, lower=True)
        lp = -0.5 * wp @ wp - np.sum(np.log(np.diag(Lp))) - 0.5 * x.size * math.log(2 * math.pi)
        worst = max(worst, rel(lp, a))
    return worst


# ------------------------------------------------------------------ layouts --

@pytest.mark.parametrize("which", [0, 1, 2, 3])
def test_matrix_core_lane_layout(g, ctx, which):
    out = g.gl_selftest(ctx, which)
    lanes = np.arange(64)
    if which in (0, 1):
        A = np.array([[(i + 1) + 0.25 * k for k in range(4)] for i in range(16)])
        Bm = np.array([[(2 * j - 7) - 0.5 * k for j in range(16)] for k in range(4)])
        if which == 1:
            A, Bm = A.astype(np.float32).astype(np.float64), Bm.astype(np.float32).astype(np.float64)
    else:
        A = np.array([[(i + 1) + (k & 3) for k in range(32)] for i in range(16)], dtype=np.float64)
        Bm = np.array([[(j % 5) - (k % 3) for j in range(16)] for k in range(32)], dtype=np.float64)
    D = A @ Bm
    if which == 0:  # FP64 form: rows interleaved by 4
        expect = np.array([D[l // 16 + 4 * r, l % 16] for l in lanes for r in range(4)])
    else:
        expect = np.array([D[4 * (l // 16) + r, l % 16] for l in lanes for r in range(4)])
    assert np.array_equal(out, expect)


# ----------------------------------------------------------- Σ generation --

@pytest.mark.parametrize("nu", [0.5, 1.5, 2.5, 1.0, 0.3, 0.77, 3.2])
def test_matern_generate_elementwise(g, ctx, nu):
    x1, y1 = geoinputs.jittered_grid(333, 1)
    x2, y2 = geoinputs.uniform_points(171, 2)
    theta = (1.7, 0.09, nu)
    ref = oracle.cov_matrix(x1, y1, x2, y2, theta)
    out = g.matern_generate(ctx, dev(x1), dev(y1), dev(x2), dev(y2), theta).cpu().numpy().T
    err = np.abs(out - ref) - 1e-12 * np.abs(ref)
    assert np.all(err <= 1e-300), float(np.max(np.abs(out - ref) / np.maximum(np.abs(ref), 1e-300)))


NORMAL_MIN = 2.2250738585072014e-308


@pytest.mark.parametrize("nu", [0.3, 0.77, 1.0, 1.3, 2.2, 3.2, 45.0])
@pytest.mark.parametrize("theta2", [1.0, 0.013])
def test_matern_generate_wide_range(g, ctx, nu, theta2):
    """x = r/θ2 over [1e-8, 2500] through matern_generate: Temme's series
    (x <= 2, both sides of 2), Miller's recurrence with its shallow depth at
    large x, the far field (normal values past x = 745 at large ν, the cutoff
    past 2000), and x < 1e-3; fixed coordinates on a line, θ2 scaling them.
    ≤ 1e-12 relative to the oracle wherever its value is a normal number,
    else within a few subnormal steps; no NaN."""
    xs = np.concatenate([np.geomspace(1e-8, 745.0, 181), [1.999999999, 2.0, 2.000000001, 15.9, 16.1, 30.0],
                         np.linspace(745.0, 765.0, 9), [900.0, 1200.0, 1999.0, 2001.0, 2500.0]])
    x1, y1 = xs * theta2, np.zeros(xs.size)
    x2 = np.array([0.0, 0.0, -0.25 * theta2])
    y2 = np.array([0.0, 1e-3 * theta2, 0.5 * theta2])
    theta = (1.0, theta2, nu)
    ref = oracle.cov_matrix(x1, y1, x2, y2, theta)
    out = g.matern_generate(ctx, dev(x1), dev(y1), dev(x2), dev(y2), theta).cpu().numpy().T
    assert not np.any(np.isnan(out))
    normal = np.abs(ref) >= NORMAL_MIN
    relerr = np.abs(out - ref)[normal] / np.abs(ref)[normal]
    assert np.all(relerr <= 1e-12), float(np.max(relerr))
    assert np.all(np.abs(out - ref)[~normal] <= 64 * 5e-324)


def test_matern_generate_zero_distance_and_far_field(g, ctx):
    x = np.array([0.25, 0.25, 500.0])
    y = np.array([0.5, 0.5, -300.0])
    out = g.matern_generate(ctx, dev(x), dev(y), dev(x), dev(y), (2.5, 0.1, 1.3)).cpu().numpy().T
    assert out[0, 0] == 2.5 and out[0, 1] == 2.5 and out[2, 2] == 2.5
    assert out[0, 2] == 0.0 and out[2, 1] == 0.0


# ------------------------------------------------------------------ l(θ) ---

SMALL = [(1, 128), (2, 128), (17, 128), (127, 128), (128, 128), (129, 128), (255, 128), (256, 256),
         (257, 256), (400, 128), (513, 256), (700, 512), (1100, 384)]


@pytest.mark.parametrize("n,tile", SMALL)
@pytest.mark.parametrize("theta", [(1.0, 0.1, 0.5), (1.3, 0.05, 1.3)])
def test_loglik_parity_small(g, ctx, n, tile, theta):
    x, y = geoinputs.jittered_grid(n, 100 + n)
    z = geoinputs.normal_vector(n, 100 + n)
    l, ld, q, info = oracle.loglik(x, y, z, theta)
    assert info == 0
    r = g.loglik_eval(ctx, dev(x), dev(y), dev(z), theta, g.gl_opts_default(tile=tile))
    assert r["status"] == g.GL_OK and r["info"] == 0 and r["tile"] == tile
    assert rel(r["loglik"], l) <= 1e-10
    assert abs(r["logdet"] - ld) <= 1e-10 * max(1.0, abs(ld))
    assert rel(r["quad"], q) <= 1e-10


@pytest.mark.parametrize("tile", [0, 128, 256, 512])
def test_loglik_config_n1600(g, ctx, tile):
    # 40×40 jittered grid, θ = (1, 0.1, 0.5), Z = L e with e ~ N(0, 1) (Alg. 1 on the oracle)
    n = 1600
    theta = (1.0, 0.1, 0.5)
    x, y = geoinputs.jittered_grid(n, 1000)
    e = geoinputs.normal_vector(n, 1000)
    z, info = oracle.synth(x, y, e, theta)
    assert info == 0
    l, ld, q, _ = oracle.loglik(x, y, z, theta)
    r = g.loglik_eval(ctx, dev(x), dev(y), dev(z), theta, g.gl_opts_default(tile=tile))
    assert r["status"] == g.GL_OK
    assert rel(r["loglik"], l) <= 1e-10, (r["loglik"], l)
    assert rel(r["logdet"], ld) <= 1e-10
    assert rel(r["quad"], q) <= 1e-10


@pytest.mark.parametrize("theta", [(1.0, 0.03, 1.5), (0.8, 0.2, 1.0), (1.0, 0.25, 2.5), (2.0, 0.1, 0.77)])
def test_loglik_parity_general_nu(g, ctx, theta):
    n = 900
    x, y = geoinputs.jittered_grid(n, 7)
    z = geoinputs.normal_vector(n, 7)
    l, ld, q, info = oracle.loglik(x, y, z, theta)
    assert info == 0
    tol = max(1e-10, 4 * noise_floor(x, y, z, theta))
    r = g.loglik_eval(ctx, dev(x), dev(y), dev(z), theta, g.gl_opts_default(tile=256))
    assert r["status"] == g.GL_OK
    assert rel(r["loglik"], l) <= tol, (r["loglik"], l, tol)


@pytest.mark.parametrize("n,tile", [(700, 128), (700, 256), (530, 512)])
def test_factor_parity(g, ctx, n, tile):
    theta = (1.0, 0.08, 1.5)
    x, y = geoinputs.jittered_grid(n, 3)
    z = geoinputs.normal_vector(n, 3)
    _, _, _, info, L = oracle.loglik(x, y, z, theta, return_factor=True)
    r = g.loglik_eval(ctx, dev(x), dev(y), dev(z), theta, g.gl_opts_default(tile=tile, keep_factor=1))
    try:
        assert r["status"] == g.GL_OK and r["factor"]
        Lg = g.gl_factor_to_dense(ctx, r["factor"]).cpu().numpy().T  # column-major n×n
        assert np.all(np.triu(Lg, 1) == 0.0)
        a = oracle.cov_symmetric(x, y, theta)
        cond = np.linalg.cond(a)
        err = np.max(np.abs(Lg - L)) / np.max(np.abs(L))
        assert err <= 1e-15 * n * cond, (err, cond)
        res = np.linalg.norm(Lg @ Lg.T - a) / np.linalg.norm(a)
        assert res <= 4 * n * np.finfo(float).eps
    finally:
        if r["factor"]:
            g.gl_factor_release(ctx, r["factor"])


def test_not_spd_reports_info(g, ctx):
    x, y = geoinputs.jittered_grid(300, 5)
    x[1], y[1] = x[0], y[0]  # duplicate location → singular Σ, pivot 2 vanishes exactly
    z = geoinputs.normal_vector(300, 5)
    _, _, _, info = oracle.loglik(x, y, z, (1.0, 0.1, 0.5))
    assert info == 2
    r = g.loglik_eval(ctx, dev(x), dev(y), dev(z), (1.0, 0.1, 0.5), g.gl_opts_default(tile=128))
    assert r["status"] == g.GL_NOT_SPD and r["info"] == 2 and r["loglik"] == -math.inf
    # the context stays usable
    x2, y2 = geoinputs.jittered_grid(200, 6)
    z2 = geoinputs.normal_vector(200, 6)
    r2 = g.loglik_eval(ctx, dev(x2), dev(y2), dev(z2), (1.0, 0.1, 0.5))
    assert r2["status"] == g.GL_OK
    assert rel(r2["loglik"], oracle.loglik(x2, y2, z2, (1.0, 0.1, 0.5))[0]) <= 1e-10


def test_invalid_arguments(g, ctx):
    x, y = geoinputs.jittered_grid(10, 1)
    z = geoinputs.normal_vector(10, 1)
    for theta in [(0.0, 0.1, 0.5), (1.0, -0.1, 0.5), (1.0, 0.1, 0.0), (1.0, 0.1, 60.0)]:
        with pytest.raises(g.GeolikError) as ei:
            g.loglik_eval(ctx, dev(x), dev(y), dev(z), theta)
        assert ei.value.status == g.GL_EINVAL
    with pytest.raises(g.GeolikError):
        g.loglik_eval(ctx, dev(x), dev(y), dev(z), (1, 0.1, 0.5), g.gl_opts_default(tile=100))


# --------------------------------------------------------------- kriging ---

@pytest.mark.parametrize("n,tile,theta", [(900, 128, (1.0, 0.1, 0.5)), (1000, 256, (1.2, 0.07, 1.5)),
                                          (650, 512, (0.9, 0.12, 0.9))])
def test_krige_parity(g, ctx, n, tile, theta):
    x, y = geoinputs.jittered_grid(n, 17)
    z = geoinputs.normal_vector(n, 17)
    xn, yn = geoinputs.uniform_points(37, 17)
    xn = np.concatenate([xn, x[[5, n - 1]]])  # two held-out points on observed locations
    yn = np.concatenate([yn, y[[5, n - 1]]])
    ref, info = oracle.krige(x, y, z, xn, yn, theta)
    assert info == 0
    r = g.loglik_eval(ctx, dev(x), dev(y), dev(z), theta, g.gl_opts_default(tile=tile, keep_factor=1))
    try:
        out = g.krige_predict(ctx, r["factor"], dev(xn), dev(yn)).cpu().numpy()
    finally:
        g.gl_factor_release(ctx, r["factor"])
    cond = np.linalg.cond(oracle.cov_symmetric(x, y, theta))
    tol = max(1e-10, 1e-15 * cond) * np.max(np.abs(z))
    assert np.max(np.abs(out - ref)) <= tol, (np.max(np.abs(out - ref)), tol)
    assert abs(out[-2] - z[5]) <= tol and abs(out[-1] - z[n - 1]) <= tol


# ------------------------------------------------------------ generator ---

@pytest.mark.parametrize("n,tile", [(600, 128), (777, 256)])
def test_synth_parity(g, ctx, n, tile):
    theta = (1.0, 0.1, 0.5)
    x, y = geoinputs.jittered_grid(n, 23)
    e = geoinputs.normal_vector(n, 23)
    ref, info = oracle.synth(x, y, e, theta)
    zg, ginfo = g.synth_generate(ctx, dev(x), dev(y), dev(e), theta, tile)
    assert ginfo == 0
    assert np.max(np.abs(zg.cpu().numpy() - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("n,tile", [(700, 128), (700, 256), (300, 0)])
def test_matern_generate_lower_tiles(g, ctx, n, tile):
    """Layout GL_LAYOUT_LOWER_TILES: the packed lower tiles of Σ(set 1) equal
    the dense layout entry for entry (same evaluator), with the identity
    padding beyond n; at n = 300 the entries also match the oracle's Eq. (2)."""
    theta = (1.3, 0.07, 1.5)
    x, y = geoinputs.jittered_grid(n, 61)
    xd, yd = dev(x), dev(y)
    tiles, b = g.matern_generate_tiles(ctx, xd, yd, theta, g.gl_opts_default(tile=tile))
    assert b == g.gl_pick_tile(n, tile)
    dense = g.matern_generate(ctx, xd, yd, xd, yd, theta).cpu().numpy().T
    t = tiles.cpu().numpy()
    nt = -(-n // b)
    full = np.zeros((nt * b, nt * b))
    for i in range(nt):
        for j in range(i + 1):
            off = (i * (i + 1) // 2 + j) * b * b
            full[i * b:(i + 1) * b, j * b:(j + 1) * b] = t[off:off + b * b].reshape(b, b).T
    low = np.tril_indices(n)
    assert np.allclose(full[:n, :n][low], dense[low], rtol=1e-14, atol=0.0)
    pad = full[n:, :]
    assert np.array_equal(pad[:, :n], np.zeros((nt * b - n, n)))
    assert np.array_equal(np.tril(full[n:, n:]), np.eye(nt * b - n))
    if n <= 300:
        ref = oracle.cov_symmetric(x, y, theta)
        assert np.max(np.abs(full[:n, :n][low] - ref[low]) / np.abs(ref[low])) <= 1e-12
    # Σ of one set only: another set 2, or a bad layout, is rejected
    with pytest.raises(g.GeolikError):
        bad = g.gl_opts_default(layout=g.GL_LAYOUT_LOWER_TILES)
        g.matern_generate(ctx, xd, yd, xd[:10], yd[:10], theta, bad,
                          out=torch.empty(n * 10, dtype=torch.float64, device="cuda"))
    with pytest.raises(g.GeolikError):
        g.matern_generate(ctx, xd, yd, xd, yd, theta, g.gl_opts_default(layout=7))
