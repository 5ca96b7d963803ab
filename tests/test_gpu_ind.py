"""GPU parity of the independent-blocks (IND) approximation (Sec. 6.8)
against the oracle, and its relation to the exact path."""
import math

import numpy as np
import pytest

import geoinputs
import oracle
from morton_ref import morton_reference

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def g():
    import paper_1708_02835_amd as pkg
    pkg.lib()
    return pkg


@pytest.fixture(scope="module")
def ctx(g):
    c = g.Context(0)
    yield c
    c.close()


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


@pytest.mark.parametrize("n,tile,s", [(1600, 128, 1), (1600, 128, 2), (1600, 128, 3), (1100, 256, 2),
                                      (1300, 512, 1), (1000, 384, 2), (700, 128, 40)])
@pytest.mark.parametrize("theta", [(1.0, 0.1, 0.5), (1.3, 0.07, 1.0)])
def test_ind_parity(g, ctx, n, tile, s, theta):
    x, y = geoinputs.jittered_grid(n, 13)
    z = geoinputs.normal_vector(n, 13)
    ref = oracle.loglik_ind(x, y, z, theta, s * tile)
    assert ref[3] == 0
    r = g.loglik_eval(ctx, dev(x), dev(y), dev(z), theta, g.gl_opts_default(tile=tile, ind_tiles=s))
    assert r["status"] == g.GL_OK and r["tile"] == tile
    assert abs(r["loglik"] - ref[0]) <= 1e-10 * abs(ref[0])
    assert abs(r["logdet"] - ref[1]) <= 1e-10 * abs(ref[1])
    assert abs(r["quad"] - ref[2]) <= 1e-10 * abs(ref[2])


def test_ind_covering_block_equals_exact(g, ctx):
    n, theta = 1500, (1.0, 0.1, 0.5)
    x, y = geoinputs.jittered_grid(n, 14)
    z = geoinputs.normal_vector(n, 14)
    exact = g.loglik_eval(ctx, dev(x), dev(y), dev(z), theta, g.gl_opts_default(tile=256))
    ind = g.loglik_eval(ctx, dev(x), dev(y), dev(z), theta, g.gl_opts_default(tile=256, ind_tiles=6))
    assert ind["loglik"] == exact["loglik"] and ind["logdet"] == exact["logdet"]


def test_ind_morton_order_and_great_circle(g, ctx):
    n, theta = 1200, (1.0, 150.0, 0.5)
    x, y = geoinputs.jittered_grid(n, 15)
    x, y = -100.0 + 15.0 * x, 30.0 + 15.0 * y
    z = geoinputs.normal_vector(n, 15)
    p = morton_reference(x, y)
    ref = oracle.loglik_ind(x[p], y[p], z[p], theta, 256, metric=oracle.GREAT_CIRCLE, radius=6371.0)
    r = g.loglik_eval(ctx, dev(x), dev(y), dev(z), theta,
                      g.gl_opts_default(tile=128, ind_tiles=2, reorder=1, metric=g.GL_GREAT_CIRCLE, radius=6371.0))
    assert r["status"] == g.GL_OK
    assert abs(r["loglik"] - ref[0]) <= 1e-10 * abs(ref[0])


def test_ind_not_spd_reports_global_column(g, ctx):
    """Repeated locations make their block's Σ exactly singular: in exact
    arithmetic the pivot of each repeat's column is 0, so a binary64
    factorisation meets pivots that are zero up to rounding, of either sign.
    Which sign comes out is rounding, not a property of the method (a single
    repeat is a coin flip), so 40 locations of the third block of 256 are
    repeated and what is compared is the column: the device reports NOT_SPD at
    the global column of one of the repeats, and the oracle's factor of that
    block either stops at a repeat or has a pivot there that vanishes to
    rounding."""
    n = 900
    x, y = geoinputs.jittered_grid(n, 16)
    x[600:640], y[600:640] = x[520:560], y[520:560]  # inside the third block of 256
    z = geoinputs.normal_vector(n, 16)
    r = g.loglik_eval(ctx, dev(x), dev(y), dev(z), (1.0, 0.1, 0.5), g.gl_opts_default(tile=128, ind_tiles=2))
    assert r["status"] == g.GL_NOT_SPD and 601 <= r["info"] <= 640 and r["loglik"] == -math.inf
    c = r["info"] - 513  # 0-based column within the block
    L, info = oracle.cholesky(oracle.cov_symmetric(x[512:768], y[512:768], (1.0, 0.1, 0.5)))
    assert info == 0 or 89 <= info <= 128, info
    if info == 0 or info > c + 1:
        assert L[c, c] ** 2 <= 1e-10, (info, c, L[c, c])
    # the other blocks are unaffected: the sum without the failing block matches
    ok = g.loglik_eval(ctx, dev(x[:512]), dev(y[:512]), dev(z[:512]), (1.0, 0.1, 0.5),
                       g.gl_opts_default(tile=128, ind_tiles=2))
    assert abs(ok["loglik"] - oracle.loglik_ind(x[:512], y[:512], z[:512], (1.0, 0.1, 0.5), 256)[0]) <= 1e-10 * abs(ok["loglik"])


def test_ind_rejects_unsupported_options(g, ctx):
    x, y = geoinputs.jittered_grid(300, 17)
    for kw in ({"precision": 2}, {"keep_factor": 1}, {"ind_tiles": -1}):
        with pytest.raises(g.GeolikError):
            g.loglik_eval(ctx, dev(x), dev(y), dev(x), (1.0, 0.1, 0.5), g.gl_opts_default(ind_tiles=2, **kw) if "ind_tiles" not in kw else g.gl_opts_default(**kw))


def test_ind_n100000_is_the_sum_of_exact_block_evaluations(g):
    """At the benchmark size the oracle cannot run every block; the exact path
    (itself pinned to the oracle) evaluates the 49 blocks one by one."""
    n, theta, tile, s = 100000, (1.0, 0.1, 0.5), 512, 4
    x, y = geoinputs.jittered_grid(n, 3000)
    e = geoinputs.normal_vector(n, 3000)
    ctx = g.Context(0)
    try:
        xd, yd, ed = dev(x), dev(y), dev(e)
        zd, info = g.synth_generate(ctx, xd, yd, ed, theta, tile)
        assert info == 0
        r = g.loglik_eval(ctx, xd, yd, zd, theta, g.gl_opts_default(tile=tile, ind_tiles=s))
        assert r["status"] == g.GL_OK
        blk = s * tile
        parts = [g.loglik_eval(ctx, xd[a:a + blk].contiguous(), yd[a:a + blk].contiguous(), zd[a:a + blk].contiguous(),
                               theta, g.gl_opts_default(tile=tile)) for a in range(0, n, blk)]
        total = math.fsum(p["loglik"] for p in parts)
        assert abs(r["loglik"] - total) <= 1e-12 * abs(total)
        exact = g.loglik_eval(ctx, xd, yd, zd, theta, g.gl_opts_default(tile=tile))
        print(f"n=100000 IND s={s}: l_IND={r['loglik']:.6f} exact={exact['loglik']:.6f}")
    finally:
        ctx.close()


# ------------------------------------------------ kriging under IND (k-fold) --

def _folds(n, k, seed):
    return np.random.Generator(np.random.PCG64(seed)).permutation(np.arange(n) % k).astype(np.int32)


def _oracle_cv_ind(x, y, z, theta, folds, k, block):
    out = []
    for f in range(k):
        miss = (folds == f).astype(np.int32)
        pred, info = oracle.krige_ind(x, y, z, miss, theta, block)
        assert info == 0
        out.append(float(np.mean((pred - z[folds == f]) ** 2)))
    return np.array(out)


@pytest.mark.parametrize("s,tile", [(1, 128), (2, 128), (3, 128), (1, 256)])
@pytest.mark.parametrize("theta", [(1.0, 0.1, 0.5), (1.2, 0.08, 1.3)])
def test_ind_krige_cv_parity(g, ctx, s, tile, theta):
    """Blocks of s·b consecutive locations (observed and held-out alike) are
    independent; each held-out value from its block's observed values:
    per-fold MSE against the oracle."""
    n, k = 1100, 5
    x, y = geoinputs.jittered_grid(n, 40)
    e = geoinputs.normal_vector(n, 40)
    z, info = oracle.synth(x, y, e, theta)
    assert info == 0
    folds = _folds(n, k, 41)
    mse, st = g.krige_cv(ctx, dev(x), dev(y), dev(z), theta, folds, g.gl_opts_default(tile=tile, ind_tiles=s))
    assert st == g.GL_OK
    ref = _oracle_cv_ind(x, y, z, theta, folds, k, s * tile)
    assert np.all(np.abs(np.array(mse) - ref) <= 1e-9 * ref), (mse, ref)


@pytest.mark.parametrize("s,tile", [(1, 128), (2, 128), (3, 128), (1, 256), (2, 256)])
def test_ind_krige_cv_predictions_per_location(g, ctx, s, tile):
    """Per-location IND predictions against oracle.krige_ind, element by
    element.  n = 1100 leaves a ragged last block (1100 mod s·b locations);
    every location of that block is put in fold 0, so when fold 0 is held out
    the block observes nothing and its predictions must be exactly 0, and
    when another fold is held out the block holds nothing to predict.
    Tolerance: max(1e-10, 1e-15 κ) · max|z| with κ the largest condition
    number of a block's observed covariance."""
    n, k = 1100, 4
    theta = (1.1, 0.09, 1.2)
    x, y = geoinputs.jittered_grid(n, 48)
    e = geoinputs.normal_vector(n, 48)
    z, info = oracle.synth(x, y, e, theta)
    assert info == 0
    block = s * tile
    folds = _folds(n, k, 49)
    last = (n - 1) // block * block
    assert n - last < block  # ragged
    folds[last:] = 0
    pred = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    mse, st = g.krige_cv(ctx, dev(x), dev(y), dev(z), theta, folds,
                         g.gl_opts_default(tile=tile, ind_tiles=s), pred=pred)
    assert st == g.GL_OK
    pred = pred.cpu().numpy()
    assert np.all(np.isfinite(pred))
    assert np.all(pred[last:] == 0.0)
    for f in range(k):
        miss = folds == f
        ref, info = oracle.krige_ind(x, y, z, miss.astype(np.int32), theta, block)
        assert info == 0
        conds = []
        for a in range(0, n, block):
            kb = ~miss[a:a + block]
            if kb.any():
                conds.append(np.linalg.cond(oracle.cov_symmetric(x[a:a + block][kb], y[a:a + block][kb], theta)))
        tol = max(1e-10, 1e-15 * max(conds)) * np.max(np.abs(z))
        err = np.max(np.abs(pred[miss] - ref))
        assert err <= tol, (f, err, tol)


def test_ind_krige_cv_one_block_is_exact_and_blocks_cost_accuracy(g, ctx):
    """A super tile holding every location is the exact prediction; smaller
    super tiles predict worse (the trend the paper reports for its IND
    prediction experiment)."""
    n, k, tile = 1500, 5, 128
    theta = (1.0, 0.2, 1.5)
    x, y = geoinputs.jittered_grid(n, 42)
    e = geoinputs.normal_vector(n, 42)
    z, info = oracle.synth(x, y, e, theta)
    assert info == 0
    folds = _folds(n, k, 43)
    exact, st = g.krige_cv(ctx, dev(x), dev(y), dev(z), theta, folds, g.gl_opts_default(tile=tile))
    assert st == g.GL_OK
    whole, st = g.krige_cv(ctx, dev(x), dev(y), dev(z), theta, folds, g.gl_opts_default(tile=tile, ind_tiles=64))
    assert st == g.GL_OK
    assert np.all(np.abs(np.array(whole) - np.array(exact)) <= 1e-9 * np.array(exact))
    means = [float(np.mean(g.krige_cv(ctx, dev(x), dev(y), dev(z), theta, folds,
                                      g.gl_opts_default(tile=tile, ind_tiles=s))[0])) for s in (1, 2, 4)]
    assert float(np.mean(exact)) < min(means) and means[2] < means[0]


def test_ind_krige_cv_rejects_morton_order(g, ctx):
    x, y = geoinputs.jittered_grid(300, 46)
    z = geoinputs.normal_vector(300, 46)
    with pytest.raises(g.GeolikError):
        g.krige_cv(ctx, dev(x), dev(y), dev(z), (1.0, 0.1, 0.5), _folds(300, 3, 47),
                   g.gl_opts_default(tile=128, ind_tiles=2, reorder=1))


def test_ind_krige_cv_reports_failing_fold(g, ctx):
    n, k = 600, 3
    x, y = geoinputs.jittered_grid(n, 44)
    folds = _folds(n, k, 45)
    # 30 locations repeated within the same block of 1024 and the same fold:
    # every fold observes some repeated pairs, whose block then fails
    rep = np.arange(30)
    x[300 + rep], y[300 + rep] = x[rep], y[rep]
    folds[300 + rep] = folds[rep]
    z = geoinputs.normal_vector(n, 44)
    mse, st = g.krige_cv(ctx, dev(x), dev(y), dev(z), (1.0, 0.1, 0.5), folds,
                         g.gl_opts_default(tile=128, ind_tiles=8))
    assert st == g.GL_NOT_SPD and any(math.isnan(v) for v in mse)
