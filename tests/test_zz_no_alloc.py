"""loglik_eval_noalloc (workspace in the library's static device array)
against loglik_eval (workspace allocated by the context): the same kernels
on the same inputs, so the results must be bit-identical; two calls in a
row, the second smaller than the first, plus the oracle at 1e-10 on the
small case, the largest size the array takes, and the error paths."""
import numpy as np
import pytest

import geoinputs
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def g():
    import paper_1708_02835_amd as pkg
    pkg.lib()
    return pkg


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def field(n, seed, theta):
    x, y = geoinputs.jittered_grid(n, seed)
    e = geoinputs.normal_vector(n, seed + 1)
    return x, y, e, theta


def same(a, b):
    """Bit-identical results (a failed factorisation's NaN log-det equals NaN)."""
    def eq(u, v):
        return u == v or (np.isnan(u) and np.isnan(v))
    return a["status"] == b["status"] and a["info"] == b["info"] and a["tile"] == b["tile"] and all(
        eq(a[k], b[k]) for k in ("loglik", "logdet", "quad"))


def test_noalloc_matches_loglik_eval_twice_in_a_row(g):
    with g.Context(0) as ctx:
        cases = [(3001, 0, (1.0, 0.1, 0.5), 11), (1000, 0, (1.2, 0.05, 1.3), 12)]
        for n, tile, theta, seed in cases:
            x, y, e, _ = field(n, seed, theta)
            xd, yd, ed = dev(x), dev(y), dev(e)
            zd = torch.empty_like(xd)
            g.synth_generate(ctx, xd, yd, ed, theta, out=zd)
            o = g.gl_opts_default(tile=tile)
            print(f"noalloc case n={n} tile={tile} theta={theta}", flush=True)
            a = g.loglik_eval_noalloc(ctx, xd, yd, zd, theta, o)
            b = g.loglik_eval(ctx, xd, yd, zd, theta, o)
            assert a["status"] == g.GL_OK and same(a, b), (n, a, b)
            if n <= 1000:
                ref = oracle.loglik(x, y, zd.cpu().numpy(), theta)
                assert abs(a["loglik"] - ref[0]) <= 1e-10 * abs(ref[0]), (a["loglik"], ref[0])


def test_noalloc_largest_size_and_after_eager_work(g):
    """n = 4,096 at tile 512 (the documented limit), a ragged n at tile 384, then
    a small call again: the array keeps the previous call's contents, and
    each call must clear what it needs."""
    with g.Context(0) as ctx:
        for n, tile, theta, seed in [(4096, 512, (1.0, 0.1, 0.5), 21), (3999, 384, (0.7, 0.08, 2.2), 22),
                                     (257, 128, (1.0, 0.1, 0.5), 23)]:
            x, y, e, _ = field(n, seed, theta)
            xd, yd, zd = dev(x), dev(y), dev(e)
            o = g.gl_opts_default(tile=tile)
            print(f"noalloc case n={n} tile={tile} theta={theta}", flush=True)
            b = g.loglik_eval(ctx, xd, yd, zd, theta, o)
            a = g.loglik_eval_noalloc(ctx, xd, yd, zd, theta, o)
            assert a["status"] == g.GL_OK and same(a, b), (n, a, b)


def test_noalloc_failure_and_limits(g):
    with g.Context(0) as ctx:
        # 60 locations repeated exactly: Σ has 60 zero eigenvalues whose pivots
        # come out as rounding noise of either sign, so the factorisation
        # fails; both entry points report the same column
        x, y, e, theta = field(700, 31, (1.0, 0.1, 0.5))
        x[300:360], y[300:360] = x[0:60], y[0:60]
        xd, yd, zd = dev(x), dev(y), dev(e)
        a = g.loglik_eval_noalloc(ctx, xd, yd, zd, theta)
        b = g.loglik_eval(ctx, xd, yd, zd, theta)
        assert same(a, b), (a, b)
        assert a["status"] == g.GL_NOT_SPD and a["info"] > 300 and a["loglik"] == -np.inf
        # a workspace beyond the array: GL_E2BIG, nothing launched
        x, y, e, theta = field(6000, 32, (1.0, 0.1, 0.5))
        t, v, _ = g.gl_workspace_layout(6000, 0, g.GL_FP64)
        assert ((t + 255) // 256) * 256 + v > g.GL_SCRATCH_BYTES
        with pytest.raises(g.GeolikError) as ei:
            g.loglik_eval_noalloc(ctx, dev(x), dev(y), dev(e), theta)
        assert ei.value.status == g.GL_E2BIG
        # options that need allocation are rejected
        x, y, e, theta = field(300, 33, (1.0, 0.1, 0.5))
        for bad in (dict(keep_factor=1), dict(precision=g.GL_MIXED_BF16), dict(ind_tiles=1), dict(graph=1)):
            with pytest.raises(g.GeolikError) as ei:
                g.loglik_eval_noalloc(ctx, dev(x), dev(y), dev(e), theta, g.gl_opts_default(**bad))
            assert ei.value.status == g.GL_EINVAL
        # still usable afterwards
        a = g.loglik_eval_noalloc(ctx, dev(x), dev(y), dev(e), theta)
        b = g.loglik_eval(ctx, dev(x), dev(y), dev(e), theta)
        assert same(a, b)
