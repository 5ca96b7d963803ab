"""Replayed hipGraph evaluations (gl_opts.graph = 1) against direct launches:
every replay is compared bit for bit with an eager evaluation of the same
inputs, with eager work and synchronisations between replays, across θ
changes (ν on different Bessel paths), new measurements, a size change, a
distance change and a workspace reallocation."""
import numpy as np
import pytest

import geoinputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def g():
    import paper_1708_02835_amd as pkg
    pkg.lib()
    return pkg


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def same(a, b):
    """Bit-identical results (NaN, the log-det and quad of a failed
    factorisation, equals NaN)."""
    def eq(u, v):
        return u == v or (np.isnan(u) and np.isnan(v))
    return a["status"] == b["status"] and a["info"] == b["info"] and all(
        eq(a[k], b[k]) for k in ("loglik", "logdet", "quad"))


def test_graph_replays_match_eager(g):
    ctx = g.Context(0)
    try:
        thetas = [(1.0, 0.1, 0.5), (1.3, 0.07, 1.5), (0.8, 0.12, 1.0), (1.1, 0.05, 2.5), (1.0, 0.1, 0.5)]
        for n, tile in [(1500, 128), (1300, 256), (1500, 128)]:
            x, y = geoinputs.jittered_grid(n, 40 + n)
            for rep, th in enumerate(thetas):
                z = geoinputs.normal_vector(n, 100 * rep + n)
                xd, yd, zd = dev(x), dev(y), dev(z)
                r_graph = g.loglik_eval(ctx, xd, yd, zd, th, g.gl_opts_default(tile=tile, graph=1))
                torch.cuda.synchronize()
                # eager work in between: another size, a covariance block
                g.matern_generate(ctx, xd[:50], yd[:50], xd[:70], yd[:70], th)
                r_eager = g.loglik_eval(ctx, xd, yd, zd, th, g.gl_opts_default(tile=tile))
                assert same(r_graph, r_eager), (n, tile, th, r_graph, r_eager)
        # distance change and workspace growth force a new capture
        x, y = geoinputs.jittered_grid(900, 7)
        x, y = -100.0 + 15.0 * x, 30.0 + 15.0 * y
        z = geoinputs.normal_vector(900, 7)
        o = dict(tile=128, metric=g.GL_GREAT_CIRCLE, radius=6371.0)
        a = g.loglik_eval(ctx, dev(x), dev(y), dev(z), (1.0, 150.0, 0.5), g.gl_opts_default(graph=1, **o))
        b = g.loglik_eval(ctx, dev(x), dev(y), dev(z), (1.0, 150.0, 0.5), g.gl_opts_default(**o))
        assert same(a, b)
        xb, yb = geoinputs.jittered_grid(3000, 8)
        zb = geoinputs.normal_vector(3000, 8)
        g.loglik_eval(ctx, dev(xb), dev(yb), dev(zb), (1.0, 0.1, 0.5))  # grows the workspace
        a = g.loglik_eval(ctx, dev(x), dev(y), dev(z), (1.0, 150.0, 0.5), g.gl_opts_default(graph=1, **o))
        assert same(a, b)
    finally:
        ctx.close()


def test_graph_not_spd_and_recovery(g):
    ctx = g.Context(0)
    try:
        x, y = geoinputs.jittered_grid(800, 9)
        x[500], y[500] = x[499], y[499]
        z = geoinputs.normal_vector(800, 9)
        bad = g.loglik_eval(ctx, dev(x), dev(y), dev(z), (1.0, 0.1, 0.5), g.gl_opts_default(tile=128, graph=1))
        ref = g.loglik_eval(ctx, dev(x), dev(y), dev(z), (1.0, 0.1, 0.5), g.gl_opts_default(tile=128))
        assert same(bad, ref) and bad["info"] == ref["info"]
        x2, y2 = geoinputs.jittered_grid(800, 10)
        ok = g.loglik_eval(ctx, dev(x2), dev(y2), dev(z), (1.0, 0.1, 0.5), g.gl_opts_default(tile=128, graph=1))
        ref = g.loglik_eval(ctx, dev(x2), dev(y2), dev(z), (1.0, 0.1, 0.5), g.gl_opts_default(tile=128))
        assert ok["status"] == g.GL_OK and same(ok, ref)
    finally:
        ctx.close()


def test_graph_recaptures_after_vector_reallocation(g):
    """Automatic tiles: n = 3001 takes tile 256, n = 3000 tile 128.  The eager
    evaluation at n = 3000 needs a larger vector allocation (the 64·b inverse
    blocks per diagonal tile grow with the tile count) but not larger tiles,
    so only the vectors move.  The graph captured at n = 3001 holds pointers
    into the old vectors; the third call must capture again instead of
    replaying into freed memory."""
    ctx = g.Context(0)
    try:
        th = (1.0, 0.1, 0.5)
        sizes = [(3001, 1), (3000, 0), (3001, 1)]
        t1, v1, _ = g.gl_workspace_layout(3001)
        t0, v0, _ = g.gl_workspace_layout(3000)
        assert t0 <= t1 and v0 > v1, (t0, t1, v0, v1)  # the sequence this test is for
        for n, graph in sizes:
            x, y = geoinputs.jittered_grid(n, 60 + n)
            z = geoinputs.normal_vector(n, 61 + n)
            xd, yd, zd = dev(x), dev(y), dev(z)
            r_graph = g.loglik_eval(ctx, xd, yd, zd, th, g.gl_opts_default(graph=graph))
            if n == 3000:
                continue  # the eager call that reallocates the vectors
            fresh = g.Context(0)
            try:
                r_eager = g.loglik_eval(fresh, xd, yd, zd, th, g.gl_opts_default())
            finally:
                fresh.close()
            assert same(r_graph, r_eager), (n, r_graph, r_eager)
    finally:
        ctx.close()
