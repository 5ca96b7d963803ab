"""Kernel timing by phase (gl_profile_enable / gl_profile_phases): launch
counts per phase follow the step schedule of the tiled factorisation, the
trailing flops follow 2b³ per off-diagonal and b²(b+1) per diagonal tile
update, timing leaves the result bit for bit unchanged, and the trailing-only
mode records nothing else; in the mixed modes the trailing updates are timed
per precision class and their flops add up to the binary64 total."""
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


@pytest.mark.parametrize("n,tile", [(1700, 256), (1000, 128)])
def test_phase_counts_flops_and_results(g, n, tile):
    x, y = geoinputs.jittered_grid(n, 90)
    z = geoinputs.normal_vector(n, 90)
    xd, yd, zd = dev(x), dev(y), dev(z)
    th = (1.0, 0.1, 0.5)
    nt = -(-n // tile)
    with g.Context(0) as ctx:
        plain = g.loglik_eval(ctx, xd, yd, zd, th, g.gl_opts_default(tile=tile))
        g.gl_profile_enable(ctx, 2)
        timed = g.loglik_eval(ctx, xd, yd, zd, th, g.gl_opts_default(tile=tile))
        ph = g.gl_profile_phases(ctx)
        g.gl_profile_enable(ctx, 1)
        g.loglik_eval(ctx, xd, yd, zd, th, g.gl_opts_default(tile=tile))
        trail_only = g.gl_profile_phases(ctx)
        g.gl_profile_enable(ctx, 0)
        g.loglik_eval(ctx, xd, yd, zd, th, g.gl_opts_default(tile=tile))
        off = g.gl_profile_phases(ctx)
    assert timed["loglik"] == plain["loglik"] and timed["logdet"] == plain["logdet"]
    want = {"gen": 1, "potrf": nt, "trsm": nt, "solve": 2 * nt, "trail_crit": nt - 1,
            "trail_bulk": max(nt - 2, 0), "reduce": 1, "trail_pair": 0}
    want.update({p: 0 for p in g.PHASES if p.startswith("mixed_")})
    assert {p: v["launches"] for p, v in ph.items()} == want
    assert all(v["ms"] > 0 for p, v in ph.items() if v["launches"])
    b3 = float(tile) ** 3
    flops = sum(2 * b3 * (nt - j - 1) + tile * tile * (tile + 1) for k in range(nt - 1) for j in range(k + 1, nt))
    assert ph["trail_crit"]["flops"] + ph["trail_bulk"]["flops"] == pytest.approx(flops, rel=1e-12)
    assert ph["trail_pair"]["launches"] == 0  # no two-panel passes at this size
    assert {p: v["launches"] for p, v in trail_only.items()} == dict(
        {p: 0 for p in want}, trail_crit=nt - 1, trail_bulk=max(nt - 2, 0))
    assert all(v["launches"] == 0 for v in off.values())


@pytest.mark.parametrize("precision", ["GL_MIXED_FP16", "GL_MIXED_BF16"])
def test_mixed_class_phases(g, precision):
    n, tile = 2300, 256
    x, y = geoinputs.jittered_grid(n, 91)
    z = geoinputs.normal_vector(n, 91)
    xd, yd, zd = dev(x), dev(y), dev(z)
    th = (1.0, 0.1, 0.5)
    nt = -(-n // tile)
    prec = getattr(g, precision)
    # near_tiles = 1 forces the two-panel passes of the split classes at this size
    o = g.gl_opts_default(tile=tile, precision=prec, near_tiles=1)
    with g.Context(0) as ctx:
        plain = g.loglik_eval(ctx, xd, yd, zd, th, o)
        stats = g.gl_precision_stats(ctx)
        g.gl_profile_enable(ctx, 1)
        timed = g.loglik_eval(ctx, xd, yd, zd, th, o)
        ph = g.gl_profile_phases(ctx)
        g.gl_profile_enable(ctx, 0)
    assert timed["loglik"] == plain["loglik"] and timed["logdet"] == plain["logdet"]
    mixed = {p: v for p, v in ph.items() if p.startswith("mixed_")}
    assert all(v["launches"] == 0 for p, v in ph.items() if not p.startswith("mixed_"))
    b3 = float(tile) ** 3
    flops = sum(2 * b3 * (nt - j - 1) + tile * tile * (tile + 1) for k in range(nt - 1) for j in range(k + 1, nt))
    assert sum(v["flops"] for v in mixed.values()) == pytest.approx(flops, rel=1e-12)
    for p, v in mixed.items():
        cls = p[len("mixed_"):]
        assert (v["launches"] > 0) == (stats[cls]["work_frac"] > 0), (p, v, stats[cls])
        if v["launches"]:
            assert v["ms"] > 0 and v["flops"] > 0
