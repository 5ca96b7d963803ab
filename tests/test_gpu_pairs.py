"""Two panels per trailing pass (gl_opts.near_tiles).

The far columns of a step pair receive panels k and k+1 in one pass (K = 2b).
At the default setting this starts once the tile count exceeds b tiles
(from about n = 6,000 at tile 256), so these tests force it at small n with a
small near_tiles and check:

* binary64: the result against the oracle at the FP64 bound, and against the
  one-panel schedule (near_tiles beyond the tile count) to a few ulps of
  rounding, at tiles 128, 256 and 512 with a ragged last tile; the trailing
  flops recorded by the phase timing equal the one-panel schedule's (every
  tile still receives every panel exactly once); a replayed graph equals the
  direct evaluation bit for bit;
* the split-product classes of the mixed modes (every off-band tile in the
  FP32-grade class of the mode): both schedules within the forced-class
  bound of the oracle, so a panel skipped or applied twice, or a stale panel
  copy, fails.
"""
import math

import numpy as np
import pytest

import geoinputs
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

NO_PAIRS = 1 << 30


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


def rel(a, b):
    return abs(a - b) / abs(b)


_fields = {}


def field(n, seed, theta):
    key = (n, seed, theta)
    if key not in _fields:
        x, y = geoinputs.jittered_grid(n, seed)
        e = geoinputs.normal_vector(n, seed)
        z, info = oracle.synth(x, y, e, theta)
        assert info == 0
        _fields[key] = (x, y, z, oracle.loglik(x, y, z, theta))
    return _fields[key]


@pytest.mark.parametrize("n,tile,near", [(2300, 128, 1), (2300, 128, 40), (2900, 256, 1), (2900, 512, 1)])
def test_fp64_pairs_match_oracle_and_one_panel_schedule(g, ctx, n, tile, near):
    theta = (1.0, 0.1, 0.5)
    x, y, z, ref = field(n, 41, theta)
    xd, yd, zd = dev(x), dev(y), dev(z)
    print(f"pairs n={n} tile={tile} near={near}", flush=True)
    a = g.loglik_eval(ctx, xd, yd, zd, theta, g.gl_opts_default(tile=tile, near_tiles=near))
    b = g.loglik_eval(ctx, xd, yd, zd, theta, g.gl_opts_default(tile=tile, near_tiles=NO_PAIRS))
    assert a["status"] == g.GL_OK and b["status"] == g.GL_OK
    assert rel(a["loglik"], ref[0]) <= 1e-10 and rel(a["logdet"], ref[1]) <= 1e-10
    assert rel(a["loglik"], b["loglik"]) <= 1e-12 and rel(a["quad"], b["quad"]) <= 1e-12


def test_fp64_pairs_profile_flops_and_graph(g, ctx):
    n, tile, theta = 2300, 128, (1.0, 0.1, 0.5)
    x, y, z, _ = field(n, 41, theta)
    xd, yd, zd = dev(x), dev(y), dev(z)
    nt = -(-n // tile)
    g.gl_profile_enable(ctx, 1)
    try:
        g.loglik_eval(ctx, xd, yd, zd, theta, g.gl_opts_default(tile=tile, near_tiles=1))
        ph = g.gl_profile_phases(ctx)
    finally:
        g.gl_profile_enable(ctx, 0)
    b3 = float(tile) ** 3
    flops = sum(2 * b3 * (nt - j - 1) + tile * tile * (tile + 1) for k in range(nt - 1) for j in range(k + 1, nt))
    assert ph["trail_crit"]["flops"] + ph["trail_bulk"]["flops"] + ph["trail_pair"]["flops"] == pytest.approx(
        flops, rel=1e-12)
    assert ph["trail_pair"]["launches"] > 0
    o = dict(tile=tile, near_tiles=1)
    eager = g.loglik_eval(ctx, xd, yd, zd, theta, g.gl_opts_default(**o))
    for _ in range(2):
        rep = g.loglik_eval(ctx, xd, yd, zd, theta, g.gl_opts_default(graph=1, **o))
        assert (rep["loglik"], rep["logdet"], rep["quad"]) == (eager["loglik"], eager["logdet"], eager["quad"])


# (precision, tol_hi, tol_lo): every off-band tile in the FP32-grade split class
SPLIT = [(2, 0.0, 0.0), (3, -1.0, 0.0)]


@pytest.mark.parametrize("prec,thi,tlo", SPLIT)
@pytest.mark.parametrize("n,tile", [(2048, 256), (1700, 128)])
def test_mixed_pairs_against_per_step(g, ctx, prec, thi, tlo, n, tile):
    theta = (1.0, 0.1, 0.5)
    x, y, z, ref = field(n, 42, theta)
    xd, yd, zd = dev(x), dev(y), dev(z)
    out = {}
    for near in (2, NO_PAIRS):
        o = g.gl_opts_default(precision=prec, tile=tile, band=1, tol_64=math.inf, tol_hi=thi, tol_lo=tlo,
                              near_tiles=near)
        r = g.loglik_eval(ctx, xd, yd, zd, theta, o)
        assert r["status"] == g.GL_OK
        out[near] = r
        assert rel(r["loglik"], ref[0]) <= 1e-6, (prec, n, tile, near, rel(r["loglik"], ref[0]))
        assert rel(r["logdet"], ref[1]) <= 1e-5
    assert rel(out[2]["loglik"], out[NO_PAIRS]["loglik"]) <= 2e-6
