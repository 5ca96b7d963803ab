"""CPU checks of the C-ABI library: it loads, exports every function declared
in include/geolik.h, and its host-only entry points behave as documented.
No compute call is made here (there is no GPU in this environment)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "geolik.h")


def _ensure_built():
    from paper_1708_02835_amd import build as b
    if not os.path.exists(b.LIB):
        b.build()
    return b.LIB


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_entry_points():
    names = _declared_functions()
    for must in ["matern_generate", "loglik_eval", "krige_predict", "synth_generate", "lq_submit",
                 "lq_poll", "lq_wait", "lq_create", "lq_destroy", "gl_context_create"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_ensure_built())
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert missing == []


def test_binding_names_match_header():
    import paper_1708_02835_amd as g
    missing = [n for n in _declared_functions() if not hasattr(g, n)]
    assert missing == []


def test_status_strings_and_defaults():
    _ensure_built()
    import paper_1708_02835_amd as g
    assert g.gl_status_string(g.GL_OK) == "ok"
    assert "positive definite" in g.gl_status_string(g.GL_NOT_SPD)
    for st in [g.GL_EINVAL, g.GL_ENOMEM, g.GL_EHIP, g.GL_EBUSY, g.GL_ECANCELED, g.GL_ETIMEDOUT, g.GL_ENODEV,
               g.GL_EVICTED, g.GL_E2BIG]:
        assert g.gl_status_string(st) != "unknown status"
    o = g.gl_opts_default()
    assert (o.precision, o.tile, o.keep_factor, o.band, o.reorder) == (g.GL_FP64, 0, 0, 2, -1)
    assert o.tol_hi < 0 and o.tol_lo < 0 and o.tol_64 < 0
    assert o.metric == g.GL_EUCLIDEAN and o.radius == 6371.0
    c = g.lq_config_default()
    assert c.max_inflight >= 1 and 1 <= c.streams <= 8


def test_opts_layout_matches_header():
    """The ctypes struct mirrors gl_opts field by field (names and order)."""
    import re
    import paper_1708_02835_amd as g
    hdr = open(os.path.join(ROOT, "include", "geolik.h")).read()
    body = hdr[hdr.index("typedef struct {", hdr.index("GL_GREAT_CIRCLE")):hdr.index("} gl_opts;")]
    names = re.findall(r"^\s*(?:int32_t|double)\s+(\w+);", body, re.M)
    assert names == [f for f, _ in g.gl_opts._fields_]


@pytest.mark.parametrize("n,tile", [(1, 128), (1600, 128), (40000, 512), (100000, 512), (100001, 256)])
def test_footprint_formula(n, tile):
    _ensure_built()
    import paper_1708_02835_amd as g
    nt = -(-n // tile)
    tiles = nt * (nt + 1) // 2 * tile * tile * 8
    p2 = 1
    while p2 < n:
        p2 *= 2
    vec = (3 * nt * tile + 2 * nt + nt * (nt + 1) // 2 + 64 * nt * tile + 16 + p2 + 4) * 8
    assert g.gl_footprint_bytes(n, tile, g.GL_FP64) == tiles + vec
    # mixed modes add the FP32 running sums (one b×b block per tile), the
    # double-buffered panel copies, the tile lists and the map
    tc = nt * (nt + 1) // 2
    extra32 = tc * tile * tile * 4 + 2 * nt * tile * tile * 4 + tc * 8 + ((tc + 255) // 256) * 256 + 1024
    extra16 = tc * tile * tile * 4 + 2 * 3 * nt * tile * tile * 2 + tc * 8 + ((tc + 255) // 256) * 256 + 1024
    assert g.gl_footprint_bytes(n, tile, g.GL_MIXED_FP32) == tiles + vec + extra32
    assert g.gl_footprint_bytes(n, tile, g.GL_MIXED_BF16) == tiles + vec + extra16
    extrah = tc * tile * tile * 4 + 2 * 2 * nt * tile * tile * 2 + tc * 8 + ((tc + 255) // 256) * 256 + 1024
    assert g.gl_footprint_bytes(n, tile, g.GL_MIXED_FP16) == tiles + vec + extrah


def test_automatic_tile_choice_footprints_are_monotone():
    _ensure_built()
    import paper_1708_02835_amd as g
    sizes = [g.gl_footprint_bytes(n) for n in [1000, 4000, 16000, 40000, 100000]]
    assert sizes == sorted(sizes)


def test_context_create_without_gpu_reports_enodev():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    _ensure_built()
    import paper_1708_02835_amd as g
    with pytest.raises(g.GeolikError) as ei:
        g.Context()
    assert ei.value.status == g.GL_ENODEV


def test_binding_rejects_unknown_option_names():
    _ensure_built()
    import paper_1708_02835_amd as g
    with pytest.raises(TypeError):
        g.gl_opts_default(tol64=0.5)
    with pytest.raises(TypeError):
        g.lq_config_default(max_in_flight=3)
    o = g.gl_opts_default(tol_64=0.5, ind_tiles=2)
    assert o.tol_64 == 0.5 and o.ind_tiles == 2


def test_workspace_layout_sequence_moves_only_the_vectors():
    """The size sequence behind graph re-capture: with automatic tiles n = 3001
    takes tile 256 and n = 3000 tile 128, so going 3001 -> 3000 grows the
    vector allocation (64·b inverse words per diagonal tile) but not the tile
    allocation.  A cached graph keyed on the tile allocation alone would replay
    into freed vectors; the three parts must add up to the footprint."""
    _ensure_built()
    import paper_1708_02835_amd as g
    t1, v1, m1 = g.gl_workspace_layout(3001)
    t0, v0, m0 = g.gl_workspace_layout(3000)
    assert t0 <= t1 and v0 > v1 and m0 == m1 == 0
    for n in (3000, 3001, 40000):
        for prec in (g.GL_FP64, g.GL_MIXED_BF16):
            assert sum(g.gl_workspace_layout(n, 0, prec)) == g.gl_footprint_bytes(n, 0, prec)
    with pytest.raises(g.GeolikError):
        g.gl_workspace_layout(0)
    with pytest.raises(g.GeolikError):
        g.gl_workspace_layout(100, 100)


def test_scratch_limit_matches_header():
    """The binding's copy of the no-allocation workspace limit is the header's,
    and the documented n <= 4,096 fits it at every tile size."""
    import paper_1708_02835_amd as g
    text = open(HEADER).read()
    m = re.search(r"#define GL_SCRATCH_BYTES \(\(size_t\)(\d+) << (\d+)\)", text)
    assert m and int(m.group(1)) << int(m.group(2)) == g.GL_SCRATCH_BYTES
    for tile in (0, 128, 256, 384, 512):
        t, v, _ = g.gl_workspace_layout(4096, tile, g.GL_FP64)
        assert ((t + 255) // 256) * 256 + v <= g.GL_SCRATCH_BYTES


def test_pick_tile_matches_documented_rule():
    import paper_1708_02835_amd as g
    assert [g.gl_pick_tile(n) for n in (1, 3000, 3001, 24000, 24001, 100000)] == [128, 128, 256, 256, 512, 512]
    assert g.gl_pick_tile(5000, 384) == 384
    for bad in ((0, 0), (100, 200)):
        with pytest.raises(g.GeolikError):
            g.gl_pick_tile(*bad)
