"""Every sweep configuration the autotuner may pick, and the tuner's choices
kept across contexts, through the C-ABI.

Bars:
* each configuration (row kernel with 8/16/32/64 lanes per row, tiled kernel
  with tiles of 2^11/2^12/2^13 vertices, 1/2/4/8/16 lanes per chunk or the
  sliced layout (lanes code 64), and 2/4
  blocks per lane and step) gives one
  Jacobi iteration of Eq. 2 within 1e-4 relative (floor 1) of the FP64 oracle
  on the same FP32 inputs, finest and coarse level, with a ragged last tile;
* an autotuned layout is reproducible in its context, and a second context
  that imports the exported choices tunes nothing and gives the same bits;
* malformed tuner records and configurations are rejected.
"""
import math

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

CONFIGS = [(0, 8, 0), (0, 16, 0), (0, 32, 0), (0, 64, 0)] + \
    [(tb, g, nb) for tb in (11, 12, 13) for g in (1, 2, 4, 8, 16, 64) for nb in (2, 4)]


@pytest.fixture(scope="module")
def mm():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1506_04383_amd as m

    return m


@pytest.fixture(scope="module")
def ctx(mm):
    c = mm.Context(0)
    yield c
    c.close()


def _cfg_id(c):
    return f"rows-{c[1]}" if c[0] == 0 else f"tile{c[0]}-{c[1]}x{c[2]}"


@pytest.fixture(scope="module")
def case(orc, mm, ctx):
    """RGG with 12345 vertices (ragged last tile at every tile size), k = 2."""
    g = synth.rgg(12345, 4, 10.0)
    rng = np.random.default_rng(3)
    x = (rng.random((g.n, 2)) * math.sqrt(g.n)).astype(np.float32)
    c = rng.integers(1, 9, g.n).astype(np.int32)
    kh = mm.khop_build(ctx, ctx.graph(g.row_ptr, g.col), 2)
    F = mm.repulsion(ctx, x, 0.0, 0.5)["F"]
    ref = orc.khop_build(g.row_ptr, g.col, 2)
    out = {}
    for level, cw in ((0, None), (1, c)):
        xr, dr = orc.sweep(ref, x.astype(np.float64), F.cpu().numpy().astype(np.float64), 0.37,
                           0.0, level, cw, 1.0)
        out[level] = (xr, dr)
    yield g, x, c, kh, F, out
    kh.free()


@pytest.mark.parametrize("level", [0, 1])
@pytest.mark.parametrize("config", CONFIGS, ids=_cfg_id)
def test_every_sweep_configuration_matches_oracle(mm, ctx, case, config, level):
    g, x, c, kh, F, ref = case
    print(f"[sweep cfg] {_cfg_id(config)} level={level} n={g.n}", flush=True)
    xo, d = mm.sweep(ctx, kh, x, F, 0.37, 0.0, level, c if level else None, 1.0, config=config)
    xr, dr = ref[level]
    err = np.abs(xo.cpu().numpy() - xr) / np.maximum(np.abs(xr), 1.0)
    print(f"  max err {err.max():.3e}", flush=True)
    assert err.max() < 1e-4
    assert abs(math.sqrt(d[0] / d[1]) - dr) <= 1e-3 * dr + 1e-7


def test_bad_configuration_rejected(mm, ctx, case):
    g, x, c, kh, F, _ = case
    for cfg in [(0, 4, 0), (0, 128, 0), (10, 8, 2), (13, 32, 2), (14, 8, 2), (12, 6, 2),
                (0, 8, 2), (12, 8, 3), (12, 8, 8)]:
        with pytest.raises(mm.MulmentError, match="EINVAL"):
            mm.sweep(ctx, kh, x, F, 0.37, config=cfg)


def test_tuned_layout_export_import(mm, ctx):
    g = synth.rmat(14, 8 * (1 << 14), 5)
    kw = dict(k=2, theta=0.5, alpha_decay=0.3, seed=2, validate=0, autotune=1)
    c1 = mm.Context(0)
    try:
        dg = c1.graph(g.row_ptr, g.col)
        x1, s1 = mm.layout(c1, dg, mm.Params(**kw))
        recs = c1.tune_export()
        assert 1 <= recs.shape[0] <= s1["levels"] and s1["t_tune_ms"] > 0
        x1b, s1b = mm.layout(c1, dg, mm.Params(**kw))
        assert s1b["t_tune_ms"] == 0
        assert np.array_equal(x1.cpu().numpy(), x1b.cpu().numpy())
    finally:
        c1.close()
    c2 = mm.Context(0)
    try:
        c2.tune_import(recs)
        assert np.array_equal(np.sort(c2.tune_export(), axis=0), np.sort(recs, axis=0))
        x2, s2 = mm.layout(c2, c2.graph(g.row_ptr, g.col), mm.Params(**kw))
        assert s2["t_tune_ms"] == 0
        assert [l["tile_bits"] for l in s2["per_level"]] == [l["tile_bits"] for l in s1["per_level"]]
        assert [l["group"] for l in s2["per_level"]] == [l["group"] for l in s1["per_level"]]
        assert np.array_equal(x2.cpu().numpy(), x1.cpu().numpy())
        c2.tune_clear()
        assert c2.tune_export().shape[0] == 0
    finally:
        c2.close()


def test_bad_tune_records_rejected(mm, ctx):
    good = np.array([[0, 1000, 50000, 2, 13, 8, 4]], np.int64)
    ctx.tune_import(good)
    for col, val in [(4, 10), (4, 14), (5, 3), (5, 32), (0, 2), (1, -1), (3, 0), (6, 3), (6, 8)]:
        bad = good.copy()
        bad[0, col] = val
        with pytest.raises(mm.MulmentError, match="EINVAL"):
            ctx.tune_import(bad)
    ctx.tune_clear()
