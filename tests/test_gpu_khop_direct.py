"""Tile-major stress sets built straight from the 2-hop search (the rows
whose search used a bitmap are read from their CSR row and kept hop-2
bitmap; mm_params.khop_direct = 1, the default) against the same sets built
from the canonical ids (khop_direct = 0), through the C-ABI.

The direct build must give the same tile-major layout (entries, chunk order)
and the same rho_u bit for bit, so whole layouts must agree bit for bit:
* with the default rules (tiles of 2^13 on the finest level, 2^12 or 2^11
  on coarse ones, tiled where the mean chunk has >= 8 entries);
* with every level forced through tuner records to one tiled configuration
  (tiles of 2^11 / 2^12 / 2^13; the sliced layout or 8 / 16 lanes per
  chunk; 2 or 4 blocks per lane and step).
The graphs are R-MAT graphs with hubs, so most rows of the finest level and
all rows of the dense coarse levels take the bitmap search, the others the
per-wave lists; coarse levels cover rho_u with node weights (sqrt c terms
summed in the canonical order).  The verbose log confirms that the direct
build ran.
"""
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


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


def _layout(mm, ctx, dg, capfd, **kw):
    os.environ["MM_VERBOSE"] = "1"
    try:
        x, st = mm.layout(ctx, dg, mm.Params(**kw))
        x = x.cpu().numpy()
    finally:
        os.environ.pop("MM_VERBOSE", None)
    err = capfd.readouterr().err
    return x, st, err.count("(straight from the search)")


@pytest.mark.parametrize("scale", [14, 16])
def test_direct_default_rules(mm, ctx, capfd, scale):
    g = synth.rmat(scale, 8 * (1 << scale), 5)
    print(f"[khop direct] rmat{scale} n={g.n} default rules", flush=True)
    dg = ctx.graph(g.row_ptr, g.col)
    kw = dict(k=2, theta=0.5, seed=2, validate=0, max_final_iters=40)
    x1, s1, n1 = _layout(mm, ctx, dg, capfd, khop_direct=1, **kw)
    x0, s0, n0 = _layout(mm, ctx, dg, capfd, khop_direct=0, **kw)
    print(f"  levels {s1['levels']}, direct on {n1} levels", flush=True)
    assert n1 >= 2 and n0 == 0
    assert [l["tile_bits"] for l in s1["per_level"]] == [l["tile_bits"] for l in s0["per_level"]]
    assert [l["khop_entries"] for l in s1["per_level"]] == [l["khop_entries"] for l in s0["per_level"]]
    assert np.array_equal(x1, x0)


FORCED = [(11, 64, 4), (12, 64, 2), (13, 64, 4), (11, 8, 2), (12, 16, 4), (13, 8, 2)]


@pytest.mark.parametrize("cfg", FORCED, ids=lambda c: f"tile{c[0]}-{c[1]}x{c[2]}")
def test_direct_forced_configuration(mm, ctx, capfd, cfg):
    g = synth.rmat(14, 8 * (1 << 14), 7)
    print(f"[khop direct] rmat14 n={g.n} forced {cfg}", flush=True)
    dg = ctx.graph(g.row_ptr, g.col)
    kw = dict(k=2, theta=0.5, seed=3, validate=0, max_final_iters=30)
    _, s, _ = _layout(mm, ctx, dg, capfd, **kw)
    recs = np.array([[1 if l["level"] > 0 else 0, l["n"], l["khop_entries"], 2, *cfg]
                     for l in s["per_level"]], np.int64)
    ctx.tune_import(recs)
    try:
        x1, s1, n1 = _layout(mm, ctx, dg, capfd, khop_direct=1, autotune=1, **kw)
        x0, s0, n0 = _layout(mm, ctx, dg, capfd, khop_direct=0, autotune=1, **kw)
    finally:
        ctx.tune_clear()
    print(f"  levels {s1['levels']}, direct on {n1} levels", flush=True)
    assert s1["t_tune_ms"] == 0 and s0["t_tune_ms"] == 0
    assert n1 >= 2 and n0 == 0
    assert all(l["tile_bits"] == cfg[0] for l in s1["per_level"])
    assert np.array_equal(x1, x0)
