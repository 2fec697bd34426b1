"""Batched layout of many graphs (one union, per-graph hierarchy and
schedule) vs each graph laid out alone on the GPU and by the FP64 oracle.

Bars: per-graph hierarchy depth equal to the oracle's (integer, exact);
final maxent-stress M_S of every graph within 1% (the end-to-end objective
bar) of the same graph laid out alone on the GPU and of the oracle's layout;
warm-started batches likewise vs single warm starts.  Batch and single runs
share hierarchy and draws; they differ only in FP summation order (far-field
prefix sums over the union, per-graph reductions, row instead of tiled
sweep), which measured 2e-3 at most on these graphs after ~10^3 iterations.
"""
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


K = 3
PARAMS = dict(k=K, theta=0.5, alpha_decay=0.5, coarsest_n=20, seed=3)


def _M(mm, ctx, g, x):
    kh = mm.khop_build(ctx, ctx.graph(g.row_ptr, g.col), K)
    M = mm.objective(ctx, kh, x, 0.008)["M"]
    kh.free()
    return M


@pytest.fixture(scope="module")
def batch(mm, ctx):
    gs = synth.batch_graphs(20, 7, nmin=40, nmax=1500)
    rp, col, offs = synth.concat(gs)
    print(f"[batch] {len(gs)} graphs, n={offs[-1]}", flush=True)
    xy, lev, st = mm.layout_batch(ctx, rp, col, offs, mm.Params(**PARAMS))
    return gs, offs, xy, lev, st


def test_batch_hierarchy_matches_oracle(orc, batch):
    gs, offs, xy, lev, st = batch
    op = orc.Params(**PARAMS)
    for i, g in enumerate(gs):
        levels, _, _ = orc.hierarchy(orc.Level(g.row_ptr, g.col), op)
        assert lev[i] == len(levels), i


def test_batch_equals_single_layouts(mm, ctx, batch):
    gs, offs, xy, lev, st = batch
    worst = 0.0
    for i, g in enumerate(gs):
        xb = xy[int(offs[i]):int(offs[i + 1])]
        x1, st1 = mm.layout(ctx, ctx.graph(g.row_ptr, g.col), mm.Params(**PARAMS))
        assert st1["levels"] == lev[i]
        Mb, M1 = _M(mm, ctx, g, xb), _M(mm, ctx, g, x1)
        worst = max(worst, abs(Mb - M1) / abs(M1))
    print(f"  max rel. difference of M_S batch vs alone: {worst:.2e}")
    assert worst <= 0.01


def test_batch_matches_oracle(orc, mm, ctx, batch):
    gs, offs, xy, lev, st = batch
    op = orc.Params(**PARAMS)
    errs = []
    for i, g in enumerate(gs):
        xb = xy[int(offs[i]):int(offs[i + 1])]
        xo, _ = orc.layout(g, op)
        kh = orc.khop_build(g.row_ptr, g.col, K)
        Mo = orc.objective(kh, xo, 0.008)["M"]
        errs.append(abs(_M(mm, ctx, g, xb) - Mo) / abs(Mo))
    print(f"  M_S vs oracle: max {max(errs):.2e} mean {np.mean(errs):.2e}")
    assert max(errs) <= 0.01


def test_batch_warm_start(mm, ctx, batch):
    gs, offs, xy, lev, st = batch
    rp, col, _ = synth.concat(gs)
    init = xy.detach().clone()
    init[:, 0] += 0.25  # a shifted start
    xw, lev2, st2 = mm.layout_batch(ctx, rp, col, offs, mm.Params(**PARAMS), init_xy=init)
    assert st2["levels"] == 1
    for i in (0, 5, 11, 19):
        g = gs[i]
        x1, _ = mm.layout(ctx, ctx.graph(g.row_ptr, g.col), mm.Params(**PARAMS),
                          init_xy=init[int(offs[i]):int(offs[i + 1])])
        Mb = _M(mm, ctx, g, xw[int(offs[i]):int(offs[i + 1])])
        M1 = _M(mm, ctx, g, x1)
        assert abs(Mb - M1) <= 0.01 * abs(M1)


def test_batch_rejects_cross_edges(mm, ctx):
    gs = [synth.grid(4, 4), synth.grid(3, 5)]
    rp, col, offs = synth.concat(gs)
    col = col.copy()
    col[0] = int(offs[1])  # vertex 0's first edge points into graph 1
    with pytest.raises(mm.MulmentError):
        mm.layout_batch(ctx, rp, col, offs, mm.Params(**{**PARAMS, "validate": 0}))
    with pytest.raises(mm.MulmentError):
        mm.layout_batch(ctx, rp, synth.concat(gs)[1], np.array([0, 1, offs[-1]]),
                        mm.Params(**PARAMS))
