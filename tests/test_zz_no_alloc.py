"""mm_sweep_noalloc (the sweep that allocates nothing, for callers that cannot
allocate device memory) against mm_sweep, through the C-ABI.

Two calls in a row on one context, the second on a smaller graph, at the
finest level and at a coarse level (node weights): the output and the
relative-change sums equal mm_sweep's bit for bit (same kernel, same launch),
and both are within 1e-4 * max(|x_orc|, 1) of the oracle's FP64 update on the
same FP32 inputs.  Sets above the scratch limit are rejected before any
launch.
"""
import math

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


def _case(orc, mm, ctx, g, k, level, seed):
    rng = np.random.default_rng(seed)
    x = (rng.random((g.n, 2)) * math.sqrt(g.n)).astype(np.float32)
    c = rng.integers(1, 9, g.n).astype(np.int32) if level > 0 else None
    kh = mm.khop_build(ctx, ctx.graph(g.row_ptr, g.col), k)
    F = mm.repulsion(ctx, x, 0.0, 0.5)["F"]
    xa, da = mm.sweep_noalloc(ctx, kh, x, F, 0.37, 0.0, level, c, 1.0)
    xb, db = mm.sweep(ctx, kh, x, F, 0.37, 0.0, level, c, 1.0, mode=mm.SWEEP_ROWS)
    kh.free()
    xa = xa.cpu().numpy()
    xb = xb.cpu().numpy()
    ref = orc.khop_build(g.row_ptr, g.col, k)
    xr, dr = orc.sweep(ref, x.astype(np.float64), F.cpu().numpy().astype(np.float64), 0.37, 0.0,
                       level, c, 1.0)
    err = (np.abs(xa - xr) / np.maximum(np.abs(xr), 1.0)).max()
    print(f"  n={g.n} k={k} level={level}: max err vs oracle {err:.2e}, "
          f"bit-equal to mm_sweep {np.array_equal(xa, xb)}", flush=True)
    assert np.array_equal(xa, xb)
    assert da == db
    assert err < 1e-4
    assert abs(math.sqrt(da[0] / da[1]) - dr) <= 1e-3 * dr + 1e-7


@pytest.mark.parametrize("level", [0, 1])
def test_noalloc_sweep_two_calls(orc, mm, ctx, level):
    print(f"[noalloc] level={level}: RGG 12000 then RGG 3000", flush=True)
    _case(orc, mm, ctx, synth.rgg(12000, 4), 3, level, 11)
    _case(orc, mm, ctx, synth.rgg(3000, 5), 3, level, 12)


def test_noalloc_sweep_rejects_oversize(mm, ctx):
    n = mm.SWEEP_NOALLOC_MAX_N + 3
    print(f"[noalloc] path of {n} vertices (over the limit)", flush=True)
    v = np.arange(n - 1)
    g = synth.csr_from_edges(n, v, v + 1)
    kh = mm.khop_build(ctx, ctx.graph(g.row_ptr, g.col), 1)
    x = np.zeros((n, 2), np.float32)
    x[:, 0] = np.arange(n)
    F = np.zeros((n, 2), np.float32)
    with pytest.raises(mm.MulmentError) as ei:
        mm.sweep_noalloc(ctx, kh, x, F, 0.1)
    kh.free()
    assert ei.value.status == 1 and "scratch limit" in str(ei.value)
