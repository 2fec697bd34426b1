"""Coincident pairs inside the stress sets: one Jacobi iteration of Eq. 2 on
the GPU against the FP64 oracle, through the C-ABI.

A pair at distance 0 contributes w x_v to the stress sum and nothing to the
r-values (the oracle's D == 0 branch).  The kernels encode it three ways: a
tiny bias on D^2 at the finest level (q = 0), a tiny bias on g^2 D^2 on coarse
levels (q = 0), a D^2 > 0 select for q != 0; the row kernel tests D^2 > 0.
Each is run here on layouts where a quarter of the vertices sit exactly on a
neighbour (chains of coincident vertices included), at the finest and a coarse
level, q = 0 and 1, in the row kernel, the default tiled (sliced) kernel and
forced sliced and consecutive tiled configurations.  Bar: 1e-4 * max(|x_orc|,
1) per coordinate, as every sweep; the relative change within 1e-3.
"""
import math

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

KERNELS = [("rows", 1, None), ("tiled", 2, None), ("sliced-13x2", None, (13, 64, 2)),
           ("tile12-8x4", None, (12, 8, 4))]


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


def coincident_layout(g, seed, frac=0.25):
    """Random points, then a fraction of the vertices (in a random order)
    moved exactly onto a random neighbour's current position."""
    rng = np.random.default_rng(seed)
    x = (rng.random((g.n, 2)) * math.sqrt(g.n)).astype(np.float32)
    for u in rng.permutation(g.n)[: int(frac * g.n)]:
        nb = g.col[g.row_ptr[u]:g.row_ptr[u + 1]]
        x[u] = x[nb[rng.integers(0, nb.size)]]
    return x


def _graphs():
    return {"rgg4k": (lambda: synth.rgg(4000, 3), 3),
            "rmat12": (lambda: synth.rmat(12, 8 * 4096, 5), 2)}


@pytest.fixture(scope="module")
def cases(orc, mm, ctx):
    out = {}
    for name, (mk, k) in _graphs().items():
        g = mk()
        x = coincident_layout(g, 41)
        ref = orc.khop_build(g.row_ptr, g.col, k)
        # pairs of the stress sets at distance 0 (both directions)
        rows = np.repeat(np.arange(g.n), np.diff(ref.off))
        same = np.all(x[rows] == x[ref.nbr], axis=1)
        kh = mm.khop_build(ctx, ctx.graph(g.row_ptr, g.col), k)
        out[name] = (g, k, x, ref, kh, int(same.sum()))
    yield out
    for v in out.values():
        v[4].free()


@pytest.mark.parametrize("kernel", KERNELS, ids=[k[0] for k in KERNELS])
@pytest.mark.parametrize("q", [0.0, 1.0])
@pytest.mark.parametrize("level", [0, 1])
@pytest.mark.parametrize("name", ["rgg4k", "rmat12"])
def test_sweep_with_coincident_pairs(mm, ctx, orc, cases, name, level, q, kernel):
    g, k, x, ref, kh, n_same = cases[name]
    label, mode, config = kernel
    print(f"[coincident] {name} k={k} level={level} q={q} kernel={label} "
          f"(stress-set entries at distance 0: {n_same})", flush=True)
    assert n_same > 0
    rng = np.random.default_rng(5)
    c = rng.integers(1, 9, g.n).astype(np.int32) if level > 0 else None
    F = mm.repulsion(ctx, x, q, 0.5)["F"]
    Fh = F.cpu().numpy()
    assert np.isfinite(Fh).all()
    alpha = 0.37
    if config is None:
        xo, d = mm.sweep(ctx, kh, x, F, alpha, q, level, c, 1.0, mode=mode)
    else:
        xo, d = mm.sweep(ctx, kh, x, F, alpha, q, level, c, 1.0, config=config)
    xr, dr = orc.sweep(ref, x.astype(np.float64), Fh.astype(np.float64), alpha, q, level, c, 1.0)
    xo = xo.cpu().numpy()
    assert np.isfinite(xo).all()
    err = np.abs(xo - xr) / np.maximum(np.abs(xr), 1.0)
    print(f"  max err {err.max():.3e}", flush=True)
    assert err.max() < 1e-4
    assert abs(math.sqrt(d[0] / d[1]) - dr) <= 1e-3 * dr + 1e-7
