"""General stress sets S ⊇ E (footnote to Eq. 1) on the GPU: sets imported
through mm_khop_import (distance-thresholded and randomly sampled, target
distances from brute-force hop distances) against the FP64 oracle on the
same arrays.  Bars as for the k-hop sets: one sweep within
1e-4 * max(|x_orc|, 1) for every kernel configuration, objectives within
1e-5 relative, exported arrays bit-identical to the imported ones."""
import functools
import math

import numpy as np
import pytest

import general_sets as gs
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


@functools.lru_cache(maxsize=None)
def _case(name):
    rng = np.random.default_rng(23)
    if name == "rgg4k_thresh":
        g = synth.rgg(4000, 3)
        x = (rng.random((g.n, 2)) * math.sqrt(g.n)).astype(np.float32)
        k = 3
        arrays = gs.thresholded(g, g.points * math.sqrt(g.n), k, 2.2)
    elif name == "rmat12_sampled":
        g = synth.rmat(12, 8 * 4096, 5)
        x = (rng.random((g.n, 2)) * math.sqrt(g.n)).astype(np.float32)
        k = 2
        arrays = gs.sampled(g, k, 0.3, seed=4)
    else:  # a layout-space threshold: pairs within 3 hops that lie close in x
        g = synth.grid(48, 40)
        x = (rng.random((g.n, 2)) * math.sqrt(g.n)).astype(np.float32)
        k = 3
        arrays = gs.thresholded(g, x, k, 8.0)
    return g, x, k, arrays


CASES = ["rgg4k_thresh", "rmat12_sampled", "grid_layout_thresh"]
CONFIGS = [None, (0, 32, 0), (11, 1, 2), (12, 8, 4), (13, 16, 2), (11, 64, 2), (13, 64, 4)]


def _cfg_id(c):
    return "auto" if c is None else "-".join(map(str, c))


@pytest.mark.parametrize("name", CASES)
def test_import_export_roundtrip(orc, mm, ctx, name):
    """Host and device imports keep the arrays bit for bit."""
    import torch

    g, x, k, (off, hend, nbr) = _case(name)
    print(f"[import] {name} n={g.n} k={k} |S|={nbr.size}", flush=True)
    ball = orc.khop_build(g.row_ptr, g.col, k)
    assert g.nnz < nbr.size < ball.nbr.size  # strictly between E and the k-hop ball
    for src in ("host", "device"):
        if src == "host":
            kh = mm.khop_import(ctx, g.n, k, off, hend, nbr)
        else:
            dv = [torch.from_numpy(a).cuda() for a in (off, hend, nbr)]
            kh = mm.khop_import(ctx, g.n, k, *dv)
        assert (kh.n, kh.k, kh.total) == (g.n, k, nbr.size)
        eo, eh, en = kh.export()
        assert np.array_equal(eo, off) and np.array_equal(eh, hend) and np.array_equal(en, nbr)
        kh.free()


@pytest.mark.parametrize("config", CONFIGS, ids=_cfg_id)
@pytest.mark.parametrize("level,q", [(0, 0.0), (1, 0.0), (0, 1.0)])
@pytest.mark.parametrize("name", CASES)
def test_sweep_on_imported_set(orc, mm, ctx, name, level, q, config):
    """One Jacobi iteration of Eq. 2 over an imported S, every kernel family."""
    g, x, k, (off, hend, nbr) = _case(name)
    print(f"[sweep S] {name} level={level} q={q} cfg={_cfg_id(config)}", flush=True)
    c = np.random.default_rng(5).integers(1, 9, g.n).astype(np.int32) if level else None
    kh = mm.khop_import(ctx, g.n, k, off, hend, nbr)
    F = mm.repulsion(ctx, x, q, 0.5)["F"]
    alpha = 0.37
    if config is None:
        xo, d = mm.sweep(ctx, kh, x, F, alpha, q, level, c, 1.0, mode=mm.SWEEP_TILED)
    else:
        xo, d = mm.sweep(ctx, kh, x, F, alpha, q, level, c, 1.0, config=config)
    xr, dr = orc.sweep(orc.KHop(k, off, hend, nbr), x.astype(np.float64),
                       F.cpu().numpy().astype(np.float64), alpha, q, level, c, 1.0)
    err = np.abs(xo.cpu().numpy() - xr) / np.maximum(np.abs(xr), 1.0)
    print(f"  max err {err.max():.3e}", flush=True)
    assert err.max() < 1e-4
    assert abs(math.sqrt(d[0] / d[1]) - dr) <= 1e-3 * dr + 1e-7
    kh.free()


@pytest.mark.parametrize("level,q", [(0, 0.0), (1, 0.0), (0, 1.0)])
@pytest.mark.parametrize("name", CASES)
def test_objective_on_imported_set(orc, mm, ctx, name, level, q):
    g, x, k, (off, hend, nbr) = _case(name)
    c = np.random.default_rng(6).integers(1, 5, g.n).astype(np.int32) if level else None
    kh = mm.khop_import(ctx, g.n, k, off, hend, nbr)
    o = mm.objective(ctx, kh, x, 0.008, q, level, c)
    r = orc.objective(orc.KHop(k, off, hend, nbr), x.astype(np.float64), 0.008, q, level, c)
    assert o["coincident"] == r["coincident"]
    for key in ("stress", "ent", "M"):
        assert abs(o[key] - r[key]) <= 1e-5 * abs(r[key]), key
    kh.free()


def test_import_rejects_asymmetric_device_set(mm, ctx):
    """Device arrays go through the same checks; nothing is created."""
    import torch

    off = torch.tensor([0, 2, 4, 6], dtype=torch.int64).cuda()
    hend = torch.tensor([2, 2, 2, 2, 1, 2], dtype=torch.int32).cuda()  # (0, 2) at 1, (2, 0) at 2
    nbr = torch.tensor([1, 2, 0, 2, 1, 0], dtype=torch.int32).cuda()
    with pytest.raises(mm.MulmentError, match="no mirror"):
        mm.khop_import(ctx, 3, 2, off, hend, nbr)
    with pytest.raises(mm.MulmentError, match="no mirror"):
        mm.khop_import(ctx, 3, 2, off.cpu().numpy(), hend.cpu().numpy(), nbr.cpu().numpy())
    hend[0] = 1  # the valid path 0-1-2 with k = 2
    kh = mm.khop_import(ctx, 3, 2, off, hend, nbr)
    assert kh.total == 6
    kh.free()
