"""Cluster far field of Eq. 3 (MulMent_h) on the GPU vs the FP64 oracle,
through the C-ABI.

Bars: the far field within 1e-4 of max(|F_u|, mean |F|) per vertex (FP32
against FP64, as for the exact far field); with identity maps it equals the
GPU's exact all-pairs field within 1e-5; a MulMent_h layout's maxent-stress
within 1% of the oracle's MulMent_h layout, run-to-run and graph-replay
bit-identical.
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


def _maps(n, n1, nh, seed):
    rng = np.random.default_rng(seed)
    cl1 = rng.integers(0, n1, n).astype(np.int32)
    cl1[:n1] = np.arange(n1)
    up = rng.integers(0, nh, n1).astype(np.int32)
    up[:nh] = np.arange(nh)
    return cl1, up[cl1].astype(np.int32)


def _maps_spatial(x, g1, gh):
    """Nested square cells (g1 = a multiple of gh per side) as the two
    cluster maps, the way a hierarchy groups nearby vertices; ids dense."""
    lo, hi = x.min(0), x.max(0)
    u = (x - lo) / np.maximum(hi - lo, 1e-9)
    c1 = np.minimum((u * g1).astype(np.int64), g1 - 1)
    cid1 = c1[:, 0] * g1 + c1[:, 1]
    chh = c1 // (g1 // gh)
    cidh = chh[:, 0] * gh + chh[:, 1]
    _, cl1 = np.unique(cid1, return_inverse=True)
    _, clh = np.unique(cidh, return_inverse=True)
    return (cl1.astype(np.int32), int(cl1.max()) + 1, clh.astype(np.int32), int(clh.max()) + 1)


def _err(F, Fr):
    nr = np.linalg.norm(Fr, axis=1)
    scale = np.maximum(nr, nr.mean())
    return float(np.max(np.linalg.norm(F - Fr, axis=1) / scale))


@pytest.mark.parametrize("n,n1,nh,q,weights", [(1000, 500, 60, 0.0, False),
                                               (1000, 500, 60, 1.0, True),
                                               (4099, 2000, 1, 0.0, False),
                                               (3, 2, 1, 0.0, False),
                                               (4099, 64, 8, 0.0, True),
                                               (20000, 128, 16, 0.0, False),
                                               (50000, 256, 32, 1.0, False)])
def test_cluster_far_matches_oracle(orc, mm, ctx, n, n1, nh, q, weights):
    """Random cluster maps for the small cases; for the large ones nested
    spatial cells (n1, nh = cells per side), as a hierarchy builds them --
    random maps put representatives near the centre, where FP32 offsets to
    them lose digits that have nothing to do with the method."""
    print(f"[cluster far] n={n} n1={n1} nh={nh} q={q} w={weights}", flush=True)
    rng = np.random.default_rng(n + nh)
    x = (rng.random((n, 2)) * np.sqrt(n)).astype(np.float32)
    if n > 1000 and nh > 1:
        cl1, n1, clh, nh = _maps_spatial(x.astype(np.float64), n1, nh)
    else:
        cl1, clh = _maps(n, n1, nh, n)
    c = rng.integers(1, 6, n).astype(np.int32) if weights else None
    F = mm.repulsion_cluster(ctx, x, cl1, n1, clh, nh, node_w=c, q=q).cpu().numpy()
    Fr = orc.cluster_far_field(x.astype(np.float64), c, cl1, n1, clh, nh, q)
    e = _err(F, Fr)
    print(f"  max err {e:.2e}", flush=True)
    assert e < 1e-4


def test_identity_maps_equal_exact(mm, ctx):
    n = 3000
    x = (np.random.default_rng(5).random((n, 2)) * 50).astype(np.float32)
    ident = np.arange(n, dtype=np.int32)
    F = mm.repulsion_cluster(ctx, x, ident, n, ident, n).cpu().numpy()
    Fe = mm.repulsion(ctx, x, 0.0, -1.0)["F"].cpu().numpy()
    assert _err(F, Fe.astype(np.float64)) < 1e-5


def test_out_of_range_rejected(mm, ctx):
    x = np.zeros((4, 2), np.float32)
    x[:, 0] = np.arange(4)
    with pytest.raises(mm.MulmentError, match="EINVAL"):
        mm.repulsion_cluster(ctx, x, np.array([0, 1, 2, 5], np.int32), 4,
                             np.array([0, 0, 1, 1], np.int32), 2)


@pytest.mark.parametrize("name,h", [("grid32", 1), ("rgg4k", 2), ("rgg4k", 10)])
def test_mulment_h_layout_matches_oracle(orc, mm, ctx, name, h):
    g = synth.grid(32, 32) if name == "grid32" else synth.rgg(4000, 3)
    print(f"[MulMent_{h}] {name} n={g.n}", flush=True)
    kw = dict(k=3, theta=0.5, alpha_decay=0.5, coarsest_n=20, seed=2, approx_h=h)
    dg = ctx.graph(g.row_ptr, g.col)
    xg, st = mm.layout(ctx, dg, mm.Params(**kw))
    xg2, _ = mm.layout(ctx, dg, mm.Params(**kw))
    xd, _ = mm.layout(ctx, dg, mm.Params(use_graphs=0, **kw))
    assert np.array_equal(xg.cpu().numpy(), xg2.cpu().numpy())
    assert np.array_equal(xg.cpu().numpy(), xd.cpu().numpy())
    xo, sto = orc.layout(g, orc.Params(**kw))
    assert [l["n"] for l in st["per_level"]][::-1] == [l["n"] for l in sto["levels"]]
    kh = orc.khop_build(g.row_ptr, g.col, 3)
    mg = orc.objective(kh, xg.cpu().numpy().astype(np.float64), 0.008)["M"]
    mo = orc.objective(kh, xo, 0.008)["M"]
    print(f"  M gpu {mg:.6g} oracle {mo:.6g}", flush=True)
    assert abs(mg - mo) <= 0.01 * abs(mo)


@pytest.mark.parametrize("h", [2, 7])
def test_update_protocol_matches_oracle(orc, mm, ctx, h):
    """Warm start of a churned RGG at alpha_min with the hierarchy cut at h
    levels (Sec. 4.3): maxent-stress within 1% of the oracle's update."""
    g = synth.rgg(3000, 11)
    q = synth.churn_snapshot(g, 12, 0.05, 2)
    kw = dict(k=3, theta=0.5, alpha_decay=0.5, coarsest_n=20, seed=4, approx_h=h)
    xg0, _ = mm.layout(ctx, ctx.graph(g.row_ptr, g.col), mm.Params(**kw))
    x0 = xg0.cpu().numpy()
    dq = ctx.graph(q.row_ptr, q.col)
    xu, st = mm.layout(ctx, dq, mm.Params(**kw), init_xy=x0)
    xu2, _ = mm.layout(ctx, dq, mm.Params(**kw), init_xy=x0)
    assert st["levels"] == 1
    assert np.array_equal(xu.cpu().numpy(), xu2.cpu().numpy())
    xo, sto = orc.layout(q, orc.Params(**kw), init_xy=x0.astype(np.float64))
    assert len(sto["hierarchy"]) <= h
    kh = orc.khop_build(q.row_ptr, q.col, 3)
    mg = orc.objective(kh, xu.cpu().numpy().astype(np.float64), 0.008)["M"]
    mo = orc.objective(kh, xo, 0.008)["M"]
    print(f"  h={h} M gpu {mg:.6g} oracle {mo:.6g}", flush=True)
    assert abs(mg - mo) <= 0.01 * abs(mo)
