"""Learned far-field correction on the GPU vs the FP64 oracle, through the C-ABI.

Bars (stated per result):
* training samples: (target, cell) lists bit-exact per target; features
  within 1e-4 absolute (FP32 vs FP64, features are O(1)); exact residual
  targets within 1e-4 * (|h*| + 1e-3); kappa e within 1e-5 relative;
* MLP forward (BF16 MFMA, FP32 accumulation) within 1e-2 of max |h| of the
  oracle fed the same BF16-rounded weights and features;
* MLP gradient within 2e-2 relative (norm) per parameter tensor, loss within
  1e-2 relative;
* learned far field within 2e-3 * max(|F_u|, mean |F|) of the oracle with the
  same BF16-rounded weights; a zero network gives the plain field bit for
  bit;
* gain: after training on samples of layouts made by the method, the far
  field at theta = 1 with the network is closer to the exact field than
  plain Barnes-Hut at theta = 1.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

BLOCKS = [("W1", (64, 8)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("W3", (2, 64)),
          ("b3", (2,))]


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


def bf16(a):
    """Round to BF16 (nearest even), returned as float64."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def bf16_weights(w):
    """The network the GPU evaluates: BF16 matrices, FP32 biases."""
    w = np.asarray(w, dtype=np.float32).astype(np.float64).copy()
    o = 0
    for name, shp in BLOCKS:
        k = int(np.prod(shp))
        if name.startswith("W"):
            w[o:o + k] = bf16(w[o:o + k])
        o += k
    return w


def _layout(n, seed, clumps=True):
    rng = np.random.default_rng(seed)
    xy = rng.random((n, 2)) * 30.0
    if clumps:
        c = rng.random((8, 2)) * 30.0
        k = rng.integers(0, 8, n // 2)
        xy[: n // 2] = c[k] + rng.normal(0, 0.4, (n // 2, 2))
    return xy.astype(np.float32)


def _dev(mm, a):
    import torch

    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


@pytest.mark.parametrize("count", [1, 17, 1000, 4099])
def test_mlp_forward_matches_oracle(orc, mm, ctx, count):
    from oracle import mlp

    print(f"[mlp fwd] count={count}", flush=True)
    rng = np.random.default_rng(count)
    w = mlp.init(2, out_scale=1.0).astype(np.float32)
    w[512:576] = rng.normal(0, 0.1, 64)  # b1
    X = rng.normal(0, 0.7, (count, 8)).astype(np.float32)
    X[:, 7] = 0
    h = mm.mlp_forward(ctx, _dev(mm, X), _dev(mm, w)).cpu().numpy()
    ref, _ = mlp.forward(bf16_weights(w), bf16(X))
    err = np.abs(h - ref).max() / np.abs(ref).max()
    print(f"  max err / max|h| = {err:.2e}")
    assert err < 1e-2


@pytest.mark.parametrize("count", [16, 300, 5000])
def test_mlp_grad_matches_oracle(orc, mm, ctx, count):
    from oracle import mlp

    print(f"[mlp grad] count={count}", flush=True)
    rng = np.random.default_rng(100 + count)
    w = mlp.init(4, out_scale=1.0).astype(np.float32)
    w += rng.normal(0, 0.02, w.size).astype(np.float32)
    X = rng.normal(0, 0.7, (count, 8)).astype(np.float32)
    X[:, 7] = 0
    Y = rng.normal(0, 0.5, (count, 2)).astype(np.float32)
    loss, g = mm.mlp_grad(ctx, _dev(mm, X), _dev(mm, Y), _dev(mm, w))
    g = g.cpu().numpy().astype(np.float64)
    L_ref, g_ref = mlp.loss_grad(bf16_weights(w), bf16(X), Y.astype(np.float64))
    assert abs(loss - L_ref) <= 1e-2 * L_ref
    o = 0
    for name, shp in BLOCKS:
        k = int(np.prod(shp))
        a, b = g[o:o + k], g_ref[o:o + k]
        rel = np.linalg.norm(a - b) / np.linalg.norm(b)
        print(f"  {name}: rel err {rel:.2e}")
        assert rel < 2e-2, name
        o += k


@pytest.mark.parametrize("n,seed,theta", [(700, 1, 1.0), (3000, 2, 1.0), (3000, 3, 0.5),
                                          (20000, 4, 1.0)])
def test_samples_match_oracle(orc, mm, ctx, n, seed, theta):
    print(f"[samples] n={n} seed={seed} theta={theta}", flush=True)
    xy = _layout(n, seed)
    S = mm.far_samples(ctx, _dev(mm, xy), theta)
    u = S["u"].cpu().numpy()
    node = S["node"].cpu().numpy()
    feat = S["feat"].cpu().numpy().astype(np.float64)
    tgt = S["target"].cpu().numpy().astype(np.float64)
    coef = S["coef"].cpu().numpy().astype(np.float64)
    R = orc.far_samples(xy.astype(np.float64), theta)
    assert u.size == R.u.size
    # GPU rows: by Morton rank of u, visit order within u; oracle: by u.
    perm = np.argsort(u, kind="stable")
    assert np.array_equal(u[perm], R.u)
    assert np.array_equal(node[perm].astype(np.int64), R.node)
    df = np.abs(feat[perm] - R.feat).max()
    dt = (np.abs(tgt[perm] - R.target) / (np.abs(R.target) + 1e-3)).max()
    dc = (np.abs(coef[perm] - R.coef) / np.abs(R.coef).max(axis=1, keepdims=True)).max()
    print(f"  samples={u.size} feat err {df:.2e} target rel err {dt:.2e} coef rel err {dc:.2e}")
    assert df < 1e-4 and dt < 1e-4 and dc < 1e-5


def test_zero_network_is_plain_barnes_hut(mm, ctx):
    xy = _dev(mm, _layout(5000, 7))
    w = _dev(mm, np.zeros(mm.MLP_PARAMS, np.float32))
    FL = mm.repulsion_learned(ctx, xy, 1.0, w).cpu().numpy()
    F0 = mm.repulsion(ctx, xy, 0.0, 1.0)["F"].cpu().numpy()
    assert np.array_equal(FL, F0)


@pytest.mark.parametrize("n,seed", [(900, 5), (12000, 6)])
def test_learned_field_matches_oracle(orc, mm, ctx, n, seed):
    from oracle import mlp

    print(f"[learned F] n={n}", flush=True)
    xy = _layout(n, seed)
    w = mlp.init(7, out_scale=0.3).astype(np.float32)
    F = mm.repulsion_learned(ctx, _dev(mm, xy), 1.0, _dev(mm, w)).cpu().numpy()
    F2 = mm.repulsion_learned(ctx, _dev(mm, xy), 1.0, _dev(mm, w)).cpu().numpy()
    assert np.array_equal(F, F2)  # deterministic
    ref = orc.barnes_hut_learned(xy.astype(np.float64), 1.0, bf16_weights(w))
    plain = orc.barnes_hut(xy.astype(np.float64), 1.0).F
    mag = np.maximum(np.linalg.norm(ref, axis=1), np.linalg.norm(ref, axis=1).mean())
    err = (np.linalg.norm(F - ref, axis=1) / mag).max()
    corr = (np.linalg.norm(ref - plain, axis=1) / mag).max()
    print(f"  max err {err:.2e} (correction size {corr:.2e})")
    assert corr > 1e-3  # the network changes the field
    assert err < 2e-3


def _train(mm, ctx, seeds, steps=1500, theta=1.0):
    """Samples at theta from layouts of RGG 2^12 (mean degree 8) made by the
    method, then Adam on the GPU.  Returns (weights, losses)."""
    import torch

    from oracle import mlp

    feats, tgts = [], []
    for s in seeds:
        g = synth.rgg(1 << 12, s, 8.0)
        dg = ctx.graph(g.row_ptr, g.col)
        xy, _ = mm.layout(ctx, dg, mm.Params(k=3, theta=0.5, alpha_decay=0.5, coarsest_n=50,
                                             seed=s, validate=0))
        S = mm.far_samples(ctx, xy, theta)
        feats.append(S["feat"])
        tgts.append(S["target"])
    feat = torch.cat(feats)
    tgt = torch.cat(tgts)
    w = torch.as_tensor(mlp.init(11, out_scale=0.1).astype(np.float32), device="cuda")
    adam = torch.zeros(2 * mm.MLP_PARAMS, dtype=torch.float32, device="cuda")
    losses = mm.mlp_train(ctx, feat, tgt, w, adam, steps, 1024, 2e-3, 5)
    return w, losses.cpu().numpy(), feat.shape[0]


@pytest.fixture(scope="module")
def trained(mm, ctx):
    print("[train] RGG 2^12 x 3 layouts", flush=True)
    return _train(mm, ctx, [21, 22, 23])


def test_training_is_deterministic(mm, ctx, trained):
    w, losses, m = trained
    w2, losses2, _ = _train(mm, ctx, [21, 22, 23])
    assert np.array_equal(losses, losses2)
    assert np.array_equal(w.cpu().numpy(), w2.cpu().numpy())


def test_trained_network_beats_plain_barnes_hut(mm, ctx, trained):
    w, losses, m = trained
    first, last = losses[:20].mean(), losses[-100:].mean()
    print(f"  samples {m}; loss {first:.3e} -> {last:.3e}")
    assert last < 0.5 * first
    g = synth.rgg(1 << 12, 99, 8.0)
    dg = ctx.graph(g.row_ptr, g.col)
    xy, _ = mm.layout(ctx, dg, mm.Params(k=3, theta=0.5, alpha_decay=0.5, coarsest_n=50,
                                         seed=99, validate=0))
    Fx = mm.repulsion(ctx, xy, 0.0, -1.0)["F"].double()
    scale = Fx.norm(dim=1).mean()

    def err(F):
        return float(((F.double() - Fx).norm(dim=1).mean() / scale).item())

    e_plain = err(mm.repulsion(ctx, xy, 0.0, 1.0)["F"])
    e_learn = err(mm.repulsion_learned(ctx, xy, 1.0, w))
    e_half = err(mm.repulsion(ctx, xy, 0.0, 0.5)["F"])
    print(f"  mean rel error vs exact: theta=1 {e_plain:.3e}, theta=1+MLP {e_learn:.3e}, "
          f"theta=0.5 {e_half:.3e}")
    assert e_learn < 0.6 * e_plain


def test_learned_layout_matches_oracle(orc, mm, ctx, trained):
    w, _, _ = trained
    g = synth.grid(32, 32)
    p = mm.Params(k=3, theta=1.0, alpha_decay=0.5, max_levels=3, seed=1, mlp_weights=w)
    xy, st = mm.layout(ctx, ctx.graph(g.row_ptr, g.col), p)
    kh = mm.khop_build(ctx, ctx.graph(g.row_ptr, g.col), 3)
    M_gpu = mm.objective(ctx, kh, xy, 0.008)["M"]
    kh.free()
    op = orc.Params(k=3, theta=1.0, alpha_decay=0.5, max_levels=3, seed=1,
                    mlp=bf16_weights(w.cpu().numpy()))
    x_orc, _ = orc.layout(g, op)
    khr = orc.khop_build(g.row_ptr, g.col, 3)
    M_orc = orc.objective(khr, x_orc, 0.008)["M"]
    print(f"  M_S gpu {M_gpu:.6e} oracle {M_orc:.6e}")
    assert abs(M_gpu - M_orc) <= 0.01 * abs(M_orc)
