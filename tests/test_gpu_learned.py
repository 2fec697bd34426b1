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


def test_mlp_init_is_box_muller_of_splitmix64(orc, mm, ctx):
    """mm_mlp_init: parameter p is sd_p * sqrt(-2 ln u1) cos(2 pi u2) with
    u1 = (top 24 bits of draw 2p, plus 1) / 2^24 and u2 = (top 24 bits of
    draw 2p + 1) / 2^24 of SplitMix64 stream (seed, 0, tag 65) (draws from
    the oracle's generator), sd = sqrt(2/8), sqrt(2/64), out_scale/8, 0 by
    block; FP32 logf/cospif against FP64: within 1e-5 relative of max |w|.
    Same seed, same bits."""
    seed, scale = 17, 0.3
    w = mm.mlp_init(ctx, seed, scale).cpu().numpy().astype(np.float64)
    w2 = mm.mlp_init(ctx, seed, scale).cpu().numpy()
    assert np.array_equal(w.astype(np.float32), w2)
    r = orc.draws(seed, 0, 65, 0, 2 * mm.MLP_PARAMS)
    u1 = ((r[0::2] >> np.uint64(40)).astype(np.float64) + 1.0) * 2.0 ** -24
    u2 = (r[1::2] >> np.uint64(40)).astype(np.float64) * 2.0 ** -24
    z = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    sd = np.concatenate([np.full(512, np.sqrt(2 / 8)), np.zeros(64), np.full(4096, np.sqrt(2 / 64)),
                         np.zeros(64), np.full(128, scale / 8), np.zeros(2)])
    ref = sd * z
    err = np.abs(w - ref).max() / np.abs(ref).max()
    print(f"  max err {err:.2e}; W2 std {w[576:4672].std():.4f} (He {np.sqrt(2 / 64):.4f})")
    assert err < 1e-5
    assert np.all(w[sd == 0] == 0)


def _adam_data(count, seed):
    rng = np.random.default_rng(seed)
    X = rng.normal(0, 0.7, (count, 8)).astype(np.float32)
    X[:, 7] = 0
    Y = (0.3 * np.tanh(X[:, :2] * X[:, 2:4]) + rng.normal(0, 0.05, (count, 2))).astype(np.float32)
    from oracle import mlp

    w = mlp.init(5, out_scale=1.0)
    w = (w + rng.normal(0, 0.1, w.size)).astype(np.float32)  # biases away from 0 too
    return X, Y, w


def test_adam_steps_match_oracle(orc, mm, ctx):
    """mm_mlp_train one step at a time (steps 1..5, bias correction of each
    step number) against the oracle's Adam step (Kingma and Ba 2015, Alg. 1)
    fed the gradient the GPU computes on the same minibatch: the oracle's
    minibatch rows, gathered on the host and passed to mm_mlp_grad in order,
    give the GPU training step's gradient bit for bit (the same kernel sees
    the same rows in the same order).  Moments within 1e-6 relative (FP32
    storage of an FP64 step), weight updates within 3e-4 of the largest
    update: storing a weight below 4 in FP32 rounds it by at most 2^-23 ~
    1.2e-7, against updates of up to lr = 1e-3."""
    import torch

    from oracle import mlp

    count, B, lr, seed = 3000, 512, 1e-3, 9
    X, Y, w0 = _adam_data(count, 31)
    Xd, Yd = _dev(mm, X), _dev(mm, Y)
    w = _dev(mm, w0)
    adam = torch.zeros(2 * mm.MLP_PARAMS, dtype=torch.float32, device="cuda")
    P = mm.MLP_PARAMS
    for t in range(1, 6):
        w_prev = w.cpu().numpy().astype(np.float64)
        m_prev = adam[:P].cpu().numpy().astype(np.float64)
        v_prev = adam[P:].cpu().numpy().astype(np.float64)
        rows = mlp.minibatch_rows(count, B, seed, t)
        loss_g, g = mm.mlp_grad(ctx, _dev(mm, X[rows]), _dev(mm, Y[rows]), w)
        loss_t = mm.mlp_train(ctx, Xd, Yd, w, adam, 1, B, lr, seed, step0=t - 1).cpu().numpy()
        w_ref, m_ref, v_ref = mlp.adam_step(w_prev, g.cpu().numpy().astype(np.float64), m_prev,
                                            v_prev, t, lr)
        m_gpu = adam[:P].cpu().numpy().astype(np.float64)
        v_gpu = adam[P:].cpu().numpy().astype(np.float64)
        dw_gpu = w.cpu().numpy().astype(np.float64) - w_prev
        dw_ref = w_ref - w_prev
        em = (np.abs(m_gpu - m_ref) / np.abs(m_ref).max()).max()
        ev = (np.abs(v_gpu - v_ref) / np.abs(v_ref).max()).max()
        ew = (np.abs(dw_gpu - dw_ref) / np.abs(dw_ref).max()).max()
        print(f"  step {t}: loss {loss_t[0]:.4e} (grad call {loss_g:.4e}); "
              f"m err {em:.1e} v err {ev:.1e} update err {ew:.1e}", flush=True)
        assert loss_t[0] == np.float32(loss_g)
        assert em < 1e-6 and ev < 1e-6 and ew < 3e-4


def test_adam_training_matches_oracle(orc, mm, ctx):
    """Ten GPU Adam steps (mm_mlp_train, minibatches of 1024 drawn from 5000
    samples) against the oracle's ten steps from the same start on the same
    draws, its gradient taken with the network the GPU evaluates (BF16
    matrices and inputs): minibatch losses within 2e-2 relative, weights
    within 2e-2 per tensor (norm of the difference over the oracle tensor's
    norm), moments within 5e-2 per tensor."""
    import torch

    from oracle import mlp

    count, B, lr, seed, steps = 5000, 1024, 2e-3, 13, 10
    X, Y, w0 = _adam_data(count, 32)
    w = _dev(mm, w0)
    adam = torch.zeros(2 * mm.MLP_PARAMS, dtype=torch.float32, device="cuda")
    losses = mm.mlp_train(ctx, _dev(mm, X), _dev(mm, Y), w, adam, steps, B, lr, seed)
    losses = losses.cpu().numpy().astype(np.float64)
    wr = w0.astype(np.float64)
    mr = np.zeros_like(wr)
    vr = np.zeros_like(wr)
    lr_ref = []
    Xb = bf16(X)
    for t in range(1, steps + 1):
        rows = mlp.minibatch_rows(count, B, seed, t)
        L, g = mlp.loss_grad(bf16_weights(wr), Xb[rows], Y[rows].astype(np.float64))
        lr_ref.append(L)
        wr, mr, vr = mlp.adam_step(wr, g, mr, vr, t, lr)
    el = np.abs(losses - lr_ref) / np.array(lr_ref)
    print(f"  losses gpu {losses[0]:.4e} .. {losses[-1]:.4e}, oracle {lr_ref[0]:.4e} .. "
          f"{lr_ref[-1]:.4e}; max rel err {el.max():.2e}", flush=True)
    assert el.max() < 2e-2
    wg = w.cpu().numpy().astype(np.float64)
    P = mm.MLP_PARAMS
    mg = adam[:P].cpu().numpy().astype(np.float64)
    o = 0
    for name, shp in BLOCKS:
        k = int(np.prod(shp))
        sl = slice(o, o + k)
        e_w = np.linalg.norm(wg[sl] - wr[sl]) / np.linalg.norm(wr[sl])
        e_m = np.linalg.norm(mg[sl] - mr[sl]) / np.linalg.norm(mr[sl])
        e_dw = np.linalg.norm((wg[sl] - w0[sl]) - (wr[sl] - w0[sl])) / np.linalg.norm(wr[sl] - w0[sl])
        print(f"  {name}: weights {e_w:.2e}, first moment {e_m:.2e}, "
              f"change of the weights {e_dw:.2e}", flush=True)
        assert e_w < 2e-2 and e_m < 5e-2, name
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
