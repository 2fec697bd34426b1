"""Pins of the FP64 oracle of the learned far-field correction (q = 0).

The correction of an accepted cell is kappa (h0 e + h1 p) with
kappa = m t^2 / d; training targets are the exact residual of the cell in
those units.  Pinned against: finite differences (backward pass), a
hand-built network, the multipole series of the 2-D log-potential field
sum_v 1/conj(z - w_v) (targets, rotated moments), cell geometry
(containment of the cell's points), and the exact all-pairs field (a
network that outputs the exact targets must reproduce it)."""
import numpy as np
import pytest

import oracle
from oracle import mlp


def _layout(n, seed, clumps=False):
    rng = np.random.default_rng(seed)
    xy = rng.random((n, 2)) * 20.0
    if clumps:
        c = rng.random((6, 2)) * 20.0
        k = rng.integers(0, 6, n // 2)
        xy[: n // 2] = c[k] + rng.normal(0, 0.3, (n // 2, 2))
    return xy.astype(np.float32).astype(np.float64)


def test_mlp_backward_matches_finite_differences():
    rng = np.random.default_rng(3)
    w = mlp.init(5, out_scale=1.0)
    w += rng.normal(0, 0.05, w.size)  # non-zero biases
    X = rng.normal(0, 1, (37, 8))
    Y = rng.normal(0, 1, (37, 2))
    L, g = mlp.loss_grad(w, X, Y)
    idx = rng.choice(w.size, 300, replace=False)
    eps = 1e-6
    fd = np.empty(idx.size)
    for j, i in enumerate(idx):
        wp, wm = w.copy(), w.copy()
        wp[i] += eps
        wm[i] -= eps
        fd[j] = (mlp.loss_grad(wp, X, Y)[0] - mlp.loss_grad(wm, X, Y)[0]) / (2 * eps)
    err = np.abs(fd - g[idx]) / np.maximum(np.abs(g[idx]), 1e-3)
    assert err.max() < 1e-6, err.max()


def test_mlp_hand_built_network():
    p = {"W1": np.zeros((64, 8)), "b1": np.zeros(64), "W2": np.eye(64), "b2": np.zeros(64),
         "W3": np.zeros((2, 64)), "b3": np.array([0.5, 0.25])}
    p["W1"][:8, :8] = np.eye(8)
    p["W3"][0, 0] = 1.0
    p["W3"][1, 1] = -1.0
    w = mlp.pack(p)
    X = np.array([[0.3, 0.7, 0, 0, 0, 0, 0, 0], [-0.3, -0.7, 1, 1, 1, 1, 1, 1]])
    want = np.array([[0.8, 0.25 - 0.7], [0.5, 0.25]])
    h, _ = mlp.forward(w, X)
    assert np.allclose(h, want, rtol=0, atol=1e-15)
    assert np.allclose(oracle.mlp_forward_c(w, X), want, rtol=0, atol=1e-15)


def _cells(xy):
    bh = oracle.barnes_hut(xy, 1.0)
    return bh.order, bh.nodes


@pytest.mark.parametrize("clumps", [False, True])
def test_targets_match_multipole_series(clumps):
    xy = _layout(600, 11, clumps)
    S = oracle.far_samples(xy, 1.0)
    order, nodes = _cells(xy)
    checked = 0
    for j in range(S.u.size):
        depth, first, count, leaf, _ = nodes[S.node[j]]
        assert leaf == 0 and count >= 2
        pts = xy[order[first:first + count]]
        com = pts.mean(0)
        z = complex(*(xy[S.u[j]] - com))
        w = (pts[:, 0] - com[0]) + 1j * (pts[:, 1] - com[1])
        if np.abs(w).max() > 0.5 * abs(z):
            continue
        # sum_v 1/conj(z - w_v) - m/conj(z) = conj(sum_{k>=2} Q_k / z^(k+1))
        ser = sum(np.sum(w ** k) / z ** (k + 1) for k in range(2, 48))
        R = np.conj(ser)
        kex, key = S.coef[j]
        kap2 = kex * kex + key * key
        h = np.array([R.real * kex + R.imag * key, -R.real * key + R.imag * kex]) / kap2
        assert np.allclose(S.target[j], h, rtol=1e-9, atol=1e-12 * np.abs(h).max())
        # quadrupole term alone, from the rotated moments
        quad = np.conj(np.sum(w ** 2) / z ** 3)
        hq = np.array([quad.real * kex + quad.imag * key, -quad.real * key + quad.imag * kex]) / kap2
        f = S.feat[j]
        assert np.allclose(hq, [f[3] - f[4], -2 * f[5]], rtol=1e-9, atol=1e-12)
        checked += 1
    assert checked > 200


def test_features_cell_geometry():
    xy = _layout(500, 12, True)
    S = oracle.far_samples(xy, 1.0)
    order, nodes = _cells(xy)
    for j in range(0, S.u.size, 7):
        depth, first, count, leaf, _ = nodes[S.node[j]]
        pts = xy[order[first:first + count]]
        com = pts.mean(0)
        d = np.linalg.norm(xy[S.u[j]] - com)
        e = (xy[S.u[j]] - com) / d
        p = np.array([-e[1], e[0]])
        f = S.feat[j]
        t = f[0]
        s = t * d
        # kappa = m t^2 / d
        assert np.isclose(np.linalg.norm(S.coef[j]), count * t * t / d, rtol=1e-12)
        assert np.isclose(f[6], np.log2(count) / 16, rtol=0, atol=1e-15)
        assert f[7] == 0.0
        # centre of the tight cell from the offset features; all points inside
        g = com - s * (f[1] * e + f[2] * p)
        assert np.all(np.abs(pts - g) <= s / 2 * (1 + 1e-9))
        # tight: the points do not fit in one quadrant
        quad = (pts[:, 0] >= g[0]).astype(int) + 2 * (pts[:, 1] >= g[1])
        assert np.unique(quad).size >= 2
        # rotated central moments per unit mass
        M = (pts - com).T @ (pts - com) / count
        assert np.allclose([e @ M @ e / s**2, p @ M @ p / s**2, e @ M @ p / s**2], f[3:6],
                           rtol=1e-9, atol=1e-12)


def test_exact_targets_reproduce_exact_field():
    xy = _layout(700, 13, True)
    S = oracle.far_samples(xy, 1.0)
    F = oracle.barnes_hut(xy, 1.0).F.copy()
    kex, key = S.coef[:, 0], S.coef[:, 1]
    h0, h1 = S.target[:, 0], S.target[:, 1]
    np.add.at(F[:, 0], S.u, h0 * kex - h1 * key)
    np.add.at(F[:, 1], S.u, h0 * key + h1 * kex)
    Fx = oracle.farfield_exact(xy)
    scale = np.linalg.norm(Fx, axis=1).mean()
    assert np.abs(F - Fx).max() < 1e-11 * scale


def test_learned_field_composition():
    xy = _layout(400, 14, True)
    S = oracle.far_samples(xy, 1.0)
    F0 = oracle.barnes_hut(xy, 1.0).F
    # zero network: the plain Barnes-Hut field, bit for bit
    assert np.array_equal(oracle.barnes_hut_learned(xy, 1.0, np.zeros(mlp.N_PARAM)), F0)
    # any network: plain field + sum over accepted cells of kappa (h0 e + h1 p)
    w = mlp.init(9, out_scale=1.0)
    h, _ = mlp.forward(w, S.feat)
    F = F0.copy()
    kex, key = S.coef[:, 0], S.coef[:, 1]
    np.add.at(F[:, 0], S.u, h[:, 0] * kex - h[:, 1] * key)
    np.add.at(F[:, 1], S.u, h[:, 0] * key + h[:, 1] * kex)
    FL = oracle.barnes_hut_learned(xy, 1.0, w)
    assert np.abs(FL - F).max() < 1e-12 * np.abs(F0).max()
    # samples are recorded in ascending target order
    assert np.all(np.diff(S.u) >= 0)


def test_bh_learned_rows_is_the_full_field_at_those_rows(orc):
    """The sampled variant used for large checks visits the same tree."""
    from oracle import mlp

    rng = np.random.default_rng(3)
    x = rng.random((3000, 2)) * 55
    w = mlp.init(5, out_scale=0.3)
    rows = rng.choice(3000, 200, replace=False)
    full = orc.barnes_hut_learned(x, 1.0, w)
    part = orc.barnes_hut_learned_rows(x, 1.0, w, rows)
    assert np.array_equal(full[rows], part)


# ------------------------------------------------------------------ Adam

def test_adam_two_steps_hand_worked():
    """Adam (Kingma and Ba 2015, Alg. 1) by hand, one scalar, lr = 0.1,
    eps = 0, w0 = 1, gradients 1 then 3.
    t = 1: m = 0.1, v = 0.001; m_hat = 0.1/(1-0.9) = 1, v_hat = 0.001/(1-0.999)
    = 1; w1 = 1 - 0.1 * 1/1 = 0.9.
    t = 2: m = 0.9*0.1 + 0.1*3 = 0.39, v = 0.999*0.001 + 0.001*9 = 0.009999;
    m_hat = 0.39/(1-0.81) = 39/19, v_hat = 0.009999/(1-0.998001) = 9999/1999;
    w2 = 0.9 - 0.1 * (39/19) / sqrt(9999/1999) = 0.808221888..."""
    w, m, v = mlp.adam_step(np.array([1.0]), np.array([1.0]), np.zeros(1), np.zeros(1), 1, 0.1,
                            eps=0.0)
    assert abs(w[0] - 0.9) < 1e-15 and abs(m[0] - 0.1) < 1e-15 and abs(v[0] - 0.001) < 1e-15
    w, m, v = mlp.adam_step(w, np.array([3.0]), m, v, 2, 0.1, eps=0.0)
    assert abs(m[0] - 0.39) < 1e-15 and abs(v[0] - 0.009999) < 1e-15
    expect = 0.9 - 0.1 * (39.0 / 19.0) / np.sqrt(9999.0 / 1999.0)
    assert abs(expect - 0.808221888) < 1e-9
    assert abs(w[0] - expect) < 1e-14


def test_adam_constant_gradient_moves_lr_per_step():
    """With a constant gradient g from zero moments the bias-corrected
    estimates are exactly g and g^2 at every step (that is what the
    correction is for), so each step moves every parameter by
    lr g / (|g| + eps): a wrong correction power or decay fails this."""
    rng = np.random.default_rng(5)
    g = rng.normal(0, 1, 50) * 10.0 ** rng.integers(-3, 3, 50)
    w0 = rng.normal(0, 1, 50)
    w, m, v = w0.copy(), np.zeros(50), np.zeros(50)
    for t in range(1, 41):
        w_prev = w
        w, m, v = mlp.adam_step(w, g, m, v, t, 1e-3)
        np.testing.assert_allclose(w_prev - w, 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-9)
    np.testing.assert_allclose(w, w0 - 40e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-12)


def test_adam_is_invariant_to_gradient_scale_and_eps_sits_outside_the_root():
    """Scaling every gradient by c > 0 leaves the steps unchanged (up to
    eps); a gradient of 1e-8 at t = 1 moves by lr/2, which holds only with
    eps added to sqrt(v_hat)."""
    rng = np.random.default_rng(6)
    G = rng.normal(0, 1, (6, 30))
    wa = wb = np.zeros(30)
    ma = mb = va = vb = np.zeros(30)
    for t in range(1, 7):
        wa, ma, va = mlp.adam_step(wa, G[t - 1], ma, va, t, 0.01)
        wb, mb, vb = mlp.adam_step(wb, 1000.0 * G[t - 1], mb, vb, t, 0.01)
    np.testing.assert_allclose(wa, wb, rtol=1e-6, atol=1e-12)
    w, _, _ = mlp.adam_step(np.zeros(1), np.array([1e-8]), np.zeros(1), np.zeros(1), 1, 0.01)
    assert abs(w[0] + 0.005) < 1e-12


def test_minibatch_rows_follow_splitmix64_known_answers():
    """Step t's rows are draws 0, 1, ... of the SplitMix64 stream
    seed ^ (t << 48) ^ (64 << 32) modulo the sample count; the stream state
    1234567 has the published outputs in tests/golden/splitmix64.json."""
    import json
    import os

    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "splitmix64.json")))
    outs = [v for v in gold["vectors"] if v["state"] == 1234567][0]["outputs"]
    for t in (1, 7):
        seed = 1234567 ^ (t << 48) ^ (64 << 32)
        for N in (1000, 4099, 2 ** 31 - 1):
            rows = mlp.minibatch_rows(N, 3, seed, t)
            assert rows.tolist() == [o % N for o in outs]


def test_adam_training_fits_a_teacher_network():
    """train(): a student from another initialisation fits targets made by a
    teacher network (the loss falls by more than 20x in 600 steps) and the
    run is a deterministic function of its inputs."""
    rng = np.random.default_rng(8)
    X = rng.normal(0, 0.7, (4000, 8))
    X[:, 7] = 0
    teacher = mlp.init(11, out_scale=1.0)
    Y, _ = mlp.forward(teacher, X)
    w0 = mlp.init(12, out_scale=0.1)
    z = np.zeros_like(w0)
    w, m, v, L = mlp.train(w0, z, z, X, Y, 600, 256, 3e-3, 5)
    assert L[-20:].mean() < L[:5].mean() / 20
    w2, _, _, L2 = mlp.train(w0, z, z, X, Y, 600, 256, 3e-3, 5)
    assert np.array_equal(w, w2) and np.array_equal(L, L2)
    # resuming at step0 continues the same sequence of steps
    wa, ma, va, _ = mlp.train(w0, z, z, X, Y, 300, 256, 3e-3, 5)
    wb, _, _, _ = mlp.train(wa, ma, va, X, Y, 300, 256, 3e-3, 5, step0=300)
    assert np.array_equal(wb, w)
