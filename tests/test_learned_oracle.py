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
