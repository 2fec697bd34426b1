"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test names the passage of the paper (section / equation / table) it
follows.  None of these re-types an oracle formula and compares it to
itself: they use closed forms, invariants, known-answer vectors, brute force
and library routines (scipy shortest paths, a 1-D minimiser) instead.
"""
import json
import math
import os
import subprocess
import sys

import numpy as np
import pytest
from scipy.optimize import minimize_scalar
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import shortest_path

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


# ------------------------------------------------------------------ RNG (P9)

def test_splitmix64_known_answers(orc):
    """The counter-based generator is SplitMix64 as published."""
    vec = json.load(open(os.path.join(GOLDEN, "splitmix64.json")))["vectors"]
    assert orc.splitmix64_at(0, 0) == int(vec[0]["outputs_hex"][0], 16)
    for i, v in enumerate(vec[1]["outputs"]):
        assert orc.splitmix64_at(vec[1]["state"], i) == v


def test_init_layout_is_exact_24bit_grid(orc):
    """Initial layout (Section 3.1 replacement): uniform draws in [0,1) on the
    2^-24 grid, so FP32 and FP64 hold the same values."""
    x = orc.init_layout(5000, 7, 3)
    assert x.min() >= 0 and x.max() < 1
    assert np.all(x * 2**24 == np.floor(x * 2**24))
    assert np.all(x.astype(np.float32).astype(np.float64) == x)
    d = orc.draws(7, 3, 1, 0, 10000)
    assert np.array_equal((d >> np.uint64(40)).astype(np.float64) * 2.0**-24, x.reshape(-1))


# ----------------------------------------------------------- k-hop sets (P7)

def _apsp_hops(g):
    n = g.n
    a = csr_matrix((np.ones(g.nnz), g.col, g.row_ptr), shape=(n, n))
    return shortest_path(a, method="D", unweighted=True, directed=False)


def _floyd(g):
    n = g.n
    d = np.full((n, n), np.inf)
    np.fill_diagonal(d, 0)
    for u in range(n):
        d[u, g.col[g.row_ptr[u]:g.row_ptr[u + 1]]] = 1
    for w in range(n):
        d = np.minimum(d, d[:, w:w + 1] + d[w:w + 1, :])
    return d


@pytest.mark.parametrize("name,k", [("grid", 3), ("tree", 3), ("rgg", 2), ("star", 2),
                                    ("path", 1), ("path", 4), ("tri", 2), ("btree", 3)])
def test_khop_equals_brute_force_apsp(orc, name, k):
    """S_k(u) = {v != u : hop(u,v) <= k} sorted by (hop, v), against all-pairs
    shortest paths (scipy) and Floyd-Warshall."""
    g = {"grid": lambda: synth.grid(9, 7), "tree": lambda: synth.random_tree(300, 3),
         "rgg": lambda: synth.rgg(400, 5), "star": lambda: synth.star(40),
         "path": lambda: synth.path(30), "tri": synth.two_triangles,
         "btree": lambda: synth.complete_binary_tree(6)}[name]()
    kh = orc.khop_build(g.row_ptr, g.col, k)
    D = _apsp_hops(g)
    if g.n <= 400:
        assert np.array_equal(D, _floyd(g))
    for u in range(g.n):
        hops = D[u]
        want_v = [v for v in np.lexsort((np.arange(g.n), hops)) if v != u and hops[v] <= k]
        assert np.array_equal(kh.row(u), np.asarray(want_v, dtype=np.int32))
        assert np.array_equal(kh.hops(u), hops[kh.row(u)].astype(int))


# ------------------------------------------------------- far field (P1, P10)

def _points(n, seed):
    rng = np.random.default_rng(seed)
    a = rng.random((n // 2, 2)) * 10
    b = 5 + 0.01 * rng.standard_normal((n - n // 2, 2))  # a tight cluster
    return np.concatenate([a, b])


@pytest.mark.parametrize("q", [0.0, 1.0])
def test_farfield_exact_vs_bh_theta0_vs_numpy(orc, q):
    """BH at theta = 0 opens every cell, so it must equal the exact sum."""
    x = _points(300, 1)
    F = orc.farfield_exact(x, q)
    d = x[:, None, :] - x[None, :, :]
    D2 = (d**2).sum(-1)
    np.fill_diagonal(D2, np.inf)
    Fn = (d / D2[..., None] ** ((q + 2) / 2)).sum(1)
    assert rel(F, Fn) < 1e-12
    bh = orc.barnes_hut(x, 0.0, q)
    assert rel(bh.F, F) < 1e-12
    assert bh.accepted == 0 and bh.leaf_pairs == 300 * 299


def test_bh_error_decreases_with_theta(orc):
    x = _points(2000, 2)
    F = orc.farfield_exact(x)
    scale = np.maximum(np.linalg.norm(F, axis=1), np.linalg.norm(F, axis=1).mean())
    errs = []
    for th in [1.2, 0.8, 0.5, 0.3, 0.15, 0.0]:
        bh = orc.barnes_hut(x, th)
        errs.append(float(np.max(np.linalg.norm(bh.F - F, axis=1) / scale)))
    assert all(errs[i + 1] <= errs[i] * 1.05 for i in range(len(errs) - 1)), errs
    assert errs[2] < 0.05 and errs[-1] < 1e-12


def test_bh_tree_geometry(orc):
    """Quadtree invariants: pre-order, children inside parents, leaves tile the
    sorted order, codes interleave the quantised coordinates."""
    x = _points(500, 3)
    bh = orc.barnes_hut(x, 0.5)
    nodes = bh.nodes
    leaves = nodes[nodes[:, 3] == 1]
    assert leaves[:, 2].sum() == 500
    assert np.array_equal(np.cumsum(np.concatenate([[0], leaves[:-1, 2]])), leaves[:, 1])
    assert nodes[0, 0] == 0 or nodes[0, 2] == 500
    # sorted order is by (code, id)
    o = bh.order
    c = bh.codes[o]
    assert np.all((c[1:] > c[:-1]) | ((c[1:] == c[:-1]) & (o[1:] > o[:-1])))
    # codes: quantise with the power-of-two box and interleave (x even bits)
    ext = max(np.ptp(x[:, 0]), np.ptp(x[:, 1]))
    e = math.ceil(math.log2(ext))
    ix = np.minimum(np.floor((x[:, 0] - x[:, 0].min()) * 2.0 ** (24 - e)), 2**24 - 1).astype(np.uint64)
    iy = np.minimum(np.floor((x[:, 1] - x[:, 1].min()) * 2.0 ** (24 - e)), 2**24 - 1).astype(np.uint64)
    code = np.zeros(500, dtype=np.uint64)
    for b in range(24):
        code |= ((ix >> np.uint64(b)) & np.uint64(1)) << np.uint64(2 * b)
        code |= ((iy >> np.uint64(b)) & np.uint64(1)) << np.uint64(2 * b + 1)
    assert np.array_equal(code, bh.codes)
    # every internal node's points share its prefix and it branches (>= 2 children)
    for depth, first, count, leaf, prefix in nodes:
        pts = c[first:first + count]
        if leaf and count == 1:
            continue
        sh = np.uint64(2 * (24 - depth))
        assert np.all((pts >> sh) == np.uint64(prefix))
        if not leaf:
            digits = set(((pts >> (sh - np.uint64(2))) & np.uint64(3)).tolist())
            assert len(digits) >= 2


def test_bh_opening_threshold_hand_worked(orc):
    """Three points A = (0, 0), B = (0.25, 0), T = (63, 0).  Box side 64 =
    2^6, so a quantum is 2^-18: A, B, T sit in cells (0, 0), (2^16, 0),
    (63 * 2^18, 0).  The tight cell of {A, B} is the aligned cell of side
    2^17 quanta (0.5) at the origin (side 2^16 would split them), centre
    (0.25, 0.25); T's quantum-cell centre is (63 + 2^-19, 2^-19).  T accepts
    {A, B} iff side < theta * distance of the two centres, i.e. iff
    theta > 2^18 / |(2 (63 * 2^18) + 1 - 2^17, 1 - 2^17)| = 0.0079680640...
    (distances to the centroid (0.125, 0) would put the threshold at
    0.5/62.875 = 0.0079523).  A and B open everything (they lie in the cell):
    4 exact pairs.  Accepted: F_T = 2 r(T - (0.125, 0)); opened: the two
    exact terms."""
    x = np.array([[0.0, 0.0], [0.25, 0.0], [63.0, 0.0]])
    th = 2.0 ** 18 / math.hypot(2 * 63 * 2 ** 18 + 1 - 2 ** 17, 1 - 2 ** 17)
    assert abs(th - 0.0079680640) < 1e-10
    for t, acc in [(th * (1 + 1e-7), 1), (th * (1 - 1e-7), 0), (0.5 / 62.875 * (1 + 5e-4), 0)]:
        bh = orc.barnes_hut(x, t)
        assert (bh.accepted, bh.leaf_pairs) == (acc, 6 - 2 * acc)
        assert bh.nodes[1].tolist()[:3] == [7, 0, 2]  # depth 24 - 17, first, count
        if acc:
            assert abs(bh.F[2, 0] - 2 / 62.875) < 1e-15 and bh.F[2, 1] == 0.0
        else:
            assert abs(bh.F[2, 0] - (1 / 63.0 + 1 / 62.75)) < 1e-15


@pytest.mark.parametrize("theta", [0.5, 1.0])
def test_bh_error_is_the_sum_of_cell_remainders(orc, theta):
    """Every target of a clustered instance: the exact field minus the
    Barnes-Hut field equals the sum over the cells the target accepts of
    (exact cell sum - m r(x_u - centroid)), computed here from the cell's
    points, so accepted cells act exactly through their centroids and all
    other points are summed exactly.  Each such remainder obeys the
    multipole bound: with w = x_u - c, delta_v = x_v - c in complex form,
    1/conj(w - delta) - 1/conj(w) - conj(delta)/conj(w)^2 =
    conj(delta)^2 / (conj(w)^2 conj(w - delta)), and the dipole terms cancel
    (sum of delta_v = 0), so |R| <= sum_v |delta_v|^2 / (|w|^2 |x_u - x_v|)."""
    x = _points(700, 4)
    bh = orc.barnes_hut(x, theta)
    S = orc.far_samples(x, theta)
    assert S.u.size == bh.accepted > 0
    F = orc.farfield_exact(x)
    acc = np.zeros_like(F)
    worst = 0.0
    for u, nd in zip(S.u, S.node):
        depth, first, count, leaf, _ = bh.nodes[nd]
        pts = x[bh.order[first:first + count]]
        assert not leaf or count > 1
        c = pts.mean(0)
        d = x[u] - pts
        w = x[u] - c
        R = (d / (d ** 2).sum(1)[:, None]).sum(0) - count * w / (w @ w)
        acc[u] += R
        delta2 = ((pts - c) ** 2).sum(1)
        bound = (delta2 / ((w @ w) * np.sqrt((d ** 2).sum(1)))).sum()
        # (R is a difference of sums of size count/|w|: allow its rounding)
        assert np.hypot(*R) <= bound * (1 + 1e-9) + 1e-13 * count / np.sqrt(w @ w)
        worst = max(worst, np.hypot(*R) / bound)
    scale = np.maximum(np.linalg.norm(F, axis=1), np.linalg.norm(F, axis=1).mean())
    assert np.max(np.linalg.norm(F - bh.F - acc, axis=1) / scale) < 1e-11
    assert worst > 0.05  # the bound is not vacuous


# ------------------------------------------------------------- Eq. 2 (P1-P6)

def test_sweep_subtraction_equals_direct_sum(orc):
    """Eq. 2's entropy term over v not in S(u), summed directly, equals the far
    field over all v != u minus the sum over S(u) (Eq. 3's last term)."""
    g = synth.grid(8, 8)
    x = orc.init_layout(g.n, 11, 0) * 8
    for k in (1, 2, 3):
        kh = orc.khop_build(g.row_ptr, g.col, k)
        a, _ = orc.sweep(kh, x, orc.farfield_exact(x), 0.37)
        b, _ = orc.sweep_direct(kh, x, 0.37)
        assert rel(a, b) < 1e-12


@pytest.mark.parametrize("L0", [0.3, 1.7, 2.9, 5.0])
def test_two_vertices_closed_form(orc, L0):
    """One edge, S = E, no entropy pairs: Jacobi gives L' = |2d - L|; L = d is
    the fixed point, the optimal distance of the initial layout (Section 3.1)."""
    g = synth.path(2)
    kh = orc.khop_build(g.row_ptr, g.col, 1)
    ang = 0.7
    x = np.array([[1.0, 2.0], [1.0 + L0 * math.cos(ang), 2.0 + L0 * math.sin(ang)]])
    F = orc.farfield_exact(x)
    for level, c, d in [(0, None, 1.0), (1, np.array([4, 9], np.int32), 5.0)]:
        xn, _ = orc.sweep(kh, x, F, 0.5, level=level, c=c)
        assert abs(np.linalg.norm(xn[1] - xn[0]) - abs(2 * d - L0)) < 1e-12
        xf = np.array([[0.0, 0.0], [d * math.cos(ang), d * math.sin(ang)]])
        xn, delta = orc.sweep(kh, xf, orc.farfield_exact(xf), 0.5, level=level, c=c)
        assert np.max(np.abs(xn - xf)) < 1e-12


@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_path_isometry_is_fixed_point(orc, k):
    """With alpha = 0 and d = hop, a collinear unit-spaced path has zero stress
    for every k and is a fixed point of Eq. 2."""
    g = synth.path(12)
    kh = orc.khop_build(g.row_ptr, g.col, k)
    x = np.stack([np.arange(12.0), np.zeros(12)], 1) * 1.0 + np.array([3.0, -2.0])
    xn, delta = orc.sweep(kh, x, np.zeros_like(x), 0.0)
    # exact up to the rounding of w = 1/hop^2 in the weighted mean
    assert np.max(np.abs(xn - x)) < 1e-13 and delta < 1e-14
    assert orc.objective(kh, x, 0.0)["stress"] == 0.0


def test_grid_converges_to_isometry_as_alpha_vanishes(orc):
    """Grid, S = E: as alpha -> 0 the layout approaches the isometric grid
    (edge lengths 1, sparse stress ~ 0)."""
    g = synth.grid(10, 10)
    p = orc.Params(k=1, theta=-1, alpha_decay=0.3, alpha_min=1e-6, max_final_iters=20000,
                   eps_final=1e-10, max_levels=0)
    x, st = orc.layout(g, p)
    src, dst = g.edges()
    L = np.linalg.norm(x[src] - x[dst], axis=1)
    assert np.max(np.abs(L - 1)) < 2e-3
    kh = orc.khop_build(g.row_ptr, g.col, 1)
    assert orc.objective(kh, x, 0)["stress"] < 1e-4


def test_exact_below_selects_the_exact_far_field(orc):
    """exact_below >= n on every level reproduces the exact-far-field layout
    (theta < 0) bit for bit; exact_below = 0 is plain Barnes-Hut, which at
    theta = 0.5 moves the result."""
    g = synth.grid(16, 16)
    kw = dict(k=2, alpha_decay=0.5, coarsest_n=10, max_final_iters=30)
    xe, _ = orc.layout(g, orc.Params(theta=-1, **kw))
    xa, _ = orc.layout(g, orc.Params(theta=0.5, exact_below=g.n, **kw))
    xb, _ = orc.layout(g, orc.Params(theta=0.5, **kw))
    assert np.array_equal(xe, xa)
    assert not np.array_equal(xe, xb)


def test_translation_rotation_invariance(orc):
    g = synth.grid(7, 6)
    kh = orc.khop_build(g.row_ptr, g.col, 2)
    x = orc.init_layout(g.n, 5, 0) * 6
    T = lambda y: orc.sweep(kh, y, orc.farfield_exact(y), 0.25)[0]
    base = T(x)
    t = np.array([13.5, -7.25])
    assert np.max(np.abs(T(x + t) - (base + t))) < 1e-12 * 20
    th = 0.83
    R = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    assert np.max(np.abs(T(x @ R.T) - base @ R.T)) < 1e-12 * 20


def _fd_grad(orc, kh, x, alpha, h=1e-6, q=0.0):
    g = np.zeros_like(x)
    for i in range(x.shape[0]):
        for j in range(2):
            xp = x.copy(); xp[i, j] += h
            xm = x.copy(); xm[i, j] -= h
            g[i, j] = (orc.objective(kh, xp, alpha, q)["M"] -
                       orc.objective(kh, xm, alpha, q)["M"]) / (2 * h)
    return g


@pytest.mark.parametrize("k,q", [(1, 0.0), (2, 0.0), (2, 1.0), (1, 0.5)])
def test_update_is_gradient_step_of_objective(orc, k, q):
    """Eq. 1 vs Eq. 2: grad_u M_{2 alpha}(x) = 2 rho_u (x_u - T_alpha(x)_u) at any
    layout, for the logarithmic entropy (q = 0) and the power entropies
    E_q = -D^-q / q of the general model (their gradient is r_q); the update
    and the objective are independent code paths."""
    g = synth.grid(4, 5)
    kh = orc.khop_build(g.row_ptr, g.col, k)
    x = orc.init_layout(g.n, 9, 0) * 4
    alpha = 0.2
    Tx, _ = orc.sweep(kh, x, orc.farfield_exact(x, q), alpha, q)
    rho = np.array([np.sum(1.0 / kh.hops(u).astype(float) ** 2) for u in range(g.n)])
    grad = 2 * rho[:, None] * (x - Tx)
    fd = _fd_grad(orc, kh, x, 2 * alpha, q=q)
    assert np.max(np.abs(grad)) > 1.0
    assert np.max(np.abs(fd - grad)) < 1e-5 * np.max(np.abs(grad))


def test_fixed_point_is_stationary(orc):
    """A converged fixed point of T_alpha is a stationary point of M at 2 alpha."""
    g = synth.grid(5, 5)
    kh = orc.khop_build(g.row_ptr, g.col, 2)
    x = orc.init_layout(g.n, 3, 0) * 4
    for _ in range(20000):
        x, d = orc.sweep(kh, x, orc.farfield_exact(x), 0.3)
        if d < 1e-14:
            break
    assert d < 1e-13
    fd = _fd_grad(orc, kh, x, 0.6)
    assert np.max(np.abs(fd)) < 1e-6


# --------------------------------------------------- objectives (P11)

def test_objectives_hand_computed(orc):
    """Eq. 1 and the full stress measure (Section 4) on hand-worked layouts."""
    g = synth.path(3)
    x = np.array([[0.0, 0.0], [1.0, 0.0], [3.0, 0.0]])
    kh = orc.khop_build(g.row_ptr, g.col, 1)
    o = orc.objective(kh, x, 0.008)
    assert abs(o["stress"] - 1.0) < 1e-15 and abs(o["ent"] - math.log(3)) < 1e-15
    assert abs(o["M"] - (1 - 0.008 * math.log(3))) < 1e-15
    fs = orc.full_stress(g.row_ptr, g.col, x)
    assert abs(fs["F_unscaled"] - 1.25) < 1e-15
    # optimal scale: closed form vs a numeric 1-D minimiser
    pairs = [(1.0, 1.0), (2.0, 1.0), (3.0, 2.0)]  # (D, d)
    f = lambda s: sum((s * D - d) ** 2 / d**2 for D, d in pairs)
    res = minimize_scalar(f, bracket=(0.1, 2.0), tol=1e-14)
    assert abs(fs["s_opt"] - res.x) < 1e-7
    assert abs(fs["F"] - f(res.x)) < 1e-12
    # 4-cycle on the unit square: edges exact, the two diagonals are entropy pairs
    g = synth.cycle(4)
    x = np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 1.0], [0.0, 1.0]])
    kh = orc.khop_build(g.row_ptr, g.col, 1)
    o = orc.objective(kh, x, 0.5)
    assert abs(o["stress"]) < 1e-15 and abs(o["ent"] - math.log(2)) < 1e-15
    fs = orc.full_stress(g.row_ptr, g.col, x)
    assert abs(fs["F_unscaled"] - 2 * (math.sqrt(2) - 2) ** 2 / 4) < 1e-15


# ------------------------------------------------ coarsening (P8)

def test_lp_hand_worked_path(orc):
    """Path 0-1-2-3, U = 2, seed 1, level 1.  Round-0 colours (SplitMix64,
    pinned above) are [1,0,1,0]: sub-round 0 moves 1 -> label 0 (tie between
    labels 0 and 2 goes to the smaller) and 3 -> label 2; nothing else is
    feasible or better afterwards."""
    assert [int(v) & 1 for v in orc.draws(1, 1, 16, 0, 4)] == [1, 0, 1, 0]
    g = synth.path(4)
    lab, moves = orc.lp(g.row_ptr, g.col, 2.0, 10, 1, 1)
    assert lab.tolist() == [0, 0, 2, 2] and moves.tolist() == [2, 0]
    cl, Gc = orc.contract(orc.Level(g.row_ptr, g.col), lab)
    assert cl.tolist() == [0, 0, 1, 1]
    assert Gc.row_ptr.tolist() == [0, 1, 2] and Gc.col.tolist() == [1, 0]
    assert Gc.c.tolist() == [2, 2] and Gc.w.tolist() == [1, 1]


def test_lp_hand_worked_two_triangles(orc):
    """Triangles {0,1,2}, {3,4,5} joined by 2-3, U = 3, seed 1.  Worked by hand:
    r0/s0 (active 1,3): 1->0, 3->2; r0/s1 (active 0,2,4,5): 2->0 (score 2),
    4 and 5 both propose label 2 but only 4 fits (admission in ascending v);
    r1/s0: 5->2; then no moves."""
    g = synth.two_triangles()
    lab, moves = orc.lp(g.row_ptr, g.col, 3.0, 10, 1, 1)
    assert lab.tolist() == [0, 0, 0, 2, 2, 2] and moves.tolist() == [4, 1, 0]
    cl, Gc = orc.contract(orc.Level(g.row_ptr, g.col), lab)
    assert Gc.n == 2 and Gc.c.tolist() == [3, 3] and Gc.w.tolist() == [1, 1]


@pytest.mark.parametrize("gname", ["rgg", "tree", "grid"])
def test_lp_contraction_invariants(orc, gname):
    g = {"rgg": lambda: synth.rgg(3000, 4), "tree": lambda: synth.random_tree(3000, 4),
         "grid": lambda: synth.grid(40, 40)}[gname]()
    lv = orc.Level(g.row_ptr, g.col)
    for h in range(1, 5):
        cw = np.ones(lv.n, np.int64) if lv.c is None else lv.c.astype(np.int64)
        U = max(float(cw.max()), 2.0**h)
        lab, _ = orc.lp(lv.row_ptr, lv.col, U, 10, 3, h, lv.c, lv.w)
        W = np.bincount(lab, weights=cw, minlength=lv.n)
        assert W.max() <= U
        cl, Gc = orc.contract(lv, lab)
        assert Gc.c.sum() == cw.sum()
        ew = np.ones(lv.col.size, np.int64) if lv.w is None else lv.w.astype(np.int64)
        src = np.repeat(np.arange(lv.n), np.diff(lv.row_ptr))
        intra = ew[cl[src] == cl[lv.col]].sum()
        assert Gc.w.sum() == ew.sum() - intra
        assert orc.validate(Gc.row_ptr, Gc.col, Gc.c, Gc.w) == 0
        lv = Gc


# --------------------------------------------------- prolongation (P9)

def test_prolongation_within_radius(orc):
    """Uncoarsening (Section 3.2): fine vertices land within sqrt(c(v')) of
    their representative; angle and radius fractions are uniform."""
    from scipy.stats import kstest
    n = 20000
    cluster = (np.arange(n) % 1000).astype(np.int32)
    cc = (np.arange(1000) % 17 + 1).astype(np.int32)
    cx = orc.init_layout(1000, 2, 1) * 50
    fx = orc.prolong(cluster, cc, cx, 4, 0)
    off = fx - cx[cluster]
    r = np.linalg.norm(off, axis=1)
    assert np.all(r <= np.sqrt(cc[cluster]) * (1 + 1e-14))
    assert kstest(r / np.sqrt(cc[cluster]), "uniform").pvalue > 1e-3
    ang = (np.arctan2(off[:, 1], off[:, 0]) + 2 * np.pi) % (2 * np.pi) / (2 * np.pi)
    assert kstest(ang, "uniform").pvalue > 1e-3


# ------------------------------------------------ end to end (P12, P13)

def test_btree_maxent_stress_in_paper_band(orc):
    """Weak: the complete binary tree (n = 1023) with the paper's configuration
    (S = E, decay 0.3, f = 20, b = 2), exact entropy term (MulMent_0).  After the
    optimal scaling used for the paper's comparisons, M(x) at alpha = 0.008 lies
    in the range the paper prints for this graph (Table 3: PMDS -7231,
    MulMent_0 -9128, GHN -9688), with 5% slack."""
    ref = json.load(open(os.path.join(GOLDEN, "paper_values.json")))["btree"]
    g = synth.complete_binary_tree(9)
    assert (g.n, g.m) == (ref["n"], ref["m"])
    p = orc.Params(k=1, theta=-1, alpha_decay=0.3, max_final_iters=5000)
    x, _ = orc.layout(g, p)
    s = orc.full_stress(g.row_ptr, g.col, x)["s_opt"]
    kh = orc.khop_build(g.row_ptr, g.col, 1)
    M = orc.objective(kh, x * s, 0.008)["M"]
    assert ref["M_GHN"] * 1.05 <= M <= ref["M_PMDS"] * 0.95, M


def test_thread_count_independence(orc, tmp_path):
    """The result does not depend on the number of threads (Section 4.1)."""
    code = (
        "import sys, numpy as np; sys.path.insert(0, %r); import synth, oracle;"
        "g = synth.rgg(1500, 2);"
        "p = oracle.Params(k=2, theta=0.5, alpha_decay=0.5, max_final_iters=30, coarsest_n=50);"
        "x, _ = oracle.layout(g, p); np.save(sys.argv[1], x)"
    ) % os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    outs = []
    for t in (1, 3):
        f = str(tmp_path / f"x{t}.npy")
        env = dict(os.environ, OMP_NUM_THREADS=str(t))
        subprocess.run([sys.executable, "-c", code, f], check=True, env=env)
        outs.append(np.load(f))
    assert np.array_equal(outs[0], outs[1])


# ------------------------------------------------- hierarchy driver (P8)

def _attempts(trace):
    return [(t["h"], round(t["f"], 9), round(t["W"], 9), round(t["U"], 9), t["n"], t["fired"],
             t["redo"], round(t.get("f_next", t["f"]), 9)) for t in trace]


def test_hierarchy_rules_on_a_matching(orc):
    """Ten disjoint edges (0-1, 2-3, ..., 18-19), unit weights, |V| = 20,
    b = 2, f = 20, seed 1 (Section 3.1).  Worked by hand:
    h = 1 (first contraction): W = min(2, 20/20) = 1, U = max(1, W) = 1: no
    vertex fits next to another (1 + 1 > 1), n stays 20 > 0.9 * 20, the rule
    fires; W was bounded by |V|/f (1 < 2), so f := 14 and the level is
    rebuilt: W = min(2, 20/14) = 1.43 = U, still nothing fits, f := 9.8,
    rebuilt: W = min(2, 20/9.8 = 2.04) = 2 = U.  Now a pair merges in the
    first round its endpoints draw different colours (the first active
    endpoint joins the other's label; equal colours swap the labels); with
    seed 1 every pair has differing colours by round 3 (bits below), so
    n = 10 <= 18: level 1 is kept (two rebuilds).
    h = 2: ten isolated vertices of weight 2.  W = min(4, 20/9.8) = 2.04 (|V|
    is the total weight 20, not the 10 vertices), U = max(2, W) = 2.04; no
    edges, n stays 10, fires, bounded (2.04 < 4): f := 6.86, rebuild
    (W = U = 20/6.86 = 2.92), fires, bounded: f := 4.802, rebuild:
    W = min(4, 4.16) = 4 = U, fires, not bounded by |V|/f (4.16 >= 4): f :=
    3.3614 without a rebuild; no progress, coarsening stops."""
    n = 20
    g = synth.csr_from_edges(n, np.arange(0, n, 2), np.arange(1, n, 2))
    bits = [[int(b) & 1 for b in orc.draws(1, 1, 16 + r, 0, n)] for r in range(4)]
    first_diff = [min(r for r in range(4) if bits[r][2 * i] != bits[r][2 * i + 1])
                  for i in range(10)]
    assert first_diff == [0, 0, 3, 0, 3, 1, 0, 2, 0, 0]
    tr = []
    levels, clusters, info = orc.hierarchy(orc.Level(g.row_ptr, g.col), orc.Params(seed=1), tr)
    assert [lv.n for lv in levels] == [20, 10]
    assert clusters[0].tolist() == [i // 2 for i in range(n)]
    assert levels[1].c.tolist() == [2] * 10 and levels[1].col.size == 0
    assert _attempts(tr) == [
        (1, 20.0, 1.0, 1.0, 20, True, 0, 14.0),
        (1, 14.0, round(20 / 14, 9), round(20 / 14, 9), 20, True, 1, 9.8),
        (1, 9.8, 2.0, 2.0, 10, False, 2, 9.8),
        (2, 9.8, round(20 / 9.8, 9), round(20 / 9.8, 9), 10, True, 0, 6.86),
        (2, 6.86, round(20 / 6.86, 9), round(20 / 6.86, 9), 10, True, 1, 4.802),
        (2, 4.802, 4.0, 4.0, 10, True, 2, 3.3614)]
    assert info == [{"h": 1, "U": 2.0, "n": 10, "lp_rounds": 5, "redo": 2}]


def test_hierarchy_rule_fires_without_rebuild_and_keeps_the_level(orc):
    """Star with centre 0 and 29 leaves, |V| = 30, seed 1, stop at <= 29
    vertices.  h = 1: W = min(2, 30/20 = 1.5) = U: nothing fits, fires,
    bounded (1.5 < 2): f := 14, rebuild: W = min(2, 30/14 = 2.14) = 2 = U.
    Round 0, colour 0: the centre (bit 1) waits, the active leaves all
    propose the centre's label and admission in ascending id takes leaf 1
    only (1 + 1 <= 2); colour 1: the centre's best label is its own (tie);
    round 1 moves nothing.  n = 29 > 0.9 * 30: fires, but W was not bounded
    by |V|/f (2.14 >= 2), so f := 9.8 with no rebuild, and the level is kept
    (progress); 29 vertices end the coarsening."""
    g = synth.star(29)
    b0 = [int(b) & 1 for b in orc.draws(1, 1, 16, 0, 30)]
    assert b0[0] == 1 and b0[1] == 0
    tr = []
    levels, clusters, info = orc.hierarchy(orc.Level(g.row_ptr, g.col),
                                           orc.Params(seed=1, coarsest_n=29), tr)
    assert [lv.n for lv in levels] == [30, 29]
    assert clusters[0].tolist() == [0, 0] + list(range(1, 29))
    assert levels[1].c.tolist() == [2] + [1] * 28
    assert _attempts(tr) == [(1, 20.0, 1.5, 1.5, 30, True, 0, 14.0),
                             (1, 14.0, 2.0, 2.0, 29, True, 1, 9.8)]
    assert info == [{"h": 1, "U": 2.0, "n": 29, "lp_rounds": 2, "redo": 1}]


def test_hierarchy_rebuild_limit(orc):
    """Five isolated vertices, b = 1e6 so W = |V|/f always: every attempt
    fires and is rebuilt with f := 0.7 f (U = max(1, W) = 1 while W < 1)
    until the tenth rebuild; the eleventh attempt fires without a rebuild
    and, with no progress, ends the coarsening at the input graph."""
    rp = np.zeros(6, np.int32)
    tr = []
    levels, _, info = orc.hierarchy(orc.Level(rp, np.zeros(0, np.int32)),
                                    orc.Params(seed=1, b=1e6), tr)
    assert [lv.n for lv in levels] == [5] and info == []
    f = 20.0
    exp = []
    for r in range(11):
        W = 5 / f
        exp.append((1, round(f, 9), round(W, 9), round(max(1.0, W), 9), 5, True, r,
                    round(0.7 * f, 9)))
        f *= 0.7
    assert _attempts(tr) == exp
