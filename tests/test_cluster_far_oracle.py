"""Pins of the oracle's cluster far field (the first two sums of Eq. 3,
Section 3.2) against facts the paper and the mathematics fix.

* With the identity as both cluster maps, Eq. 3 is the exact sum (the paper
  notes this for M = identity).
* When every cluster's members coincide, a representative carrying nu_j at
  their common point reproduces the exact sum term by term.
* For an approximation level h > 1 beneath, vertices that share u's
  representative there but not u's own cluster one level down are left out
  (the merged-vertex error of Section 3.2); a hand-built case gives the
  missing amount in closed form.
* The representative sits at the node-weighted midpoint (a hand-worked case
  with weights 1 and 3).
"""
import math

import numpy as np
import pytest

import synth


def _pts(n, seed):
    return np.random.default_rng(seed).random((n, 2)) * 10.0


@pytest.mark.parametrize("q", [0.0, 1.0])
def test_identity_maps_give_the_exact_sum(orc, q):
    x = _pts(300, 1)
    ident = np.arange(300, dtype=np.int32)
    F = orc.cluster_far_field(x, None, ident, 300, ident, 300, q)
    Fe = orc.farfield_exact(x, q)
    assert np.allclose(F, Fe, rtol=1e-12, atol=1e-12)


def test_coincident_clusters_are_exact(orc):
    rng = np.random.default_rng(2)
    k = 40
    centre = rng.random((k, 2)) * 10.0
    cl = rng.integers(0, k, 400).astype(np.int32)
    cl[:k] = np.arange(k)  # every cluster non-empty
    x = centre[cl]
    F = orc.cluster_far_field(x, None, cl, k, cl, k)
    Fe = orc.farfield_exact(x)
    assert np.allclose(F, Fe, rtol=1e-12, atol=1e-12)


def test_merged_vertices_are_left_out(orc):
    """Level l: u's cluster A (3 vertices at p1) and cluster B (2 vertices at
    p2) share one representative two levels down; every other cluster is
    coincident and has its own representative.  Eq. 3 misses exactly the
    B-terms: F = F_exact - 2 r(p1 - p2) for u in A."""
    p1, p2 = np.array([1.0, 2.0]), np.array([1.5, 2.7])
    others = np.array([[8.0, 1.0], [3.0, 9.0], [7.5, 7.5]])
    x = np.vstack([np.repeat(p1[None], 3, 0), np.repeat(p2[None], 2, 0),
                   np.repeat(others, 2, 0)])
    cl1 = np.array([0, 0, 0, 1, 1, 2, 2, 3, 3, 4, 4], np.int32)
    clh = np.array([0, 0, 0, 0, 0, 1, 1, 2, 2, 3, 3], np.int32)
    F = orc.cluster_far_field(x, None, cl1, 5, clh, 4)
    Fe = orc.farfield_exact(x)
    d = p1 - p2
    miss = 2.0 * d / (d @ d)
    for u in range(3):
        assert np.allclose(F[u], Fe[u] - miss, rtol=1e-12, atol=1e-12)
    # the B vertices miss the three A vertices the same way
    for u in (3, 4):
        assert np.allclose(F[u], Fe[u] + 3.0 * d / (d @ d), rtol=1e-12, atol=1e-12)


def test_representative_is_the_weighted_midpoint(orc):
    a, b, u = np.array([0.0, 0.0]), np.array([4.0, 0.0]), np.array([3.0, 5.0])
    x = np.array([a, b, u])
    c = np.array([1, 3, 1], np.int32)
    cl = np.array([0, 0, 1], np.int32)
    F = orc.cluster_far_field(x, c, cl, 2, cl, 2)
    mid = (1.0 * a + 3.0 * b) / 4.0  # (3, 0)
    d = u - mid
    assert np.allclose(F[2], 2.0 * d / (d @ d), rtol=1e-14)
    # a and b: exact term of the other member plus u's representative
    for i, o in ((0, 1), (1, 0)):
        dd = x[i] - x[o]
        e = x[i] - u
        assert np.allclose(F[i], dd / (dd @ dd) + e / (e @ e), rtol=1e-14)


def test_out_of_range_cluster_rejected(orc):
    x = _pts(5, 3)
    bad = np.array([0, 1, 2, 3, 9], np.int32)
    with pytest.raises(ValueError):
        orc.cluster_far_field(x, None, bad, 5, bad, 5)


def test_mulment_h_layout_close_to_exact(orc):
    """MulMent_1 on a 16x16 grid (k = 2): final maxent-stress within 5% of
    the layout with the exact far field (the approximation trades a little
    quality, Section 4)."""
    g = synth.grid(16, 16)
    kw = dict(k=2, alpha_decay=0.5, coarsest_n=10, max_final_iters=60)
    xe, _ = orc.layout(g, orc.Params(theta=-1, **kw))
    xa, st = orc.layout(g, orc.Params(theta=-1, approx_h=1, **kw))
    kh = orc.khop_build(g.row_ptr, g.col, 2)
    Me, Ma = orc.objective(kh, xe, 0.008)["M"], orc.objective(kh, xa, 0.008)["M"]
    assert not np.array_equal(xe, xa)
    assert abs(Ma - Me) <= 0.05 * abs(Me), (Ma, Me)


def test_update_protocol_cuts_the_hierarchy(orc):
    """Sec. 4.3 update algorithm: a warm start refines the finest level at
    alpha_min only; with approx_h = h the coarsening stops after h levels and
    the last of them gives the representatives.  On an unchanged graph the
    update continues the optimisation at alpha_min, so the maxent-stress does
    not rise."""
    g = synth.grid(16, 16)
    kw = dict(k=2, alpha_decay=0.5, coarsest_n=4, max_final_iters=40)
    x0, _ = orc.layout(g, orc.Params(theta=-1, approx_h=2, **kw))
    x1, st = orc.layout(g, orc.Params(theta=-1, approx_h=2, **kw), init_xy=x0)
    assert len(st["hierarchy"]) == 2 and len(st["levels"]) == 1
    x2, st2 = orc.layout(g, orc.Params(theta=-1, **kw), init_xy=x0)
    assert len(st2["hierarchy"]) == 0
    assert not np.array_equal(x1, x2)  # Eq. 3 vs the exact far field
    kh = orc.khop_build(g.row_ptr, g.col, 2)
    m0, m1 = orc.objective(kh, x0, 0.008)["M"], orc.objective(kh, x1, 0.008)["M"]
    assert m1 <= m0, (m0, m1)
