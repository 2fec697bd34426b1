"""General stress sets S ⊇ E (footnote to Eq. 1) without a GPU: the oracle's
Eq. 2 and Eq. 1 on sets that are not k-hop balls, pinned by the gradient
identity and the direct entropy sum; the library's host-side validation
of imported sets (mm_khop_validate) on valid and malformed arrays."""
import numpy as np
import pytest

import general_sets as gs
import synth


def _valid_path3():
    # path 0-1-2, k = 2: row 0 = [1 | 2], row 1 = [0, 2 | ], row 2 = [1 | 0]
    off = np.array([0, 2, 4, 6], np.int64)
    hend = np.array([1, 2, 2, 2, 1, 2], np.int32)
    nbr = np.array([1, 2, 0, 2, 1, 0], np.int32)
    return off, hend, nbr


def test_brute_force_khop_ball_equals_oracle_khop(orc):
    """The helper's layout of a full k-hop ball is the oracle's k-hop set."""
    g = synth.rgg(600, 4)
    D = gs.hop_matrix(g)
    iu, ju = np.nonzero((D >= 1) & (D <= 3))
    off, hend, nbr = gs.to_arrays(g.n, 3, iu, ju, D[iu, ju].astype(np.int64))
    ref = orc.khop_build(g.row_ptr, g.col, 3)
    assert np.array_equal(off, ref.off) and np.array_equal(hend, ref.hend)
    assert np.array_equal(nbr, ref.nbr)


@pytest.mark.parametrize("k,q", [(2, 0.0), (3, 0.0), (3, 1.0)])
def test_update_is_gradient_step_on_general_set(orc, k, q):
    """grad_u M_{2 alpha}(x) = 2 rho_u (x_u - T_alpha(x)_u) holds for any
    symmetric S with its own target distances, here E plus a random half of
    the pairs within k hops (a set no k-hop ball equals)."""
    g = synth.grid(4, 5)
    off, hend, nbr = gs.sampled(g, k, 0.5, seed=3)
    kh = orc.KHop(k, off, hend, nbr)
    ball = orc.khop_build(g.row_ptr, g.col, k)
    assert 0 < kh.nbr.size < ball.nbr.size
    x = orc.init_layout(g.n, 9, 0) * 4
    alpha = 0.2
    Tx, _ = orc.sweep(kh, x, orc.farfield_exact(x, q), alpha, q)
    rho = np.array([np.sum(1.0 / kh.hops(u).astype(float) ** 2) for u in range(g.n)])
    grad = 2 * rho[:, None] * (x - Tx)
    h = 1e-6
    fd = np.zeros_like(x)
    for i in range(g.n):
        for j in range(2):
            xp = x.copy(); xp[i, j] += h
            xm = x.copy(); xm[i, j] -= h
            fd[i, j] = (orc.objective(kh, xp, 2 * alpha, q)["M"] -
                        orc.objective(kh, xm, 2 * alpha, q)["M"]) / (2 * h)
    assert np.max(np.abs(grad)) > 1.0
    assert np.max(np.abs(fd - grad)) < 1e-5 * np.max(np.abs(grad))


def test_subtraction_equals_direct_sum_on_thresholded_set(orc):
    """Eq. 2's entropy term over v not in S(u): far field minus the S(u) part
    equals the direct sum, for a distance-thresholded S."""
    g = synth.rgg(300, 5)
    x = orc.init_layout(g.n, 4, 0) * 10
    off, hend, nbr = gs.thresholded(g, x, 3, 2.5)
    kh = orc.KHop(3, off, hend, nbr)
    a, _ = orc.sweep(kh, x, orc.farfield_exact(x), 0.37)
    b, _ = orc.sweep_direct(kh, x, 0.37)
    assert np.max(np.abs(a - b)) / np.max(np.abs(b)) < 1e-12


def test_validate_accepts_general_sets():
    import paper_1506_04383_amd as mm

    mm.khop_validate(3, 2, *_valid_path3())
    g = synth.rgg(500, 2)
    mm.khop_validate(g.n, 3, *gs.thresholded(g, g.points, 3, 0.08))
    mm.khop_validate(g.n, 2, *gs.sampled(g, 2, 0.3, seed=1))


def test_validate_rejects_empty_row():
    """A row with no entries has rho_u = 0, the divisor of Eq. 2 (vertex 2 of
    a 3-vertex set holding only the pair (0, 1))."""
    import paper_1506_04383_amd as mm

    with pytest.raises(mm.MulmentError, match="row 2 is empty") as e:
        mm.khop_validate(3, 1, np.array([0, 1, 2, 2]), np.array([1, 1, 0]), np.array([1, 0]))
    assert e.value.status == 1  # MM_EINVAL


def _corrupt(which):
    off, hend, nbr = (a.copy() for a in _valid_path3())
    if which == "off0":
        off[0] = 1
    elif which == "offdec":
        off[2] = 1
    elif which == "hend_dec":
        hend[0:2] = [2, 1]
    elif which == "hend_end":
        hend[1] = 1
    elif which == "range":
        nbr[1] = 3
    elif which == "negative":
        nbr[1] = -1
    elif which == "self":
        nbr[1] = 0
    elif which == "order":
        nbr[2:4] = [2, 0]
    elif which == "twice":
        nbr[1] = 1
    elif which == "mirror":
        hend[0:2] = [2, 2]  # row 0 puts 2 at distance 1, row 2 puts 0 at distance 2
    return off, hend, nbr


@pytest.mark.parametrize("which,msg", [
    ("off0", "off[0]"), ("offdec", "decreases"), ("hend_dec", "decreases"),
    ("hend_end", "ends at"), ("range", "out of range"), ("negative", "out of range"),
    ("self", "holds itself"), ("order", "strictly increasing"), ("twice", "twice"),
    ("mirror", "no mirror")])
def test_validate_rejects_malformed_sets(which, msg):
    import paper_1506_04383_amd as mm

    with pytest.raises(mm.MulmentError) as e:
        mm.khop_validate(3, 2, *_corrupt(which))
    assert msg in str(e.value)
    assert e.value.status == 1  # MM_EINVAL


def test_validate_rejects_bad_sizes():
    import paper_1506_04383_amd as mm

    with pytest.raises(mm.MulmentError, match="k must be"):
        mm.khop_validate(3, 9, np.zeros(4, np.int64), np.zeros(27, np.int32), np.zeros(0))
    with pytest.raises(mm.MulmentError, match="n < 2"):
        mm.khop_validate(1, 1, np.zeros(2, np.int64), np.zeros(1, np.int32), np.zeros(0))
    with pytest.raises(ValueError):
        mm.khop_validate(3, 2, np.zeros(3, np.int64), np.zeros(6, np.int32), np.zeros(0))
