"""FP64 CPU oracle of multilevel maxent-stress layout.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package; the GPU library never
calls it and shares no code with it.  The heavy loops live in mm_oracle.c
(plain C, FP64); this module marshals numpy arrays and restates the
multilevel driver of the paper's Section 3:

* hierarchy (Section 3.1): size-constrained label propagation with
  U = max(max_v c(v), W), W = min(b^h, |V|/f), contraction, and the rule
  "contracted graph not 10% smaller -> f := 0.7 f";
* initial layout and prolongation (Sections 3.1, 3.2);
* local improvement (Section 3.2): Jacobi iterations of Eq. 2 with
  target distances sqrt(c_u)+sqrt(c_v) on coarse levels, the alpha schedule
  alpha := decay*alpha down to alpha_min with at most `a` iterations per
  round, an early alpha drop when the relative change is below epsilon, and
  iteration at alpha_min until the relative change is below eps_final.

Readings of points the paper leaves open are listed in the repository's
design notes and restated in the docstrings below.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from dataclasses import dataclass, field, replace

import numpy as np

from .build import LIB, build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            _build()
        L = C.CDLL(LIB)
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C")
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C")
        u64p = np.ctypeslib.ndpointer(np.uint64, flags="C")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C")
        vp = C.c_void_p
        L.orc_set_threads.restype = C.c_int
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_splitmix64_at.restype = C.c_uint64
        L.orc_splitmix64_at.argtypes = [C.c_uint64, C.c_uint64]
        L.orc_draws.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint64, C.c_int64, u64p]
        L.orc_validate.argtypes = [C.c_int32, i32p, i32p, vp, vp]
        L.orc_khop_build.argtypes = [C.c_int32, i32p, i32p, C.c_int32, i64p, vp, vp]
        L.orc_farfield_exact.argtypes = [C.c_int32, f64p, C.c_double, f64p]
        L.orc_cluster_far.argtypes = [C.c_int32, f64p, vp, i32p, C.c_int32, i32p, C.c_int32,
                                      C.c_double, f64p]
        L.orc_bh.argtypes = [C.c_int32, f64p, C.c_double, C.c_double, f64p, vp, vp, vp,
                             C.c_int64, i64p]
        L.orc_sweep.argtypes = [C.c_int32, C.c_int32, C.c_int32, i64p, i32p, i32p, vp,
                                C.c_double, f64p, f64p, C.c_double, C.c_double, f64p, f64p]
        L.orc_sweep_direct.argtypes = [C.c_int32, C.c_int32, C.c_int32, i64p, i32p, i32p, vp,
                                       C.c_double, f64p, C.c_double, C.c_double, f64p, f64p]
        L.orc_sweep_rows.argtypes = [C.c_int32, i32p, i32p, C.c_int32, C.c_int32, vp,
                                     C.c_double, f64p, f64p, C.c_double, C.c_double, i32p,
                                     C.c_int32, f64p, i64p]
        L.orc_lp.argtypes = [C.c_int32, i32p, i32p, vp, vp, C.c_double, C.c_int32,
                             C.c_uint64, C.c_int32, i32p, i32p]
        L.orc_contract.restype = C.c_int32
        L.orc_contract.argtypes = [C.c_int32, i32p, i32p, vp, vp, i32p, i32p, i32p, i32p,
                                   i32p, i32p, i64p]
        L.orc_init_layout.argtypes = [C.c_int32, C.c_uint64, C.c_int32, f64p]
        L.orc_prolong.argtypes = [C.c_int32, i32p, vp, f64p, C.c_uint64, C.c_int32, f64p]
        L.orc_objective.argtypes = [C.c_int32, C.c_int32, C.c_int32, i64p, i32p, i32p, vp,
                                    C.c_double, f64p, C.c_double, f64p]
        L.orc_full_stress.argtypes = [C.c_int32, i32p, i32p, f64p, f64p]
        L.orc_far_samples.argtypes = [C.c_int32, f64p, C.c_double, C.c_int64, i32p, i64p, f64p,
                                      f64p, f64p, i64p]
        L.orc_bh_learned.argtypes = [C.c_int32, f64p, C.c_double, f64p, f64p]
        L.orc_bh_learned_rows.argtypes = [C.c_int32, f64p, C.c_double, f64p, i32p, C.c_int32,
                                          f64p]
        L.orc_mlp_forward.argtypes = [f64p, C.c_int64, f64p, f64p]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _i32(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.int32)


# ------------------------------------------------------------------ primitives

def set_threads(n: int) -> int:
    """Threads of the oracle's parallel loops from now on; returns the previous
    maximum (results do not depend on it)."""
    return int(lib().orc_set_threads(int(n)))


def splitmix64_at(state: int, i: int) -> int:
    return int(lib().orc_splitmix64_at(state, i))


def draws(seed: int, level: int, tag: int, i0: int, count: int) -> np.ndarray:
    out = np.empty(count, dtype=np.uint64)
    lib().orc_draws(seed, level, tag, i0, count, out)
    return out


def validate(row_ptr, col, node_w=None, edge_w=None) -> int:
    row_ptr, col = _i32(row_ptr), _i32(col)
    node_w, edge_w = _i32(node_w), _i32(edge_w)
    n = row_ptr.size - 1
    if n < 2:
        return 1
    return int(lib().orc_validate(n, row_ptr, col, _ptr(node_w), _ptr(edge_w)))


@dataclass
class KHop:
    """S_k(u) for every u: off[n+1], hend[n*k] (cumulative per-hop counts), nbr."""

    k: int
    off: np.ndarray
    hend: np.ndarray
    nbr: np.ndarray

    @property
    def n(self):
        return self.off.size - 1

    def row(self, u):
        return self.nbr[self.off[u]:self.off[u + 1]]

    def hops(self, u):
        """hop of every entry of row u."""
        hc = self.hend[u * self.k:(u + 1) * self.k]
        return np.repeat(np.arange(1, self.k + 1), np.diff(np.concatenate([[0], hc])))


def khop_build(row_ptr, col, k: int) -> KHop:
    row_ptr, col = _i32(row_ptr), _i32(col)
    n = row_ptr.size - 1
    off = np.zeros(n + 1, dtype=np.int64)
    if lib().orc_khop_build(n, row_ptr, col, k, off, None, None) != 0:
        raise MemoryError("khop count")
    hend = np.zeros(n * k, dtype=np.int32)
    nbr = np.zeros(int(off[-1]), dtype=np.int32)
    if lib().orc_khop_build(n, row_ptr, col, k, off, _ptr(hend), _ptr(nbr)) != 0:
        raise MemoryError("khop fill")
    return KHop(k, off, hend, nbr)


def farfield_exact(xy, q: float = 0.0) -> np.ndarray:
    xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1)
    n = xy.size // 2
    F = np.zeros(2 * n)
    lib().orc_farfield_exact(n, xy, q, F)
    return F.reshape(n, 2)


def cluster_far_field(xy, c, cl1, n1: int, clh, nh: int, q: float = 0.0) -> np.ndarray:
    """First two sums of Eq. 3 (Section 3.2): exact r-values within the own
    cluster of the next coarser level (cl1) plus, for every other vertex j of
    the approximation level (clh), nu_j r(x_u, xp_j) with nu_j the number of
    vertices j represents here and xp_j their node-weighted midpoint."""
    xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1)
    n = xy.size // 2
    cl1 = _i32(cl1)
    clh = _i32(clh)
    cw = _i32(c)
    F = np.zeros(2 * n)
    rc = lib().orc_cluster_far(n, xy, None if cw is None else cw.ctypes.data_as(C.c_void_p),
                               cl1, int(n1), clh, int(nh), q, F)
    if rc != 0:
        raise ValueError(f"orc_cluster_far failed ({rc})")
    return F.reshape(n, 2)


@dataclass
class BHResult:
    F: np.ndarray
    codes: np.ndarray
    order: np.ndarray
    nodes: np.ndarray  # (count, 5): depth, first, count, is_leaf, prefix (pre-order)
    accepted: int
    leaf_pairs: int
    coincident: int


def barnes_hut(xy, theta: float, q: float = 0.0) -> BHResult:
    xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1)
    n = xy.size // 2
    F = np.zeros(2 * n)
    codes = np.zeros(n, dtype=np.uint64)
    order = np.zeros(n, dtype=np.int32)
    cap = 2 * n + 1
    nodes = np.zeros(5 * cap, dtype=np.int64)
    stats = np.zeros(4, dtype=np.int64)
    rc = lib().orc_bh(n, xy, q, theta, F, _ptr(codes), _ptr(order), _ptr(nodes), cap, stats)
    if rc != 0:
        raise MemoryError("orc_bh")
    nn = int(stats[3])
    return BHResult(F.reshape(n, 2), codes, order, nodes[:5 * nn].reshape(nn, 5),
                    int(stats[0]), int(stats[1]), int(stats[2]))


@dataclass
class Samples:
    """Accepted (target, cell) pairs of a Barnes-Hut traversal with features,
    exact residual targets (h units) and kappa e, in (u, visit) order."""

    u: np.ndarray
    node: np.ndarray
    feat: np.ndarray    # (count, 8)
    target: np.ndarray  # (count, 2)
    coef: np.ndarray    # (count, 2)


def far_samples(xy, theta: float) -> Samples:
    xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1)
    n = xy.size // 2
    cnt = np.zeros(1, dtype=np.int64)
    z32, z64, zf = (np.zeros(1, dtype=np.int32), np.zeros(1, dtype=np.int64), np.zeros(8))
    if lib().orc_far_samples(n, xy, theta, 0, z32, z64, zf, zf, zf, cnt) != 0:
        raise MemoryError("far_samples")
    m = int(cnt[0])
    u = np.zeros(max(m, 1), dtype=np.int32)
    node = np.zeros(max(m, 1), dtype=np.int64)
    feat = np.zeros(8 * max(m, 1))
    tgt = np.zeros(2 * max(m, 1))
    coef = np.zeros(2 * max(m, 1))
    if lib().orc_far_samples(n, xy, theta, m, u, node, feat, tgt, coef, cnt) != 0:
        raise MemoryError("far_samples")
    return Samples(u[:m], node[:m], feat[:8 * m].reshape(m, 8), tgt[:2 * m].reshape(m, 2),
                   coef[:2 * m].reshape(m, 2))


def barnes_hut_learned(xy, theta: float, weights) -> np.ndarray:
    """Barnes-Hut far field (q = 0) with the learned cell correction."""
    xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1)
    w = np.ascontiguousarray(weights, dtype=np.float64).reshape(-1)
    n = xy.size // 2
    F = np.zeros(2 * n)
    if lib().orc_bh_learned(n, xy, theta, w, F) != 0:
        raise MemoryError("bh_learned")
    return F.reshape(n, 2)


def barnes_hut_learned_rows(xy, theta: float, weights, rows) -> np.ndarray:
    """barnes_hut_learned for the given points only (same tree, same visit)."""
    xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1)
    w = np.ascontiguousarray(weights, dtype=np.float64).reshape(-1)
    rows = _i32(rows)
    n = xy.size // 2
    F = np.zeros(2 * rows.size)
    if lib().orc_bh_learned_rows(n, xy, theta, w, rows, rows.size, F) != 0:
        raise MemoryError("bh_learned_rows")
    return F.reshape(-1, 2)


def mlp_forward_c(weights, feat) -> np.ndarray:
    """The C forward pass used inside barnes_hut_learned."""
    w = np.ascontiguousarray(weights, dtype=np.float64).reshape(-1)
    f = np.ascontiguousarray(feat, dtype=np.float64).reshape(-1)
    out = np.zeros(f.size // 8 * 2)
    lib().orc_mlp_forward(w, f.size // 8, f, out)
    return out.reshape(-1, 2)


def sweep(kh: KHop, x, F, alpha: float, q: float = 0.0, level: int = 0,
          c=None, scale: float = 1.0):
    """One Jacobi iteration (Eq. 2) with the far field F given (all v != u).

    Returns (x', delta) with delta = |x'-x| / |x|."""
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1)
    F = np.ascontiguousarray(F, dtype=np.float64).reshape(-1)
    c = _i32(c)
    n = x.size // 2
    xo = np.zeros(2 * n)
    d = np.zeros(2)
    lib().orc_sweep(n, level, kh.k, kh.off, kh.hend, kh.nbr, _ptr(c), scale, x, F, alpha, q,
                    xo, d)
    return xo.reshape(n, 2), math.sqrt(d[0] / d[1]) if d[1] > 0 else math.inf


def sweep_direct(kh: KHop, x, alpha: float, q: float = 0.0, level: int = 0, c=None,
                 scale: float = 1.0):
    """Eq. 2 with the entropy sum taken directly over v not in S(u)."""
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1)
    c = _i32(c)
    n = x.size // 2
    xo = np.zeros(2 * n)
    d = np.zeros(2)
    if lib().orc_sweep_direct(n, level, kh.k, kh.off, kh.hend, kh.nbr, _ptr(c), scale, x,
                              alpha, q, xo, d) != 0:
        raise MemoryError("sweep_direct")
    return xo.reshape(n, 2), math.sqrt(d[0] / d[1]) if d[1] > 0 else math.inf


def sweep_rows(row_ptr, col, k: int, x, F, alpha: float, rows, q: float = 0.0, level: int = 0,
               c=None, scale: float = 1.0):
    """Eq. 2 for the given rows only, each S(u) found by its own BFS."""
    row_ptr, col, c = _i32(row_ptr), _i32(col), _i32(c)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1)
    F = np.ascontiguousarray(F, dtype=np.float64).reshape(-1)
    rows = _i32(rows)
    n = row_ptr.size - 1
    out = np.zeros(2 * rows.size)
    sizes = np.zeros(rows.size, dtype=np.int64)
    if lib().orc_sweep_rows(n, row_ptr, col, level, k, _ptr(c), scale, x, F, alpha, q, rows,
                            rows.size, out, sizes) != 0:
        raise MemoryError("sweep_rows")
    return out.reshape(-1, 2), sizes


def lp(row_ptr, col, U: float, rounds: int, seed: int, level_h: int, c=None, w=None,
       label=None):
    """Synchronous size-constrained label propagation (see mm_oracle.h)."""
    row_ptr, col, c, w = _i32(row_ptr), _i32(col), _i32(c), _i32(w)
    n = row_ptr.size - 1
    lab = np.arange(n, dtype=np.int32) if label is None else _i32(label).copy()
    moves = np.zeros(max(rounds, 1), dtype=np.int32)
    r = lib().orc_lp(n, row_ptr, col, _ptr(c), _ptr(w), U, rounds, seed, level_h, lab, moves)
    if r < 0:
        raise MemoryError("lp")
    return lab, moves[:r]


@dataclass
class Level:
    row_ptr: np.ndarray
    col: np.ndarray
    c: np.ndarray | None = None  # node weights (None = 1)
    w: np.ndarray | None = None  # edge weights (None = 1)

    @property
    def n(self):
        return self.row_ptr.size - 1


def contract(lv: Level, label):
    n = lv.n
    nnz = lv.col.size
    cluster = np.zeros(n, dtype=np.int32)
    crp = np.zeros(n + 1, dtype=np.int32)
    ccol = np.zeros(max(nnz, 1), dtype=np.int32)
    cc = np.zeros(n, dtype=np.int32)
    cw = np.zeros(max(nnz, 1), dtype=np.int32)
    cnnz = np.zeros(1, dtype=np.int64)
    nc = lib().orc_contract(n, _i32(lv.row_ptr), _i32(lv.col), _ptr(_i32(lv.c)),
                            _ptr(_i32(lv.w)), _i32(label), cluster, crp, ccol, cc, cw, cnnz)
    if nc < 0:
        raise MemoryError("contract")
    e = int(cnnz[0])
    return cluster, Level(crp[:nc + 1].copy(), ccol[:e].copy(), cc[:nc].copy(), cw[:e].copy())


def init_layout(n: int, seed: int, level: int) -> np.ndarray:
    xy = np.zeros(2 * n)
    lib().orc_init_layout(n, seed, level, xy)
    return xy.reshape(n, 2)


def prolong(cluster, coarse_c, coarse_xy, seed: int, level: int) -> np.ndarray:
    cluster = _i32(cluster)
    cxy = np.ascontiguousarray(coarse_xy, dtype=np.float64).reshape(-1)
    out = np.zeros(2 * cluster.size)
    lib().orc_prolong(cluster.size, cluster, _ptr(_i32(coarse_c)), cxy, seed, level, out)
    return out.reshape(-1, 2)


def objective(kh: KHop, x, alpha: float, q: float = 0.0, level: int = 0, c=None,
              scale: float = 1.0) -> dict:
    """Maxent-stress (Eq. 1 over the stress set S = S_k): M = stress - alpha*ent."""
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1)
    n = x.size // 2
    out = np.zeros(3)
    if lib().orc_objective(n, level, kh.k, kh.off, kh.hend, kh.nbr, _ptr(_i32(c)), scale, x, q,
                           out) != 0:
        raise MemoryError("objective")
    return {"stress": out[0], "ent": out[1], "coincident": int(out[2]),
            "M": out[0] - alpha * out[1]}


def full_stress(row_ptr, col, x) -> dict:
    """Full stress over all pairs with hop distances; F at the optimal scale s*."""
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1)
    n = x.size // 2
    out = np.zeros(3)
    if lib().orc_full_stress(n, _i32(row_ptr), _i32(col), x, out) != 0:
        raise MemoryError("full_stress")
    return {"F_unscaled": out[0], "s_opt": out[1], "F": out[2]}


# ------------------------------------------------------------------ driver

@dataclass
class Params:
    """Layout parameters; defaults are the paper's configuration.

    k: hop radius of the stress set (1 = edges only, the paper's default model).
    theta < 0 selects the exact all-pairs far field, theta >= 0 Barnes-Hut;
    levels with at most exact_below vertices use the exact far field either way.
    approx_h > 0 selects the cluster far field of Eq. 3 with the graph h levels
    beneath (or the coarsest) on every level that has a coarser one (MulMent_h);
    the coarsest level then uses the exact far field.
    """

    k: int = 1
    q: float = 0.0
    theta: float = 0.5
    alpha0: float = 1.0
    alpha_decay: float = 0.3
    alpha_min: float = 0.008
    iters_per_round: int = 2
    eps_round: float = 1e-4
    eps_final: float = 1e-4
    max_final_iters: int = 200
    max_levels: int = 62
    coarsest_n: int = 2
    b: float = 2.0
    f: float = 20.0
    lp_rounds: int = 10
    coarse_dist_scale: float = 1.0
    seed: int = 1
    mlp: np.ndarray | None = None  # far-field correction weights (q = 0, theta >= 0)
    exact_below: int = 0
    approx_h: int = 0



def schedule(alpha0, alpha_decay, alpha_min):
    """alpha values of the rounds before the final phase at alpha_min."""
    out = []
    a = alpha0
    while a > alpha_min:
        out.append(a)
        a = max(a * alpha_decay, alpha_min)
    return out


def hierarchy(g0: Level, p: Params, trace: list | None = None):
    """Coarsening (Section 3.1).  Returns (levels, clusters, info).
    trace (optional list) receives one record per contraction attempt: the
    level index h, f, W and U of the attempt, the contracted size n, whether
    the 10% rule fired (then also f_next, the f it leaves), and the
    attempt's rebuild counter.

    Reading: |V| in W = min(b^h, |V|/f) is the total node weight; h is the
    index of the level being built (1 for the first contraction).  When the
    contracted graph is not 10% smaller, f := 0.7 f for all later levels, and
    the level is rebuilt with the new f only if W was bounded by |V|/f (else
    a rebuild could not change the result); at most 10 rebuilds per level.
    Coarsening stops at max_levels, at <= max(coarsest_n, 2) vertices, or
    when a contraction makes no progress or would leave fewer than 2
    vertices (the paper coarsens down to two nodes).
    """
    levels = [g0]
    clusters = []
    f = p.f
    cV = float(g0.n if g0.c is None else int(np.sum(g0.c, dtype=np.int64)))
    h = 1
    redo = 0
    info = []
    while len(levels) - 1 < p.max_levels and levels[-1].n > max(p.coarsest_n, 2):
        G = levels[-1]
        W = min(p.b ** h, cV / f)
        maxc = 1 if G.c is None else int(G.c.max())
        U = max(float(maxc), W)
        label, moves = lp(G.row_ptr, G.col, U, p.lp_rounds, p.seed, h, G.c, G.w)
        cluster, Gc = contract(G, label)
        if trace is not None:
            trace.append({"h": h, "f": f, "W": W, "U": U, "n": Gc.n,
                          "fired": bool(Gc.n > 0.9 * G.n), "redo": redo})
        if Gc.n > 0.9 * G.n:
            bounded_by_f = (cV / f) < p.b ** h
            f = 0.7 * f
            if trace is not None:
                trace[-1]["f_next"] = f
            if bounded_by_f and redo < 10:
                redo += 1
                continue
        if Gc.n >= G.n or Gc.n < 2:
            break
        info.append({"h": h, "U": U, "n": Gc.n, "lp_rounds": int(moves.size), "redo": redo})
        levels.append(Gc)
        clusters.append(cluster)
        h += 1
        redo = 0
    return levels, clusters, info


def far_field(x, p: Params):
    if p.theta < 0 or x.shape[0] <= p.exact_below:
        return farfield_exact(x, p.q)
    if p.mlp is not None:
        return barnes_hut_learned(x, p.theta, p.mlp)
    return barnes_hut(x, p.theta, p.q).F


def refine(lv: Level, level: int, x, p: Params, kh: KHop | None = None, start_alpha=None,
           far=None):
    """Local improvement on one level (Section 3.2).  far(x) -> F overrides the
    far field chosen by p (the cluster far field of Eq. 3)."""
    if kh is None:
        kh = khop_build(lv.row_ptr, lv.col, p.k)
    alpha = p.alpha0 if start_alpha is None else start_alpha
    iters = 0
    hist = []

    def T(x, a):
        F = far(x) if far is not None else far_field(x, p)
        return sweep(kh, x, F, a, p.q, level, lv.c, p.coarse_dist_scale)

    while alpha > p.alpha_min:
        for _ in range(p.iters_per_round):
            x, d = T(x, alpha)
            iters += 1
            hist.append((alpha, d))
            if d < p.eps_round:
                break
        alpha = max(alpha * p.alpha_decay, p.alpha_min)
    final = 0
    for _ in range(p.max_final_iters):
        x, d = T(x, p.alpha_min)
        iters += 1
        final += 1
        hist.append((p.alpha_min, d))
        if d < p.eps_final:
            break
    return x, {"iters": iters, "final_iters": final, "hist": hist, "khop_entries": int(kh.off[-1])}


def place_pair(x, lv: Level, level: int, p: Params):
    """Two-vertex coarsest graph: keep the seeded direction, set the distance to
    the optimal one (Section 3.1), i.e. the target distance of the pair."""
    c0 = 1 if lv.c is None else int(lv.c[0])
    c1 = 1 if lv.c is None else int(lv.c[1])
    d = 1.0 if level == 0 else (math.sqrt(c0) + math.sqrt(c1)) * p.coarse_dist_scale
    x = np.array(x, dtype=np.float64).reshape(2, 2)
    dx, dy = x[1, 0] - x[0, 0], x[1, 1] - x[0, 1]
    D = math.sqrt(dx * dx + dy * dy)
    if D == 0.0:
        dx, dy, D = 1.0, 0.0, 1.0
    x[1, 0] = x[0, 0] + d * dx / D
    x[1, 1] = x[0, 1] + d * dy / D
    return x


def layout(g, p: Params, init_xy=None):
    """Full multilevel layout.  g: object with row_ptr/col (+ optional node_w,
    edge_w).  Returns (x[n,2] FP64, stats)."""
    g0 = Level(_i32(g.row_ptr), _i32(g.col), _i32(getattr(g, "node_w", None)),
               _i32(getattr(g, "edge_w", None)))
    if init_xy is not None:
        # warm start on the finest level only (the update algorithm of Sec.
        # 4.3); with approx_h > 0 the coarsening stops after h levels, whose
        # last graph serves the cluster far field of Eq. 3
        far = None
        info = []
        if p.approx_h > 0:
            levels, clusters, info = hierarchy(g0, replace(p, max_levels=min(p.max_levels,
                                                                             p.approx_h)))
            L = len(levels) - 1
            if L > 0:
                clh = clusters[0]
                for j in range(1, L):
                    clh = clusters[j][clh]
                args = (g0.c, clusters[0], levels[1].n, clh, levels[L].n, p.q)
                far = lambda xx, a=args: cluster_far_field(xx, *a)
        stats = {"levels": [], "hierarchy": info}
        x, st = refine(g0, 0, np.asarray(init_xy, dtype=np.float64), p,
                       start_alpha=p.alpha_min, far=far)
        stats["levels"].append({"level": 0, "n": g0.n, **st})
        return x, stats
    levels, clusters, info = hierarchy(g0, p)
    L = len(levels) - 1
    stats = {"levels": [], "hierarchy": info}
    x = init_layout(levels[L].n, p.seed, L)
    if levels[L].n == 2:
        x = place_pair(x, levels[L], L, p)
    for lvl in range(L, -1, -1):
        if lvl < L:
            x = prolong(clusters[lvl], levels[lvl + 1].c, x, p.seed, lvl)
        far = None
        if p.approx_h > 0 and lvl < L:
            # Eq. 3: own cluster one level down, representatives h levels
            # down (or on the coarsest level)
            lh = min(lvl + p.approx_h, L)
            clh = clusters[lvl]
            for j in range(lvl + 1, lh):
                clh = clusters[j][clh]
            args = (levels[lvl].c, clusters[lvl], levels[lvl + 1].n, clh, levels[lh].n, p.q)
            far = lambda xx, a=args: cluster_far_field(xx, *a)
        x, st = refine(levels[lvl], lvl, x, p, far=far)
        stats["levels"].append({"level": lvl, "n": levels[lvl].n, **st})
    return x, stats
