"""Dynamic-graph churn (the random change model of the paper's dynamic-network section).

From graph G: BFS spanning tree from a random root; remove x% of the edges,
drawn among the non-tree edges (so the graph stays connected); insert x% new
edges, each from a random vertex to a random vertex at hop distance
1 < d <= D in G.  Pure graph construction, no layout arithmetic.
"""
from __future__ import annotations

import numpy as np
from scipy.sparse.csgraph import breadth_first_order

from .graphs import Graph, csr_from_edges
import scipy.sparse as sp


def _bfs_hops(g: Graph, s: int, limit: int) -> dict:
    dist = {s: 0}
    frontier = [s]
    for h in range(1, limit + 1):
        nxt = []
        for u in frontier:
            for v in g.col[g.row_ptr[u]:g.row_ptr[u + 1]]:
                v = int(v)
                if v not in dist:
                    dist[v] = h
                    nxt.append(v)
        frontier = nxt
    return dist


def churn_snapshot(g: Graph, seed: int, frac: float = 0.01, D: int = 2) -> Graph:
    rng = np.random.default_rng(seed)
    n = g.n
    a = sp.csr_matrix((np.ones(g.nnz, dtype=np.int8), g.col, g.row_ptr), shape=(n, n))
    root = int(rng.integers(n))
    _, pred = breadth_first_order(a, root, directed=False, return_predecessors=True)
    src, dst = g.edges()
    tree = np.zeros(src.size, dtype=bool)
    child = np.arange(n)
    par = pred
    ok = par >= 0
    tkey = set((np.minimum(child[ok], par[ok]) * n + np.maximum(child[ok], par[ok])).tolist())
    key = src * n + dst
    tree = np.fromiter((int(k) in tkey for k in key), dtype=bool, count=key.size)
    non_tree = np.flatnonzero(~tree)
    n_change = int(round(frac * src.size))
    drop = rng.choice(non_tree, size=min(n_change, non_tree.size), replace=False)
    keep = np.ones(src.size, dtype=bool)
    keep[drop] = False
    new_s, new_d = [], []
    existing = set(key.tolist())
    tries = 0
    while len(new_s) < n_change and tries < 100 * max(n_change, 1):
        tries += 1
        u = int(rng.integers(n))
        hops = _bfs_hops(g, u, D)
        cand = sorted(v for v, h in hops.items() if 1 < h <= D)
        if not cand:
            continue
        v = cand[int(rng.integers(len(cand)))]
        k = min(u, v) * n + max(u, v)
        if k in existing:
            continue
        existing.add(k)
        new_s.append(u)
        new_d.append(v)
    s2 = np.concatenate([src[keep], np.asarray(new_s, dtype=np.int64)])
    d2 = np.concatenate([dst[keep], np.asarray(new_d, dtype=np.int64)])
    out = csr_from_edges(n, s2, d2, name=g.name + "_churn")
    out.points = g.points
    return out
