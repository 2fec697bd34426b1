"""Labelled stress sets S ⊇ E of the general model (footnote to Eq. 1) for
the tests, built by brute force: target distances d_uv are hop distances
from scipy's breadth-first all-pairs shortest paths, so neither the oracle
nor the library takes part in making them.  Small graphs only (the hop
matrix is dense)."""
import numpy as np
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import shortest_path
from scipy.spatial import cKDTree


def hop_matrix(g) -> np.ndarray:
    A = csr_matrix((np.ones(g.nnz), g.col, g.row_ptr), shape=(g.n, g.n))
    return shortest_path(A, directed=False, unweighted=True)


def to_arrays(n: int, k: int, src, dst, hop):
    """(off int64[n+1], hend int32[n*k], nbr int32) from the pairs of both
    directions; rows grouped by distance, ids ascending inside a group."""
    src, dst, hop = (np.asarray(a, dtype=np.int64) for a in (src, dst, hop))
    order = np.lexsort((dst, hop, src))
    src, dst, hop = src[order], dst[order], hop[order]
    off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(src, minlength=n), out=off[1:])
    counts = np.zeros((n, k), dtype=np.int64)
    np.add.at(counts, (src, hop - 1), 1)
    hend = np.cumsum(counts, axis=1).astype(np.int32).reshape(-1)
    return off, hend, dst.astype(np.int32)


def thresholded(g, pts, k: int, r: float, D=None):
    """S = E ∪ {{u, v} : hop(u, v) <= k and |p_u - p_v| < r}, d_uv = hop(u, v):
    a distance-thresholded stress set (p: any point set, e.g. a layout)."""
    D = hop_matrix(g) if D is None else D
    pairs = cKDTree(np.asarray(pts, dtype=np.float64)).query_pairs(r, output_type="ndarray")
    u, v = pairs[:, 0].astype(np.int64), pairs[:, 1].astype(np.int64)
    h = D[u, v]
    keep = np.isfinite(h) & (h <= k)
    eu, ev = g.edges()
    u = np.concatenate([u[keep], eu])
    v = np.concatenate([v[keep], ev])
    key = np.unique(np.minimum(u, v) * g.n + np.maximum(u, v))
    u, v = key // g.n, key % g.n
    h = D[u, v].astype(np.int64)
    return to_arrays(g.n, k, np.concatenate([u, v]), np.concatenate([v, u]),
                     np.concatenate([h, h]))


def sampled(g, k: int, frac: float, seed: int, D=None):
    """S = E ∪ a seeded random fraction of the pairs within k hops."""
    D = hop_matrix(g) if D is None else D
    iu, ju = np.triu_indices(g.n, 1)
    h = D[iu, ju]
    within = np.isfinite(h) & (h <= k)
    rng = np.random.default_rng(seed)
    keep = within & ((h == 1) | (rng.random(h.size) < frac))
    u, v, h = iu[keep], ju[keep], h[keep].astype(np.int64)
    return to_arrays(g.n, k, np.concatenate([u, v]), np.concatenate([v, u]),
                     np.concatenate([h, h]))
