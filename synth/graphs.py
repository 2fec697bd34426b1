"""Graph generators (CSR, int32, symmetric, sorted rows, no self-loops or duplicates).

Shapes follow the workloads the paper evaluates on (its instance table lists
grids/meshes, Delaunay triangulations, road networks, trees and sparse matrix
graphs); the paper's files themselves are not used.  Seeds go through numpy's
PCG64 (``numpy.random.default_rng``).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components


@dataclass
class Graph:
    """Undirected simple graph in CSR form.

    row_ptr: int32[n+1], col: int32[2m] (each undirected edge stored twice,
    rows sorted ascending).  node_w / edge_w are None for unit weights.
    """

    row_ptr: np.ndarray
    col: np.ndarray
    node_w: np.ndarray | None = None
    edge_w: np.ndarray | None = None
    name: str = ""
    points: np.ndarray | None = None  # generator coordinates, if any (not a layout)

    @property
    def n(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    @property
    def m(self) -> int:
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr.astype(np.int64))

    def edges(self) -> tuple[np.ndarray, np.ndarray]:
        """Undirected edges (u < v) in row order."""
        src = np.repeat(np.arange(self.n, dtype=np.int64), self.degrees())
        dst = self.col.astype(np.int64)
        keep = src < dst
        return src[keep], dst[keep]


def csr_from_edges(n: int, src, dst, name: str = "") -> Graph:
    """Symmetric CSR from an arbitrary directed/undirected edge list.

    Self-loops are dropped, both directions are added, duplicates removed and
    rows sorted.
    """
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    keep = src != dst
    src, dst = src[keep], dst[keep]
    a = np.concatenate([src, dst])
    b = np.concatenate([dst, src])
    key = np.unique(a * n + b)
    a = (key // n).astype(np.int64)
    b = (key % n).astype(np.int32)
    counts = np.bincount(a, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("graph too large for int32 CSR")
    return Graph(row_ptr.astype(np.int32), b.astype(np.int32), name=name)


def relabel(g: Graph, perm_new_of_old: np.ndarray) -> Graph:
    """Relabel vertices: new id of old vertex v is perm_new_of_old[v]."""
    src = np.repeat(np.arange(g.n, dtype=np.int64), g.degrees())
    p = np.asarray(perm_new_of_old, dtype=np.int64)
    out = csr_from_edges(g.n, p[src], p[g.col.astype(np.int64)], name=g.name)
    if g.points is not None:
        pts = np.empty_like(g.points)
        pts[p] = g.points
        out.points = pts
    return out


def largest_component(g: Graph) -> Graph:
    """Largest connected component, ids relabelled to ascending order."""
    n = g.n
    a = sp.csr_matrix(
        (np.ones(g.nnz, dtype=np.int8), g.col, g.row_ptr), shape=(n, n)
    )
    ncomp, lab = connected_components(a, directed=False)
    if ncomp == 1:
        return g
    big = np.argmax(np.bincount(lab))
    keep = np.flatnonzero(lab == big)
    new_id = -np.ones(n, dtype=np.int64)
    new_id[keep] = np.arange(keep.size)
    src = np.repeat(np.arange(n, dtype=np.int64), g.degrees())
    dst = g.col.astype(np.int64)
    ok = (new_id[src] >= 0) & (new_id[dst] >= 0)
    out = csr_from_edges(keep.size, new_id[src[ok]], new_id[dst[ok]], name=g.name)
    if g.points is not None:
        out.points = g.points[keep]
    return out


# ---------------------------------------------------------------- small shapes

def grid(rows: int, cols: int) -> Graph:
    """rows x cols grid, v = cols*i + j, edges to the right and down."""
    v = np.arange(rows * cols, dtype=np.int64).reshape(rows, cols)
    src = np.concatenate([v[:, :-1].ravel(), v[:-1, :].ravel()])
    dst = np.concatenate([v[:, 1:].ravel(), v[1:, :].ravel()])
    return csr_from_edges(rows * cols, src, dst, name=f"grid{rows}x{cols}")


def path(n: int) -> Graph:
    v = np.arange(n - 1)
    return csr_from_edges(n, v, v + 1, name=f"path{n}")


def cycle(n: int) -> Graph:
    v = np.arange(n)
    return csr_from_edges(n, v, (v + 1) % n, name=f"cycle{n}")


def star(leaves: int) -> Graph:
    """Centre 0 joined to vertices 1..leaves."""
    v = np.arange(1, leaves + 1)
    return csr_from_edges(leaves + 1, np.zeros_like(v), v, name=f"star{leaves}")


def complete_binary_tree(depth: int) -> Graph:
    """Complete binary tree with 2^(depth+1)-1 vertices (depth 9 -> 1023)."""
    n = 2 ** (depth + 1) - 1
    child = np.arange(1, n)
    return csr_from_edges(n, (child - 1) // 2, child, name=f"btree{n}")


def two_triangles() -> Graph:
    """Triangles {0,1,2} and {3,4,5} joined by the edge 2-3."""
    src = [0, 0, 1, 3, 3, 4, 2]
    dst = [1, 2, 2, 4, 5, 5, 3]
    return csr_from_edges(6, src, dst, name="two_triangles")


def random_tree(n: int, seed: int) -> Graph:
    """Random recursive tree: parent(v) ~ U[0, v) for v >= 1."""
    rng = np.random.default_rng(seed)
    v = np.arange(1, n, dtype=np.int64)
    parent = np.floor(rng.random(n - 1) * v).astype(np.int64)
    return csr_from_edges(n, parent, v, name=f"rtree{n}")


# ---------------------------------------------------------------- paper-shaped workloads

def rgg(n: int, seed: int, avg_degree: float = 6.0, lcc: bool = True) -> Graph:
    """Random geometric graph: n points uniform in [0,1)^2, edge iff distance <= r.

    r = sqrt(avg_degree / (pi n)) (no torus), then the largest component.
    """
    from scipy.spatial import cKDTree

    rng = np.random.default_rng(seed)
    pts = rng.random((n, 2))
    r = math.sqrt(avg_degree / (math.pi * n))
    pairs = cKDTree(pts).query_pairs(r, output_type="ndarray")
    g = csr_from_edges(n, pairs[:, 0], pairs[:, 1], name=f"rgg{n}")
    g.points = pts
    return largest_component(g) if lcc else g


def rmat(scale: int, edge_draws: int, seed: int, a=0.57, b=0.19, c=0.19,
         relabel_random: bool = True) -> Graph:
    """R-MAT graph with 2^scale vertices and ``edge_draws`` directed draws.

    Per bit level the quadrant is chosen with probabilities (a, b, c, d=1-a-b-c),
    no noise.  Self-loops and duplicates are removed, the result symmetrised,
    the largest component kept, and (by default) ids permuted at random with
    the seed so that ids carry no degree information.
    """
    rng = np.random.default_rng(seed)
    src = np.zeros(edge_draws, dtype=np.int64)
    dst = np.zeros(edge_draws, dtype=np.int64)
    ab, abc = a + b, a + b + c
    for bit in range(scale):
        r = rng.random(edge_draws)
        sbit = r >= ab
        dbit = ((r >= a) & (r < ab)) | (r >= abc)
        src |= sbit.astype(np.int64) << bit
        dst |= dbit.astype(np.int64) << bit
    n = 1 << scale
    g = largest_component(csr_from_edges(n, src, dst, name=f"rmat{scale}"))
    if relabel_random:
        g = relabel(g, rng.permutation(g.n))
    return g


def delaunay(n: int, seed: int) -> Graph:
    """Delaunay triangulation of n uniform points in the unit square."""
    from scipy.spatial import Delaunay

    rng = np.random.default_rng(seed)
    pts = rng.random((n, 2))
    tri = Delaunay(pts).simplices.astype(np.int64)
    src = np.concatenate([tri[:, 0], tri[:, 1], tri[:, 2]])
    dst = np.concatenate([tri[:, 1], tri[:, 2], tri[:, 0]])
    g = csr_from_edges(n, src, dst, name=f"del{n}")
    g.points = pts
    return g


def config_graph(name: str, seed: int = 1) -> Graph:
    """The synthetic stand-ins for the evaluated workloads, by name.

    grid32   : 32x32 grid (1024 vertices, 1984 edges)
    rgg17    : RGG, 2^17 points, mean degree ~6, largest component
    rmat20   : R-MAT scale 20, 8*2^20 draws (a,b,c)=(.57,.19,.19), LCC, random ids
    rgg16    : RGG, 2^16 points, mean degree ~6, LCC (dynamic snapshots)
    rgg22    : RGG, 2^22 points, mean degree ~8, LCC
    rgg14    : RGG, 2^14 points, mean degree ~8, LCC
    del20    : Delaunay triangulation of 2^20 uniform points (del16: 2^16)
    """
    if name == "grid32":
        return grid(32, 32)
    if name == "rgg17":
        return rgg(1 << 17, seed, 6.0)
    if name == "rgg16":
        return rgg(1 << 16, seed, 6.0)
    if name == "rgg14":
        return rgg(1 << 14, seed, 8.0)
    if name == "rgg22":
        return rgg(1 << 22, seed, 8.0)
    if name == "rmat20":
        return rmat(20, 8 * (1 << 20), seed)
    if name.startswith("del"):
        return delaunay(1 << int(name[3:]), seed)
    if name.startswith("rmat"):
        s = int(name[4:])
        return rmat(s, 8 * (1 << s), seed)
    if name.startswith("rgg"):
        return rgg(1 << int(name[3:]), seed, 6.0)
    raise KeyError(name)
