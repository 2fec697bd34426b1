"""Batches of uneven graphs: n = round(exp(U[ln nmin, ln nmax])), the type
uniform over {grid floor(sqrt n) x ceil(n / floor(sqrt n)), random recursive
tree, random geometric graph (mean degree 6, largest component)}."""
from __future__ import annotations

import math

import numpy as np

from .graphs import Graph, grid, random_tree, rgg


def batch_graphs(count: int, seed: int, nmin: int = 64, nmax: int = 8192) -> list[Graph]:
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
        kind = int(rng.integers(3))
        sub = int(rng.integers(1 << 31))
        if kind == 0:
            r = int(math.isqrt(n))
            g = grid(r, (n + r - 1) // r)
        elif kind == 1:
            g = random_tree(n, sub)
        else:
            g = rgg(n, sub, 6.0)
            if g.n < 2:
                g = random_tree(n, sub)
        out.append(g)
    return out


def concat(graphs: list[Graph]):
    """Block-diagonal union: (row_ptr, col, vertex offsets)."""
    offs = np.zeros(len(graphs) + 1, dtype=np.int64)
    rps, cols = [], []
    e0 = 0
    for i, g in enumerate(graphs):
        offs[i + 1] = offs[i] + g.n
        rps.append(np.asarray(g.row_ptr[:-1], dtype=np.int64) + e0)
        cols.append(np.asarray(g.col, dtype=np.int64) + offs[i])
        e0 += int(g.row_ptr[-1])
    rp = np.concatenate(rps + [np.array([e0])]).astype(np.int32)
    col = np.concatenate(cols).astype(np.int32)
    return rp, col, offs
