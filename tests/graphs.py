"""Small deterministic test graphs given as raw tuples (src, dst, n, directed)."""
from __future__ import annotations

import numpy as np


def _pack(edges, n, directed):
    if len(edges) == 0:
        e = np.zeros((0, 2), dtype=np.int32)
    else:
        e = np.asarray(edges, dtype=np.int32).reshape(-1, 2)
    return e[:, 0].copy(), e[:, 1].copy(), int(n), bool(directed)


def path(n, directed=False):
    return _pack([(i, i + 1) for i in range(n - 1)], n, directed)


def cycle(n, directed=False):
    return _pack([(i, (i + 1) % n) for i in range(n)], n, directed)


def star(n):
    """Center 0, leaves 1..n-1."""
    return _pack([(0, i) for i in range(1, n)], n, False)


def complete(n):
    return _pack([(i, j) for i in range(n) for j in range(i + 1, n)], n, False)


def complete_bipartite(a, b):
    """Side A = 0..a-1, side B = a..a+b-1."""
    return _pack([(i, a + j) for i in range(a) for j in range(b)], a + b, False)


def binary_tree(depth):
    """Complete binary tree with root 0 and 2**(depth+1)-1 vertices (heap numbering)."""
    n = 2 ** (depth + 1) - 1
    return _pack([((i - 1) // 2, i) for i in range(1, n)], n, False)


def grid(r, c):
    """r x c grid graph, vertex (i, j) = i*c + j."""
    e = []
    for i in range(r):
        for j in range(c):
            if j + 1 < c:
                e.append((i * c + j, i * c + j + 1))
            if i + 1 < r:
                e.append((i * c + j, (i + 1) * c + j))
    return _pack(e, r * c, False)


def hypercube(d):
    n = 1 << d
    return _pack([(v, v ^ (1 << b)) for v in range(n) for b in range(d) if v < v ^ (1 << b)], n, False)


def petersen():
    outer = [(i, (i + 1) % 5) for i in range(5)]
    spokes = [(i, i + 5) for i in range(5)]
    inner = [(5 + i, 5 + (i + 2) % 5) for i in range(5)]
    return _pack(outer + spokes + inner, 10, False)


def random_graph(rng: np.random.Generator, n: int, m: int, directed: bool, loops=True):
    """Uniform random tuples, duplicates and (optionally) self-loops kept."""
    src = rng.integers(0, n, size=m, dtype=np.int64).astype(np.int32)
    dst = rng.integers(0, n, size=m, dtype=np.int64).astype(np.int32)
    if not loops:
        keep = src != dst
        src, dst = src[keep], dst[keep]
    return src, dst, n, directed


def dense_adjacency(src, dst, n, directed):
    """Boolean adjacency of the tuples, self-loops kept (they do not change reachability)."""
    a = np.zeros((n, n), dtype=bool)
    a[src, dst] = True
    if not directed:
        a[dst, src] = True
    return a
