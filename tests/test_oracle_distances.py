"""Pins of the oracle's breadth-first distances (the search of Section III run
to the end: no k cap) to facts that do not come from the oracle itself.

  * brute force: the first boolean power of the dense adjacency matrix that
    reaches a vertex is its distance;
  * closed forms: |i - s| on a path, (j - s) mod n on a directed cycle, the
    cyclic distance on an undirected cycle, Manhattan distance on a grid,
    Hamming distance on a hypercube, the depth in a complete binary tree;
  * an independent library routine (scipy's unweighted csgraph shortest paths);
  * breadth-first-tree validity (as the Graph500 checker states it): the seed
    at 0, every arc u -> v with dist(u) known gives dist(v) <= dist(u) + 1, and
    every reached vertex but the seed has an in-neighbor one level closer.
"""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import graphgen
import oracle
from tests import graphs

ALL = 2**31 - 1  # no depth limit


def og(src, dst, n, directed):
    return oracle.OracleGraph(src, dst, n, directed)


def brute_distances(src, dst, n, directed, s):
    a = graphs.dense_adjacency(src, dst, n, directed).astype(np.int64)
    dist = np.full(n, -1, dtype=np.int32)
    dist[s] = 0
    reach = np.zeros(n, dtype=bool)
    reach[s] = True
    for l in range(1, n):
        nxt = reach | ((reach.astype(np.int64) @ a) > 0)
        dist[nxt & ~reach] = l
        if (nxt == reach).all():
            break
        reach = nxt
    return dist


def bfs_tree_valid(src, dst, n, directed, s, dist):
    """Level-structure checks of a distance vector (no search of our own)."""
    keep = src != dst
    u = np.concatenate([src[keep], dst[keep]]) if not directed else src[keep]
    v = np.concatenate([dst[keep], src[keep]]) if not directed else dst[keep]
    assert dist[s] == 0
    assert ((dist == 0).sum()) == 1
    known = dist[u] >= 0
    # an arc out of a reached vertex reaches its head, at most one level further
    assert (dist[v][known] >= 0).all()
    assert (dist[v][known] <= dist[u][known] + 1).all()
    # every reached vertex but the seed has a parent one level closer
    has_parent = np.zeros(n, dtype=bool)
    ok = known & (dist[u] == dist[v] - 1)
    has_parent[v[ok]] = True
    reached = dist > 0
    assert has_parent[reached].all()


@settings(max_examples=600, deadline=None)
@given(n=st.integers(1, 40), m=st.integers(0, 140), directed=st.booleans(), rseed=st.integers(0, 2**32 - 1))
def test_brute_force_random(n, m, directed, rseed):
    rng = np.random.default_rng(rseed)
    src, dst, n, directed = graphs.random_graph(rng, n, m, directed)
    g = og(src, dst, n, directed)
    s = int(rng.integers(0, n))
    assert np.array_equal(g.distances(s, ALL), brute_distances(src, dst, n, directed, s))


@pytest.mark.parametrize("n,m,directed", [(256, 300, False), (256, 600, True), (200, 2000, False)])
def test_depth_limit_masks_the_full_distances(n, m, directed):
    rng = np.random.default_rng(n + m)
    src, dst, n, directed = graphs.random_graph(rng, n, m, directed)
    g = og(src, dst, n, directed)
    for s in rng.integers(0, n, size=5):
        full = brute_distances(src, dst, n, directed, int(s))
        for k in (0, 1, 2, 3, 5):
            d = g.distances(int(s), k)
            assert np.array_equal(d, np.where(full <= k, full, -1))


@pytest.mark.parametrize("n", [1, 2, 7, 40])
def test_path(n):
    g = og(*graphs.path(n))
    for s in (0, n // 2, n - 1):
        assert np.array_equal(g.distances(s, ALL), np.abs(np.arange(n) - s))


@pytest.mark.parametrize("n", [2, 5, 33])
def test_cycles(n):
    gu = og(*graphs.cycle(n))
    gd = og(*graphs.cycle(n, directed=True))
    j = np.arange(n)
    for s in (0, n - 1):
        fwd = (j - s) % n
        assert np.array_equal(gd.distances(s, ALL), fwd)
        assert np.array_equal(gu.distances(s, ALL), np.minimum(fwd, n - fwd))


@pytest.mark.parametrize("r,c", [(1, 5), (4, 4), (3, 9)])
def test_grid(r, c):
    g = og(*graphs.grid(r, c))
    i, j = np.divmod(np.arange(r * c), c)
    for s in (0, r * c - 1, (r // 2) * c + c // 2):
        si, sj = divmod(s, c)
        assert np.array_equal(g.distances(s, ALL), np.abs(i - si) + np.abs(j - sj))


@pytest.mark.parametrize("d", [1, 4, 7])
def test_hypercube(d):
    g = og(*graphs.hypercube(d))
    ids = np.arange(1 << d)
    for s in (0, 5 % (1 << d)):
        ham = np.array([bin(int(x) ^ s).count("1") for x in ids])
        assert np.array_equal(g.distances(s, ALL), ham)


@pytest.mark.parametrize("depth", [0, 3, 8])
def test_binary_tree(depth):
    g = og(*graphs.binary_tree(depth))
    ids = np.arange(2 ** (depth + 1) - 1)
    # heap numbering: vertex i sits at depth floor(log2(i + 1))
    assert np.array_equal(g.distances(0, ALL), np.floor(np.log2(ids + 1)).astype(np.int64))


def test_isolated_seed_reaches_nothing():
    g = og(np.array([1], dtype=np.int32), np.array([2], dtype=np.int32), 4, False)
    assert list(g.distances(0, ALL)) == [0, -1, -1, -1]
    assert list(g.distances(1, ALL)) == [-1, 0, 1, -1]


def _scipy_distances(el, seeds):
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import shortest_path
    keep = el.src != el.dst
    a = coo_matrix((np.ones(int(keep.sum())), (el.src[keep], el.dst[keep])), shape=(el.n, el.n)).tocsr()
    a.data[:] = 1.0
    d = shortest_path(a, directed=el.directed, indices=np.asarray(seeds), unweighted=True)
    return np.where(np.isfinite(d), d, -1).astype(np.int64)


def test_scipy_rmat_undirected():
    el = graphgen.rmat(13, 8, seed=21)
    g = oracle.OracleGraph.from_edgelist(el)
    seeds = graphgen.draw_seeds(el, 10, seed=3)
    ref = _scipy_distances(el, seeds)
    for i, s in enumerate(seeds):
        d = g.distances(int(s), ALL)
        assert np.array_equal(d, ref[i])
        bfs_tree_valid(el.src, el.dst, el.n, False, int(s), d)


def test_scipy_chung_lu_directed():
    el = graphgen.chung_lu(5000, 30000, 4.0, seed=8)
    g = oracle.OracleGraph.from_edgelist(el)
    seeds = graphgen.draw_seeds(el, 10, seed=6)
    ref = _scipy_distances(el, seeds)
    for i, s in enumerate(seeds):
        d = g.distances(int(s), ALL)
        assert np.array_equal(d, ref[i])
        bfs_tree_valid(el.src, el.dst, el.n, True, int(s), d)


def test_tree_checker_catches_planted_errors():
    """The level checks above reject a distance vector with one wrong entry."""
    el = graphgen.rmat(10, 8, seed=2)
    g = oracle.OracleGraph.from_edgelist(el)
    s = int(graphgen.draw_seeds(el, 1, seed=1)[0])
    d = g.distances(s, ALL)
    far = int(np.argmax(d))
    for bad in (d[far] + 1, d[far] - 1, -1):
        e = d.copy()
        e[far] = bad
        with pytest.raises(AssertionError):
            bfs_tree_valid(el.src, el.dst, el.n, False, s, e)
