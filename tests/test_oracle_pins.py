"""Pins of the CPU oracle to facts that do not come from the oracle itself.

The paper prints no worked example (its only figure did not survive), so the
count -- |{v : 1 <= dist(s, v) <= k}|, the k-hop neighborhood count of
Section III computed by semiring products as in Section II -- is pinned by
  * brute force: boolean powers of the dense adjacency matrix (walks of length
    at most k reach exactly the vertices at distance at most k);
  * closed forms on path, cycle, star, complete, bipartite, tree, grid and
    hypercube graphs, directed paths and cycles;
  * independent library routines (scipy's csgraph shortest paths, networkx);
  * invariants: monotone in k, at most n-1, count(1) = degree, the component
    (or reach) size minus one past the eccentricity, symmetry of undirected
    neighborhoods, and invariance under tuple order, duplicate tuples, added
    self-loops and vertex relabelling.
"""
import json
import os
from math import comb

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import graphgen
import oracle
from tests import graphs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def og(src, dst, n, directed):
    return oracle.OracleGraph(src, dst, n, directed)


def brute(src, dst, n, directed, s, k):
    """(count, te, level_counts) from boolean matrix powers of the dense adjacency."""
    a = graphs.dense_adjacency(src, dst, n, directed).astype(np.int64)
    reach = np.zeros(n, dtype=bool)
    reach[s] = True
    sets = [reach.copy()]
    for _ in range(k):
        reach = reach | ((reach.astype(np.int64) @ a) > 0)
        sets.append(reach.copy())
    count = int(sets[k].sum()) - 1
    a_nl = a.copy()
    np.fill_diagonal(a_nl, 0)
    outdeg = (a_nl > 0).sum(axis=1)
    te = int(outdeg[sets[k - 1]].sum()) if k >= 1 else 0
    levels = [int(sets[l].sum() - sets[l - 1].sum()) for l in range(1, k + 1)]
    return count, te, levels


# ---------------------------------------------------------------- brute force


@settings(max_examples=1500, deadline=None)
@given(n=st.integers(1, 40), m=st.integers(0, 140), directed=st.booleans(), k=st.integers(0, 8),
       rseed=st.integers(0, 2**32 - 1))
def test_brute_force_random(n, m, directed, k, rseed):
    rng = np.random.default_rng(rseed)
    src, dst, n, directed = graphs.random_graph(rng, n, m, directed)
    g = og(src, dst, n, directed)
    s = int(rng.integers(0, n))
    c, te, lv = g.khop(s, k)
    bc, bte, blv = brute(src, dst, n, directed, s, k)
    assert c == bc
    assert te == bte
    assert list(lv) == blv


@pytest.mark.parametrize("n,m,directed", [(256, 300, False), (256, 600, True), (200, 2000, False),
                                          (128, 128, True), (256, 256, False)])
def test_brute_force_larger(n, m, directed):
    rng = np.random.default_rng(n * 7 + m)
    src, dst, n, directed = graphs.random_graph(rng, n, m, directed)
    g = og(src, dst, n, directed)
    for s in rng.integers(0, n, size=6):
        for k in (1, 2, 3, 6, 12):
            c, te, _ = g.khop(int(s), k)
            bc, bte, _ = brute(src, dst, n, directed, int(s), k)
            assert (c, te) == (bc, bte)


# ---------------------------------------------------------------- closed forms

KS = [0, 1, 2, 3, 4, 6, 10, 50]


@pytest.mark.parametrize("n", [1, 2, 3, 7, 30])
def test_path(n):
    g = og(*graphs.path(n))
    for s in range(n):
        for k in KS:
            assert g.khop(s, k)[0] == min(k, s) + min(k, n - 1 - s)


@pytest.mark.parametrize("n", [3, 4, 9, 20])
def test_cycle(n):
    g = og(*graphs.cycle(n))
    for s in (0, n // 2, n - 1):
        for k in KS:
            assert g.khop(s, k)[0] == min(2 * k, n - 1)


@pytest.mark.parametrize("n", [2, 5, 40])
def test_star(n):
    g = og(*graphs.star(n))
    for k in KS:
        assert g.khop(0, k)[0] == (n - 1) * (k >= 1)
        for leaf in (1, n - 1):
            assert g.khop(leaf, k)[0] == (k >= 1) + (n - 2) * (k >= 2)


@pytest.mark.parametrize("n", [1, 2, 6, 25])
def test_complete(n):
    g = og(*graphs.complete(n))
    for s in range(0, n, max(1, n // 4)):
        for k in KS:
            assert g.khop(s, k)[0] == (n - 1) * (k >= 1)


@pytest.mark.parametrize("a,b", [(1, 1), (3, 5), (7, 2)])
def test_complete_bipartite(a, b):
    g = og(*graphs.complete_bipartite(a, b))
    for k in KS:
        for s in range(a):
            assert g.khop(s, k)[0] == b * (k >= 1) + (a - 1) * (k >= 2)
        for s in range(a, a + b):
            assert g.khop(s, k)[0] == a * (k >= 1) + (b - 1) * (k >= 2)


@pytest.mark.parametrize("depth", [0, 1, 4, 8])
def test_binary_tree_root(depth):
    g = og(*graphs.binary_tree(depth))
    for k in KS:
        assert g.khop(0, k)[0] == 2 ** (min(k, depth) + 1) - 2


@pytest.mark.parametrize("r,c", [(1, 1), (1, 6), (4, 4), (3, 9)])
def test_grid_corner(r, c):
    g = og(*graphs.grid(r, c))
    for k in KS:
        expect = sum(1 for i in range(r) for j in range(c) if 1 <= i + j <= k)
        assert g.khop(0, k)[0] == expect


@pytest.mark.parametrize("d", [1, 3, 6])
def test_hypercube(d):
    g = og(*graphs.hypercube(d))
    for s in (0, (1 << d) - 1):
        for k in KS:
            assert g.khop(s, k)[0] == sum(comb(d, i) for i in range(1, min(k, d) + 1))


@pytest.mark.parametrize("n", [1, 2, 8])
def test_directed_path_and_cycle(n):
    gp = og(*graphs.path(n, directed=True))
    gc = og(*graphs.cycle(n, directed=True))
    for s in range(n):
        for k in KS:
            assert gp.khop(s, k)[0] == min(k, n - 1 - s)
            assert gc.khop(s, k)[0] == min(k, n - 1)


def test_isolated_and_k0():
    g = og(np.array([0], np.int32), np.array([1], np.int32), 5, False)
    for k in KS:
        assert g.khop(3, k)[0] == 0
    for s in range(5):
        assert g.khop(s, 0)[:2] == (0, 0)


def test_self_loops_and_duplicates_carry_no_adjacency():
    src = np.array([0, 0, 0, 1, 1, 2, 2], np.int32)
    dst = np.array([0, 1, 1, 1, 0, 2, 2], np.int32)
    g = og(src, dst, 3, False)
    assert g.num_arcs == 2
    assert list(g.degrees()) == [1, 1, 0]
    assert g.khop(2, 5)[0] == 0
    assert g.khop(0, 5)[:2] == (1, 2)  # te: seed and its one neighbor, degree 1 each
    assert g.khop(0, 1)[:2] == (1, 1)


def test_golden_textbook_graphs():
    with open(os.path.join(GOLDEN, "textbook_graphs.json")) as f:
        cases = json.load(f)["cases"]
    makers = {"petersen": graphs.petersen, "hypercube4": lambda: graphs.hypercube(4),
              "grid3x4": lambda: graphs.grid(3, 4), "cycle7": lambda: graphs.cycle(7),
              "directed_cycle5": lambda: graphs.cycle(5, directed=True)}
    for case in cases:
        g = og(*makers[case["graph"]]())
        for k, expect in enumerate(case["counts_by_k"]):
            assert g.khop(case["seed"], k)[0] == expect, (case["graph"], k)


# ---------------------------------------------------------------- library routines


def _scipy_counts(el, seeds, k):
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import dijkstra
    n = el.n
    keep = el.src != el.dst
    a = coo_matrix((np.ones(int(keep.sum())), (el.src[keep], el.dst[keep])), shape=(n, n)).tocsr()
    a.data[:] = 1.0
    d = dijkstra(a, directed=el.directed, indices=np.asarray(seeds), unweighted=True, limit=k + 0.5)
    return ((d > 0) & np.isfinite(d)).sum(axis=1)


def test_scipy_csgraph_g0_every_nonisolated_seed(g0, g0_oracle):
    el, _ = g0
    seeds = np.nonzero(g0_oracle.degrees() > 0)[0].astype(np.int32)
    for k in (1, 2, 3, 6):
        ours, _ = g0_oracle.count(seeds, k)
        assert np.array_equal(ours, _scipy_counts(el, seeds, k))


def test_networkx_rmat14():
    import networkx as nx
    el = graphgen.rmat(14, 16, seed=3)
    g = oracle.OracleGraph.from_edgelist(el)
    G = nx.Graph()
    G.add_nodes_from(range(el.n))
    G.add_edges_from((int(u), int(v)) for u, v in zip(el.src, el.dst) if u != v)
    seeds = graphgen.draw_seeds(el, 12, seed=11)
    for k in (1, 2, 3, 6):
        ours, _ = g.count(seeds, k)
        ref = [len(nx.single_source_shortest_path_length(G, int(s), cutoff=k)) - 1 for s in seeds]
        assert list(ours) == ref


def test_scipy_directed_chung_lu_small():
    el = graphgen.chung_lu(5000, 60000, 4.0, seed=5)
    g = oracle.OracleGraph.from_edgelist(el)
    seeds = graphgen.draw_seeds(el, 40, seed=2)
    for k in (1, 2, 3, 6):
        ours, _ = g.count(seeds, k)
        assert np.array_equal(ours, _scipy_counts(el, seeds, k))


# ---------------------------------------------------------------- invariants


def _components(src, dst, n):
    parent = list(range(n))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    for u, v in zip(src.tolist(), dst.tolist()):
        ru, rv = find(u), find(v)
        if ru != rv:
            parent[ru] = rv
    roots = [find(v) for v in range(n)]
    size = {}
    for r in roots:
        size[r] = size.get(r, 0) + 1
    return [size[r] for r in roots]


def _reach_dfs(src, dst, n, s):
    adj = [[] for _ in range(n)]
    for u, v in zip(src.tolist(), dst.tolist()):
        adj[u].append(v)
    seen = {s}
    stack = [s]
    while stack:
        u = stack.pop()
        for v in adj[u]:
            if v not in seen:
                seen.add(v)
                stack.append(v)
    return len(seen)


def test_invariants_g0(g0, g0_oracle):
    el, seeds = g0
    deg = g0_oracle.degrees()
    comp = _components(el.src, el.dst, el.n)
    for s in seeds:
        prev = 0
        counts = []
        for k in range(0, 12):
            c, _, lv = g0_oracle.khop(int(s), k)
            assert c >= prev and c <= el.n - 1
            assert (lv >= 0).all()
            nz = np.nonzero(lv == 0)[0]
            if nz.size:
                assert (lv[nz[0]:] == 0).all()
            counts.append(c)
            prev = c
        assert counts[1] == deg[s]
        assert counts[-1] == comp[s] - 1


def test_directed_reach_matches_dfs():
    el = graphgen.chung_lu(3000, 9000, 3.0, seed=9)
    g = oracle.OracleGraph.from_edgelist(el)
    for s in graphgen.draw_seeds(el, 15, seed=4):
        assert g.khop(int(s), 3000)[0] == _reach_dfs(el.src, el.dst, el.n, int(s)) - 1
        assert g.khop(int(s), 1)[0] == g.degrees()[s]


def test_undirected_symmetry():
    rng = np.random.default_rng(5)
    src, dst, n, d = graphs.random_graph(rng, 60, 90, False)
    g = og(src, dst, n, d)
    for k in (1, 2, 3):
        dist = np.stack([g.distances(s, k) for s in range(n)])
        within = (dist >= 1)
        assert np.array_equal(within, within.T)


def test_input_invariance(g0, g0_oracle):
    el, seeds = g0
    rng = np.random.default_rng(17)
    order = rng.permutation(el.m)
    dup = rng.integers(0, el.m, size=el.m // 3)
    loops = rng.integers(0, el.n, size=200).astype(np.int32)
    src2 = np.concatenate([el.src[order], el.src[dup], loops])
    dst2 = np.concatenate([el.dst[order], el.dst[dup], loops])
    g2 = og(src2, dst2, el.n, False)
    perm = graphgen.permutation(el.n, seed=99, tag=77)
    g3 = og(perm[el.src], perm[el.dst], el.n, False)
    for k in (1, 2, 3, 6):
        a, ta = g0_oracle.count(seeds, k)
        b, tb = g2.count(seeds, k)
        c, tc = g3.count(perm[seeds], k)
        assert np.array_equal(a, b) and np.array_equal(a, c)
        assert np.array_equal(ta, tb) and np.array_equal(ta, tc)


def test_te_is_degree_sum_of_inner_levels(g0, g0_oracle):
    el, seeds = g0
    deg = g0_oracle.degrees()
    for s in seeds[:8]:
        for k in (1, 2, 3, 6):
            d = g0_oracle.distances(int(s), k)
            _, te, _ = g0_oracle.khop(int(s), k)
            assert te == int(deg[(d >= 0) & (d <= k - 1)].sum())


def test_oracle_rejects_bad_input():
    with pytest.raises(ValueError):
        og(np.array([0], np.int32), np.array([5], np.int32), 3, False)
    g = og(*graphs.path(4))
    with pytest.raises(ValueError):
        g.khop(4, 1)
    with pytest.raises(ValueError):
        g.khop(0, -1)


def test_g0_regression_fixture(g0, g0_oracle):
    """The stored scale-10 counts were written by tests/golden/make_g0_fixture.py from the oracle."""
    el, seeds = g0
    with open(os.path.join(GOLDEN, "g0_rmat10_counts.json")) as f:
        fx = json.load(f)
    assert fx["seeds"] == seeds.tolist()
    for k, row in fx["counts"].items():
        c, te = g0_oracle.count(seeds, int(k))
        assert c.tolist() == row
        assert te.tolist() == fx["te"][k]
