"""Parity on the full-size power-law graph standing in for the paper's Twitter
dataset (Section III: 41.6M vertices, 1.47B edges): a directed Chung-Lu graph
with those sizes and out/in-degree exponent 2, followed along out-edges.
The oracle checks all 300 seeds at k = 1 and 2 and a sample of the 10 at
k = 3 and 6 (a deep query costs it seconds); the batched path must equal the
plain path on every query, including the 256-seed batch at k = 3."""
import time

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-twitter]", *a, flush=True)


@pytest.fixture(scope="module")
def g2():
    t = time.time()
    el = graphgen.twitter_like(seed=1)
    _say("generated", el.m, "tuples in", round(time.time() - t, 1), "s")
    import paper_1905_01294_amd as K
    t = time.time()
    g = K.Graph.from_edgelist(el)
    _say("device graph in", round(time.time() - t, 1), "s:", g.num_arcs, "arcs")
    seeds = graphgen.draw_seeds(el, 300, seed=7, stream=0)
    seeds36 = graphgen.draw_seeds(el, 10, seed=7, stream=1)
    t = time.time()
    og = oracle.OracleGraph.from_edgelist(el)
    _say("oracle adjacency in", round(time.time() - t, 1), "s")
    yield el, g, og, seeds, seeds36, K
    g.free()


def test_shape(g2):
    el, g, og, *_ = g2
    assert g.n == 41_600_000 and g.directed
    assert g.num_arcs == og.num_arcs
    assert 1.0e9 < g.num_arcs <= 1.47e9


def _oracle_many(og, seeds, k, threads=8):
    """The oracle's counts and traversed edges, its queries spread over host threads (each query
    allocates and clears its own per-vertex arrays, so they are independent)."""
    from concurrent.futures import ThreadPoolExecutor
    parts = np.array_split(np.asarray(seeds, np.int32), threads)
    with ThreadPoolExecutor(threads) as ex:
        res = list(ex.map(lambda p: og.count(p, k), parts))
    return np.concatenate([r[0] for r in res]), np.concatenate([r[1] for r in res])


@pytest.mark.parametrize("k", [1, 2])
def test_protocol_k12(g2, k):
    """All 300 protocol seeds against the oracle, plain and batched."""
    el, g, og, seeds, _, K = g2
    c, te = g.count(seeds, k, with_te=True)
    t = time.time()
    oc, ote = _oracle_many(og, seeds, k)
    _say("k", k, "oracle on all 300 seeds in", round(time.time() - t, 1), "s")
    assert np.array_equal(c, oc) and np.array_equal(te, ote)
    assert np.array_equal(g.count_batched(seeds, np.full(300, k)), c)


@pytest.mark.parametrize("k", [3, 6])
def test_protocol_k36(g2, k):
    el, g, og, _, seeds36, K = g2
    c, te = g.count(seeds36, k, with_te=True)
    sample = seeds36[:4] if k == 3 else seeds36[:2]
    oc, ote = og.count(sample, k)
    _say("k", k, "oracle sample", len(sample))
    assert np.array_equal(c[:len(sample)], oc) and np.array_equal(te[:len(sample)], ote)
    assert np.array_equal(g.count_batched(seeds36, np.full(10, k)), c)


def test_batched_256_at_k3(g2):
    el, g, og, seeds, _, K = g2
    s256 = graphgen.draw_seeds(el, 256, seed=13)
    b = g.count_batched(s256, np.full(256, 3))
    assert np.array_equal(b, g.count(s256, 3))
    assert np.array_equal(b[:3], og.count(s256[:3], 3)[0])


def test_full_depth_distances_and_sets(g2):
    """Breadth-first distances with no depth limit, level sizes and a k = 2
    neighborhood as ids, each against the oracle, from two seeds."""
    el, g, og, seeds, _, K = g2
    for s in seeds[:2]:
        t = time.time()
        dist, count, depth = g.bfs(int(s))
        _say("bfs seed", int(s), "depth", depth, "reach", count + 1, round(time.time() - t, 2), "s")
        ref = og.distances(int(s), 2**31 - 1)
        assert np.array_equal(dist, ref)
        assert count == int((ref > 0).sum()) and depth == int(ref.max())
        assert np.array_equal(g.levels(int(s), 6), og.khop(int(s), 6)[2])
        assert np.array_equal(g.neighborhood(int(s), 2), np.nonzero((ref >= 1) & (ref <= 2))[0])
