"""Parity at the full plain-path workload size: R-MAT scale 21, edge factor 32
(a/b/c/d = 0.57/0.19/0.19/0.05, symmetrised, self-loops and duplicates
dropped), 300 seeds at k = 1 and 2 and 10 seeds at k = 3 and 6, the paper's
seed protocol (Section III).  Plain GPU counts are compared with the oracle for
every one of those queries; the batched path is compared with the plain path
for 1024 seeds and with the oracle on a sample."""
import time

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-scale21]", *a, flush=True)


@pytest.fixture(scope="module")
def g1():
    t = time.time()
    el = graphgen.rmat(21, 32, seed=1)
    _say("generated", el.m, "tuples in", round(time.time() - t, 1), "s")
    t = time.time()
    og = oracle.OracleGraph.from_edgelist(el)
    _say("oracle adjacency in", round(time.time() - t, 1), "s")
    s12 = graphgen.draw_seeds(el, 300, seed=7, stream=0)
    s36 = graphgen.draw_seeds(el, 10, seed=7, stream=1)
    import paper_1905_01294_amd as K
    t = time.time()
    g = K.Graph.from_edgelist(el)
    _say("device graph in", round(time.time() - t, 1), "s", g.num_arcs, "arcs")
    yield el, og, g, s12, s36, K
    g.free()


def test_shape(g1):
    el, og, g, *_ = g1
    assert g.num_arcs == og.num_arcs
    assert np.array_equal(g.degrees(), og.degrees())


@pytest.mark.parametrize("k", [1, 2])
def test_plain_300_seeds(g1, k):
    el, og, g, s12, s36, K = g1
    t = time.time()
    c, te = g.count(s12, k, with_te=True)
    _say("gpu k", k, round(time.time() - t, 2), "s")
    oc, ote = og.count(s12, k)
    assert np.array_equal(c, oc)
    assert np.array_equal(te, ote)


@pytest.mark.parametrize("k", [3, 6])
def test_plain_10_seeds(g1, k):
    el, og, g, s12, s36, K = g1
    c, te = g.count(s36, k, with_te=True)
    t = time.time()
    oc, ote = og.count(s36, k)
    _say("oracle k", k, round(time.time() - t, 1), "s")
    assert np.array_equal(c, oc)
    assert np.array_equal(te, ote)


_ORACLE = {}


def _oracle_counts(og, seeds, k):
    """Oracle counts and traversed edges of the protocol seeds, computed once per (seeds, k)."""
    key = (seeds.tobytes(), k)
    if key not in _ORACLE:
        _ORACLE[key] = og.count(seeds, k)
    return _ORACLE[key]


@pytest.mark.parametrize("mode", ["push", "pull"])
@pytest.mark.parametrize("k", [1, 2, 3, 6])
def test_forced_directions_match_oracle(g1, mode, k):
    """Every hop top-down, or every hop bottom-up, on the ten deep protocol seeds: counts and traversed
    edges equal the oracle's at each protocol depth."""
    el, og, g, s12, s36, K = g1
    oc, ote = _oracle_counts(og, s36, k)
    g.set_option(K.KHOP_OPT_DIRECTION, K.KHOP_DIR_PUSH if mode == "push" else K.KHOP_DIR_PULL)
    try:
        c, te = g.count(s36, k, with_te=True)
    finally:
        g.set_option(K.KHOP_OPT_DIRECTION, K.KHOP_DIR_AUTO)
    assert np.array_equal(c, oc) and np.array_equal(te, ote)


@pytest.mark.parametrize("per", [64, 256, 1024])
def test_batched_1024_seeds(g1, per):
    """All 1024 seeds at k = 3 and 6, at 64, 256 and 1024 seeds per launch: every count equals the plain
    path's, and a sample equals the oracle's at both depths."""
    el, og, g, s12, s36, K = g1
    seeds = graphgen.draw_seeds(el, 1024, seed=11)
    g.set_option(K.KHOP_OPT_BATCH_SEEDS, per)
    try:
        for k in (3, 6):
            t = time.time()
            b = g.count_batched(seeds, np.full(len(seeds), k))
            _say("batched", per, "k", k, round(time.time() - t, 3), "s")
            assert np.array_equal(b, g.count(seeds, k))
            sample = seeds[::341]  # seeds 0, 341, 682, 1023: one in each quarter of the launch's words
            assert np.array_equal(b[::341], _oracle_counts(og, sample, k)[0])
    finally:
        g.set_option(K.KHOP_OPT_BATCH_SEEDS, 1024)


def test_batched_mixed_protocol(g1):
    """The whole plain protocol (300 at k=1, 300 at k=2, 10 at k=3, 10 at k=6) in batched launches."""
    el, og, g, s12, s36, K = g1
    seeds = np.concatenate([s12, s12, s36, s36])
    ks = np.concatenate([np.full(300, 1), np.full(300, 2), np.full(10, 3), np.full(10, 6)]).astype(np.int32)
    b = g.count_batched(seeds, ks)
    expect = np.concatenate([og.count(s12, 1)[0], og.count(s12, 2)[0], g.count(s36, 3), g.count(s36, 6)])
    assert np.array_equal(b, expect)
