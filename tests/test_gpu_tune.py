"""The autotuner changes only speed: counts after tuning still equal the oracle's."""
import os
import time

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def K():
    import paper_1905_01294_amd as K
    return K


def test_autotune_then_parity(K, g0, g0_oracle, tmp_path):
    os.environ["KHOP_TUNE_CACHE"] = str(tmp_path / "tune.txt")
    el, seeds = g0
    g = K.Graph.from_edgelist(el)
    t = time.time()
    g.autotune(0)
    first = time.time() - t
    opts = {o: g.get_option(o) for o in (K.KHOP_OPT_ALPHA, K.KHOP_OPT_BETA, K.KHOP_OPT_PULL_LIGHT,
                                         K.KHOP_OPT_PULL_HEAVY, K.KHOP_OPT_BATCH_SEEDS, K.KHOP_OPT_BATCH_HEAVY)}
    assert opts[K.KHOP_OPT_BATCH_SEEDS] in (64, 128, 256, 512, 1024)
    for k in (1, 2, 3, 6):
        oc, ote = g0_oracle.count(seeds, k)
        c, te = g.count(seeds, k, with_te=True)
        assert np.array_equal(c, oc) and np.array_equal(te, ote)
        assert np.array_equal(g.count_batched(seeds, np.full(len(seeds), k)), oc)
    # a second graph with the same content takes the cached result
    g2 = K.Graph.from_edgelist(el)
    t = time.time()
    g2.autotune(0)
    assert time.time() - t < max(first, 0.05)
    assert {o: g2.get_option(o) for o in opts} == opts
    assert (tmp_path / "tune.txt").exists()
    g.free()
    g2.free()


def test_autotune_fixed_batch_size(K, tmp_path):
    os.environ["KHOP_TUNE_CACHE"] = str(tmp_path / "tune2.txt")
    el = graphgen.chung_lu(30_000, 300_000, 4.0, seed=2)
    g = K.Graph.from_edgelist(el)
    og = oracle.OracleGraph.from_edgelist(el)
    g.autotune(256)
    assert g.get_option(K.KHOP_OPT_BATCH_SEEDS) == 256
    seeds = graphgen.draw_seeds(el, 100, seed=1)
    for k in (1, 3):
        oc, _ = og.count(seeds, k)
        assert np.array_equal(g.count(seeds, k), oc)
        assert np.array_equal(g.count_batched(seeds, np.full(len(seeds), k)), oc)
    with pytest.raises(K.KhopError):
        g.autotune(100)
    g.free()


def test_bad_preset_is_retuned(K, tmp_path):
    """Start from deliberately poor settings: the search moves them, counts stay equal to the oracle's, and
    the cache file records every tuned option."""
    os.environ["KHOP_TUNE_CACHE"] = str(tmp_path / "tune3.txt")
    el = graphgen.rmat(16, 16, seed=4)
    g = K.Graph.from_edgelist(el)
    og = oracle.OracleGraph.from_edgelist(el)
    bad = {K.KHOP_OPT_ALPHA: 1, K.KHOP_OPT_BETA: 1, K.KHOP_OPT_PULL_LIGHT: 1, K.KHOP_OPT_PUSH_ATOMIC: 0,
           K.KHOP_OPT_BATCH_PUSH: 1 << 30, K.KHOP_OPT_PLAIN_GRID: 1, K.KHOP_OPT_BATCH_GRID: 1,
           K.KHOP_OPT_BATCH_HEAVY: 1 << 30}
    for o, v in bad.items():
        g.set_option(o, v)
    g.autotune(0)
    assert K.khop_autotune_seconds() > 0  # searched, not read from a cache
    tuned = {o: g.get_option(o) for o in bad}
    assert sum(tuned[o] != v for o, v in bad.items()) >= 3, tuned
    seeds = graphgen.draw_seeds(el, 64, seed=5)
    for k in (1, 2, 3, 6):
        oc, ote = og.count(seeds, k)
        c, te = g.count(seeds, k, with_te=True)
        assert np.array_equal(c, oc) and np.array_equal(te, ote)
        assert np.array_equal(g.count_batched(seeds, np.full(len(seeds), k)), oc)
    lines = (tmp_path / "tune3.txt").read_text().split("\n")
    line = [x for x in lines if f":{el.n}:0" in x.split(" ")[0]][0].split()
    assert len(line) == 12  # the key and eleven settings
    assert line[0].split(":")[0] == K.khop_version().split("sources ")[1].rstrip(")")
    g.free()
