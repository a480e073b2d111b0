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
