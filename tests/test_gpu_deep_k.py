"""GPU parity at depths far past a graph's eccentricity: the plain path's
queries deeper than its pipelined form (run as searches that stop once their
frontier is empty), batched traversals longer than the per-level record ring,
and the label-filtered forms, against the CPU oracle and closed forms."""
import numpy as np
import pytest

import oracle
from tests import graphs

pytestmark = pytest.mark.gpu

BIG = 2**31 - 1


def _say(*a):
    print("[gpu-deep]", *a, flush=True)


@pytest.fixture(scope="module")
def K():
    import paper_1905_01294_amd as K
    return K


@pytest.fixture(scope="module")
def path5000(K):
    src, dst, n, directed = graphs.path(5000)
    g = K.Graph(src, dst, n, directed)
    yield g, oracle.OracleGraph(src, dst, n, directed)
    g.free()


def _path_count(n, s, k):
    return min(k, s) + min(k, n - 1 - s)


@pytest.mark.parametrize("k", [31, 32, 33, 100, 4095, 4096, 4097, 4999, 5000, 6000, BIG])
def test_plain_path_graph_deep(K, path5000, k):
    g, o = path5000
    seeds = np.array([0, 17, 2500, 4999, 4000], np.int32)
    _say("plain path5000", k)
    c, te = g.count(seeds, k, with_te=True)
    assert [int(x) for x in c] == [_path_count(5000, int(s), k) for s in seeds]
    oc, ote = o.count(seeds, k)
    assert np.array_equal(c, oc) and np.array_equal(te, ote)


@pytest.mark.parametrize("k", [33, 5000, BIG])
def test_plain_dev_deep_with_invalid_seed(K, path5000, k):
    import torch
    g, o = path5000
    seeds = np.array([0, -1, 2500, 5000, 4999], np.int32)
    d_s = torch.from_numpy(seeds).cuda()
    d_c = torch.empty(len(seeds), dtype=torch.int64, device="cuda")
    d_t = torch.empty(len(seeds), dtype=torch.int64, device="cuda")
    _say("plain dev path5000 invalid", k)
    g.count_dev(d_s, k, d_c, d_t)
    torch.cuda.synchronize()
    c, t = d_c.cpu().numpy(), d_t.cpu().numpy()
    for i, s in enumerate(seeds):
        if 0 <= s < 5000:
            oc, ote = o.count(np.array([s], np.int32), k)
            assert (c[i], t[i]) == (oc[0], ote[0])
        else:
            assert (c[i], t[i]) == (-1, -1)


def test_batched_path_graph_past_ring(K, path5000):
    """5000 levels in one batch: the per-level records wrap their 4096-slot ring."""
    g, o = path5000
    seeds = np.array([0, 4999, 2500, 0, 1234, 7, 4998, 3, 100, 0], np.int32)
    ks = np.array([5000, BIG, 4097, 4095, 3, 0, 1, 2, 4096, 6000], np.int32)
    _say("batched path5000 mixed deep")
    got = g.count_batched(seeds, ks)
    assert [int(x) for x in got] == [_path_count(5000, int(s), int(k)) for s, k in zip(seeds, ks)]


def test_batched_directed_cycle_full_reach(K):
    src, dst, n, directed = graphs.cycle(6000, directed=True)
    g = K.Graph(src, dst, n, directed)
    try:
        seeds = np.array([0, 5999, 3000], np.int32)
        ks = np.array([BIG, 5999, 5998], np.int32)
        _say("batched directed cycle 6000")
        assert [int(x) for x in g.count_batched(seeds, ks)] == [5999, 5999, 5998]
        c = g.count(seeds, BIG)
        assert [int(x) for x in c] == [5999, 5999, 5999]
    finally:
        g.free()


def test_random_components_deep_every_path(K):
    """Many components: plain, batched and label-filtered counts at huge k equal the oracle's reach."""
    rng = np.random.default_rng(2026)
    src, dst, n, directed = graphs.random_graph(rng, 30000, 26000, False)
    g = K.Graph(src, dst, n, directed)
    o = oracle.OracleGraph(src, dst, n, directed)
    try:
        seeds = rng.integers(0, n, size=48).astype(np.int32)
        for k in (40, 1000, BIG):
            _say("random components", k)
            oc, ote = o.count(seeds, k)
            c, te = g.count(seeds, k, with_te=True)
            assert np.array_equal(c, oc) and np.array_equal(te, ote)
            assert np.array_equal(g.count_batched(seeds, np.full(len(seeds), k, np.int32)), oc)
        lab = rng.random(n) < 0.7
        for k in (50, BIG):
            expect = np.array([o.khop_filtered(int(s), k, lab)[0] for s in seeds])
            assert np.array_equal(g.count_labeled(seeds, k, lab), expect)
            assert np.array_equal(g.count_batched_labeled(seeds, np.full(len(seeds), k, np.int32), lab), expect)
    finally:
        g.free()
