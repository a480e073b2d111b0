"""GPU parity of exactly-l level sizes (khop_levels) and of the k-hop
neighborhood returned as ascending vertex ids (khop_neighborhood) against the
CPU oracle, bit exact: the oracle's per-level counts, and the ids of its
vertices at distance 1..k.  Sizes span one word to many 256-word blocks of the
set kernels with a ragged last word; buffers too small for the set, the device
entry points and R-MAT scale 21 are covered."""
import numpy as np
import pytest

import graphgen
import oracle
from tests import graphs

pytestmark = pytest.mark.gpu

ALL = 2**31 - 1
MODES = ("auto", "push", "pull")


def _say(*a):
    print("[gpu-sets]", *a, flush=True)


@pytest.fixture(scope="module")
def K():
    import paper_1905_01294_amd as K
    return K


def _set_mode(K, g, mode):
    g.set_option(K.KHOP_OPT_DIRECTION, {"auto": K.KHOP_DIR_AUTO, "push": K.KHOP_DIR_PUSH,
                                        "pull": K.KHOP_DIR_PULL}[mode])


def _ref_set(og, s, k):
    d = og.distances(int(s), ALL if k < 0 else k)
    return np.nonzero(d >= 1)[0].astype(np.int32)


@pytest.fixture(scope="module")
def g0_gpu(K, g0):
    el, _ = g0
    return K.Graph.from_edgelist(el)


@pytest.mark.parametrize("mode", MODES)
def test_g0_levels(K, g0, g0_gpu, g0_oracle, mode):
    el, seeds = g0
    _set_mode(K, g0_gpu, mode)
    for s in seeds:
        for k in (1, 2, 3, 6, 12):
            lv = g0_gpu.levels(int(s), k)
            assert np.array_equal(lv, g0_oracle.khop(int(s), k)[2]), (mode, s, k)
    _set_mode(K, g0_gpu, "auto")


@pytest.mark.parametrize("mode", MODES)
def test_g0_neighborhoods(K, g0, g0_gpu, g0_oracle, mode):
    el, seeds = g0
    _set_mode(K, g0_gpu, mode)
    for s in seeds:
        for k in (0, 1, 2, 3, -1):
            ids = g0_gpu.neighborhood(int(s), k)
            assert np.array_equal(ids, _ref_set(g0_oracle, s, k)), (mode, s, k)
    c = g0_gpu.count(seeds, 2)
    assert list(c) == [len(g0_gpu.neighborhood(int(s), 2)) for s in seeds]
    _set_mode(K, g0_gpu, "auto")


def test_small_buffers(K, g0, g0_gpu, g0_oracle):
    el, seeds = g0
    s = int(seeds[0])
    ref = _ref_set(g0_oracle, s, 3)
    assert ref.size > 4
    for cap in (0, 1, ref.size // 2, ref.size - 1, ref.size, ref.size + 7):
        ids, c = g0_gpu.neighborhood(s, 3, capacity=cap)
        assert c == ref.size
        assert np.array_equal(ids, ref[:cap])


@pytest.mark.parametrize("directed", [False, True])
def test_multi_block_ragged(K, directed):
    """n = 70001: 1094 words, five blocks of the set kernels, a ragged last word."""
    rng = np.random.default_rng(404 + directed)
    src, dst, n, d = graphs.random_graph(rng, 70001, 120000, directed)
    g = K.Graph(src, dst, n, d)
    og = oracle.OracleGraph(src, dst, n, d)
    seeds = list(rng.integers(0, n, size=5)) + [n - 1, 0]
    for s in seeds:
        for k in (1, 3, 8, -1):
            ids = g.neighborhood(int(s), k)
            assert np.array_equal(ids, _ref_set(og, s, k)), (s, k)
        lv = g.levels(int(s), 8)
        assert np.array_equal(lv, og.khop(int(s), 8)[2]), s
    g.free()


def test_closed_forms(K):
    src, dst, n, d = graphs.grid(40, 70)
    g = K.Graph(src, dst, n, d)
    # from the corner, level l of a 40 x 70 grid holds the cells with i + j = l
    lv = g.levels(0, 120)
    expect = [sum(1 for i in range(40) if 0 <= l - i < 70) for l in range(1, 121)]
    assert list(lv) == expect
    ids = g.neighborhood(0, 2)
    assert list(ids) == sorted([1, 2, 70, 71, 140])
    g.free()


def test_errors(K, g0_gpu):
    n = g0_gpu.n
    for bad in (-1, n):
        with pytest.raises(K.KhopError):
            g0_gpu.levels(bad, 2)
        with pytest.raises(K.KhopError):
            g0_gpu.neighborhood(bad, 2)
    with pytest.raises(K.KhopError):
        g0_gpu.levels(0, -1)
    assert g0_gpu.levels(0, 0).size == 0


def test_device_forms(K, g0, g0_gpu, g0_oracle):
    import torch
    el, seeds = g0
    d_ids = torch.empty(el.n, dtype=torch.int32, device="cuda")
    d_count = torch.empty(1, dtype=torch.int64, device="cuda")
    d_lv = torch.empty(6, dtype=torch.int64, device="cuda")
    for s in seeds[:8]:
        for k in (2, -1):
            g0_gpu.neighborhood_dev(int(s), k, d_ids, d_count)
            torch.cuda.synchronize()
            c = int(d_count.item())
            assert np.array_equal(d_ids[:c].cpu().numpy(), _ref_set(g0_oracle, s, k))
        g0_gpu.levels_dev(int(s), 6, d_lv)
        torch.cuda.synchronize()
        assert np.array_equal(d_lv.cpu().numpy(), g0_oracle.khop(int(s), 6)[2])


@pytest.fixture(scope="module")
def g1(K):
    el = graphgen.rmat(21, 32, seed=1)
    og = oracle.OracleGraph.from_edgelist(el)
    g = K.Graph.from_edgelist(el)
    yield el, og, g
    g.free()


def test_rmat21(K, g1):
    el, og, g = g1
    for s in graphgen.draw_seeds(el, 3, seed=7, stream=3):
        ids = g.neighborhood(int(s), 2)
        ref = _ref_set(og, s, 2)
        _say("rmat21 seed", int(s), "k=2 neighborhood", ref.size)
        assert np.array_equal(ids, ref)
        assert np.array_equal(g.levels(int(s), 6), og.khop(int(s), 6)[2])
