"""GPU parity of the batched multi-source path (per-vertex seed bitsets) against
the CPU oracle and the plain GPU path, bit exact, with mixed k in one batch,
with hops forced top-down, forced bottom-up and left to the direction rule."""
import numpy as np
import pytest

import graphgen
import oracle
from tests import graphs

pytestmark = pytest.mark.gpu

KS = (1, 2, 3, 6)
# KHOP_OPT_BATCH_PUSH divisors: 1 keeps every hop top-down, 2**30 sends every
# hop after the first bottom-up, 64 is the default rule
PUSH_DIVS = (1, 64, 2**30)


def _say(*a):
    print("[gpu-batched]", *a, flush=True)


@pytest.fixture(scope="module")
def K():
    import paper_1905_01294_amd as K
    return K


@pytest.fixture(scope="module")
def g0_gpu(K, g0):
    el, _ = g0
    return K.Graph.from_edgelist(el)


@pytest.mark.parametrize("per", [64, 256, 1024])
def test_g0_uniform_k(K, g0, g0_gpu, g0_oracle, per):
    _, seeds = g0
    g0_gpu.set_option(K.KHOP_OPT_BATCH_SEEDS, per)
    for k in KS:
        _say("g0 uniform", per, k)
        assert np.array_equal(g0_gpu.count_batched(seeds, np.full(len(seeds), k)), g0_oracle.count(seeds, k)[0])
    g0_gpu.set_option(K.KHOP_OPT_BATCH_SEEDS, 1024)


@pytest.mark.parametrize("per", [64, 256, 1024])
@pytest.mark.parametrize("heavy", [1, 16, 256, 10**9])
@pytest.mark.parametrize("push_div", PUSH_DIVS)
def test_g0_mixed_k_every_vertex(K, g0_gpu, g0_oracle, per, heavy, push_div):
    rng = np.random.default_rng(per + heavy)
    seeds = np.nonzero(g0_oracle.degrees() > 0)[0].astype(np.int32)
    ks = rng.choice(np.array([0, 1, 2, 3, 6, 9]), size=len(seeds)).astype(np.int32)
    g0_gpu.set_option(K.KHOP_OPT_BATCH_SEEDS, per)
    g0_gpu.set_option(K.KHOP_OPT_BATCH_HEAVY, heavy)
    g0_gpu.set_option(K.KHOP_OPT_BATCH_PUSH, push_div)
    _say("g0 mixed", per, heavy, push_div, len(seeds))
    got = g0_gpu.count_batched(seeds, ks)
    expect = np.array([g0_oracle.khop(int(s), int(k))[0] for s, k in zip(seeds, ks)])
    assert np.array_equal(got, expect)
    g0_gpu.set_option(K.KHOP_OPT_BATCH_SEEDS, 1024)
    g0_gpu.set_option(K.KHOP_OPT_BATCH_HEAVY, 256)
    g0_gpu.set_option(K.KHOP_OPT_BATCH_PUSH, 64)


def test_duplicates_and_ragged_batches(K, g0, g0_gpu, g0_oracle):
    _, seeds = g0
    for size in (1, 2, 63, 65, 100, 1025, 2100):
        s = np.resize(seeds, size)  # repeats seeds
        ks = np.resize(np.array([3, 1, 6, 2], np.int32), size)
        _say("ragged", size)
        got = g0_gpu.count_batched(s, ks)
        expect = np.array([g0_oracle.khop(int(a), int(b))[0] for a, b in zip(s, ks)])
        assert np.array_equal(got, expect), size


def test_device_entry_point(K, g0, g0_gpu, g0_oracle):
    import torch
    _, seeds = g0
    ks = np.array([(i % 4) + 1 for i in range(len(seeds))], np.int32)
    d_s = torch.from_numpy(seeds).cuda()
    d_k = torch.from_numpy(ks).cuda()
    d_c = torch.empty(len(seeds), dtype=torch.int64, device="cuda")
    g0_gpu.count_batched_dev(d_s, d_k, d_c)
    torch.cuda.synchronize()
    expect = [g0_oracle.khop(int(a), int(b))[0] for a, b in zip(seeds, ks)]
    assert d_c.cpu().tolist() == expect


@pytest.mark.parametrize("directed", [False, True])
@pytest.mark.parametrize("push_div", PUSH_DIVS)
def test_random_graphs(K, directed, push_div):
    rng = np.random.default_rng(7 + directed)
    for trial in range(8):
        n = int(rng.integers(2, 900))
        src, dst, n, d = graphs.random_graph(rng, n, int(rng.integers(0, 5 * n)), directed)
        g = K.Graph(src, dst, n, d)
        og = oracle.OracleGraph(src, dst, n, d)
        g.set_option(K.KHOP_OPT_BATCH_HEAVY, int(rng.integers(1, 40)))
        g.set_option(K.KHOP_OPT_BATCH_PUSH, push_div)
        seeds = rng.integers(0, n, size=int(rng.integers(1, 300))).astype(np.int32)
        ks = rng.integers(0, 8, size=len(seeds)).astype(np.int32)
        _say("random", directed, trial, n, len(seeds))
        got = g.count_batched(seeds, ks)
        expect = [og.khop(int(a), int(b))[0] for a, b in zip(seeds, ks)]
        assert got.tolist() == expect, trial
        g.free()


@pytest.mark.parametrize("push_div", PUSH_DIVS)
def test_batched_equals_plain_power_law(K, push_div):
    el = graphgen.chung_lu(80_000, 1_200_000, 5.0, seed=8)
    g = K.Graph.from_edgelist(el)
    g.set_option(K.KHOP_OPT_BATCH_PUSH, push_div)
    og = oracle.OracleGraph.from_edgelist(el)
    seeds = graphgen.draw_seeds(el, 300, seed=3)
    for k in KS:
        _say("chung-lu 80k", push_div, k)
        b = g.count_batched(seeds, np.full(len(seeds), k))
        p = g.count(seeds, k)
        assert np.array_equal(b, p)
        sample = seeds[:12]
        assert np.array_equal(b[:12], og.count(sample, k)[0])
    g.free()


def test_narrowing_under_forced_top_down(K, g0, g0_oracle):
    """Rows are repacked as seeds finish while hops stay top-down: 1000 seeds
    with k falling from 9 to 1 across the batch."""
    el, _ = g0
    g = K.Graph.from_edgelist(el)
    g.set_option(K.KHOP_OPT_BATCH_PUSH, 1)
    seeds = graphgen.draw_seeds(el, 800, seed=4)
    ks = np.repeat(np.arange(9, 0, -1), -(-len(seeds) // 9))[:len(seeds)].astype(np.int32)
    got = g.count_batched(seeds, ks)
    expect = np.array([g0_oracle.khop(int(s), int(k))[0] for s, k in zip(seeds, ks)])
    assert np.array_equal(got, expect)
    g.free()


@pytest.mark.parametrize("per", [64, 1024])
def test_one_hop_queries_take_no_bit(K, per):
    """One-hop queries are answered from their seeds' rows beside the bitset
    batch: launches with only one-hop slots, with one-hop slots behind k = 0
    and k = 2 slots, isolated seeds, and a hub of 40 000 neighbors."""
    n = 40000
    src = np.concatenate([np.zeros(n - 2, np.int32), np.arange(1, 4001, 2, dtype=np.int32)])
    dst = np.concatenate([np.arange(1, n - 1, dtype=np.int32), np.arange(2, 4002, 2, dtype=np.int32)])
    g = K.Graph(src, dst, n)  # vertex n - 1 is isolated
    og = oracle.OracleGraph(src, dst, n, False)
    g.set_option(K.KHOP_OPT_BATCH_SEEDS, per)
    rng = np.random.default_rng(per)
    seeds = np.concatenate([[0, n - 1, 3001, 0], rng.integers(0, n, size=300)]).astype(np.int32)
    for ks in (np.ones(len(seeds), np.int32),
               rng.choice(np.array([0, 1, 1, 1, 2]), size=len(seeds)).astype(np.int32)):
        got = g.count_batched(seeds, ks)
        expect = np.array([og.khop(int(s), int(k))[0] for s, k in zip(seeds, ks)])
        assert np.array_equal(got, expect), per
    lab = rng.random(n) < 0.5
    got = g.count_batched_labeled(seeds, np.ones(len(seeds), np.int32), lab)
    expect = np.array([og.khop_filtered(int(s), 1, lab.astype(np.uint8))[0] for s in seeds])
    assert np.array_equal(got, expect)
    g.free()
