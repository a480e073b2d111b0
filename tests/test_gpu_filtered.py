"""GPU parity of typed and label-filtered traversal against the CPU oracle,
bit exact.

  * Relation types: graph_load_csr_typed keeps the tuples of the selected
    relations, so its counts, batched counts and distances equal the oracle's
    on those tuples.
  * Vertex labels: khop_count_labeled equals the oracle's search that enters
    only labeled vertices (oracle_khop_filtered), counts and traversed edges,
    for every direction mode, label density and the claim-free and claiming
    forms of hop 1; the mask does not leak into later unfiltered queries.
"""
import numpy as np
import pytest

import graphgen
import oracle
from tests import graphs

pytestmark = pytest.mark.gpu

MODES = ("auto", "push", "pull")


def _say(*a):
    print("[gpu-filtered]", *a, flush=True)


@pytest.fixture(scope="module")
def K():
    import paper_1905_01294_amd as K
    return K


def _set_mode(K, g, mode):
    g.set_option(K.KHOP_OPT_DIRECTION, {"auto": K.KHOP_DIR_AUTO, "push": K.KHOP_DIR_PUSH,
                                        "pull": K.KHOP_DIR_PULL}[mode])


def _check_labeled(g, og, seeds, k, lab, tag):
    c, te = g.count_labeled(seeds, k, lab, with_te=True)
    for i, s in enumerate(seeds):
        oc, ote = og.khop_filtered(int(s), k, lab.astype(np.uint8))
        assert (int(c[i]), int(te[i])) == (oc, ote), (tag, int(s), k)


@pytest.fixture(scope="module")
def g0_gpu(K, g0):
    el, _ = g0
    return K.Graph.from_edgelist(el)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("p", [1.0, 0.9, 0.5, 0.1])
def test_g0_labeled(K, g0, g0_gpu, g0_oracle, mode, p):
    el, seeds = g0
    lab = np.random.default_rng(int(p * 100)).random(el.n) < p
    _set_mode(K, g0_gpu, mode)
    for k in (1, 2, 3, 6):
        _check_labeled(g0_gpu, g0_oracle, seeds, k, lab, (mode, p))
    if p == 1.0:
        assert np.array_equal(g0_gpu.count_labeled(seeds, 3, lab), g0_gpu.count(seeds, 3))
    _set_mode(K, g0_gpu, "auto")


def test_mask_does_not_leak(K, g0, g0_gpu, g0_oracle):
    el, seeds = g0
    lab = np.random.default_rng(8).random(el.n) < 0.3
    for _ in range(3):
        _check_labeled(g0_gpu, g0_oracle, seeds[:8], 2, lab, "leak")
        assert np.array_equal(g0_gpu.count(seeds, 2), g0_oracle.count(seeds, 2)[0])
        assert np.array_equal(g0_gpu.count_batched(seeds, np.full(len(seeds), 3)), g0_oracle.count(seeds, 3)[0])


@pytest.mark.parametrize("directed", [False, True])
@pytest.mark.parametrize("mode", MODES)
def test_random_ragged(K, directed, mode):
    """n = 70001: a ragged last mask word, seeds both labeled and not."""
    rng = np.random.default_rng(11 + directed)
    src, dst, n, d = graphs.random_graph(rng, 70001, 250000, directed)
    g = K.Graph(src, dst, n, d)
    og = oracle.OracleGraph(src, dst, n, d)
    _set_mode(K, g, mode)
    lab = rng.random(n) < 0.6
    seeds = np.concatenate([rng.integers(0, n, size=6), [0, n - 1]]).astype(np.int32)
    for k in (1, 2, 4, 9):
        _check_labeled(g, og, seeds, k, lab, (directed, mode))
    g.free()


def test_hub_seed_claiming_hop1(K):
    """A seed of degree 39 999 (past the claim-free hop 1) with half its leaves unlabeled."""
    n = 40000
    src = np.concatenate([np.zeros(n - 1, np.int32), np.arange(1, 4001, 2, dtype=np.int32)])
    dst = np.concatenate([np.arange(1, n, dtype=np.int32), np.arange(2, 4002, 2, dtype=np.int32)])
    g = K.Graph(src, dst, n)
    og = oracle.OracleGraph(src, dst, n, False)
    lab = (np.arange(n) % 2) == 0
    for mode in MODES:
        _set_mode(K, g, mode)
        _check_labeled(g, og, np.array([0, 1, 2, 3001], np.int32), 2, lab, mode)
        _check_labeled(g, og, np.array([0, 5], np.int32), 3, lab, mode)
    g.free()


def test_device_form(K, g0, g0_gpu, g0_oracle):
    import torch
    el, seeds = g0
    lab = np.random.default_rng(21).random(el.n) < 0.5
    d_bits = torch.from_numpy(K.label_bits(lab, el.n).view(np.int64)).cuda()
    d_seeds = torch.from_numpy(seeds).cuda()
    d_c = torch.empty(len(seeds), dtype=torch.int64, device="cuda")
    d_t = torch.empty(len(seeds), dtype=torch.int64, device="cuda")
    g0_gpu.count_labeled_dev(d_seeds, 3, d_bits, d_c, d_t)
    torch.cuda.synchronize()
    c, te = g0_gpu.count_labeled(seeds, 3, lab, with_te=True)
    assert np.array_equal(d_c.cpu().numpy(), c) and np.array_equal(d_t.cpu().numpy(), te)


@pytest.mark.parametrize("mask", [0b0001, 0b0101, 0b1111, 0b1000])
@pytest.mark.parametrize("directed", [False, True])
def test_relation_types(K, mask, directed):
    rng = np.random.default_rng(mask + 17 * directed)
    el = graphgen.chung_lu(6000, 60000, 4.0, seed=mask) if directed else graphgen.rmat(12, 8, seed=mask)
    rel = rng.integers(0, 4, size=el.m).astype(np.uint8)
    g = K.Graph.typed(el.src, el.dst, rel, el.n, mask, directed=el.directed)
    keep = ((mask >> rel.astype(np.int64)) & 1).astype(bool)
    og = oracle.OracleGraph(el.src[keep], el.dst[keep], el.n, el.directed)
    assert g.num_arcs == og.num_arcs
    seeds = graphgen.draw_seeds(el, 24, seed=3)
    for k in (1, 2, 3, 6):
        c = g.count(seeds, k)
        assert np.array_equal(c, og.count(seeds, k)[0]), (mask, k)
        assert np.array_equal(g.count_batched(seeds, np.full(len(seeds), k)), c)
    dist, _, _ = g.bfs(int(seeds[0]))
    assert np.array_equal(dist, og.distances(int(seeds[0]), 2**31 - 1))
    # a label filter on top of the relation filter
    lab = rng.random(el.n) < 0.5
    _check_labeled(g, og, seeds[:8], 3, lab, ("typed", mask))
    g.free()


def test_typed_validation(K):
    src = np.array([0, 1], np.int32)
    dst = np.array([1, 2], np.int32)
    with pytest.raises(K.KhopError) as e:
        K.Graph.typed(src, dst, np.array([0, 64], np.uint8), 3, 1)
    assert e.value.status == K.KHOP_EINVAL
    g = K.Graph.typed(src, dst, np.array([0, 1], np.uint8), 3, 0)  # no relation selected: no arcs
    assert g.num_arcs == 0 and list(g.count(np.array([0], np.int32), 3)) == [0]
    g.free()


def test_rmat21_labeled(K):
    el = graphgen.rmat(21, 32, seed=1)
    g = K.Graph.from_edgelist(el)
    og = oracle.OracleGraph.from_edgelist(el)
    lab = np.random.default_rng(5).random(el.n) < 0.5
    seeds = graphgen.draw_seeds(el, 6, seed=7, stream=4)
    for k in (2, 3):
        _check_labeled(g, og, seeds, k, lab, "rmat21")
    _say("rmat21 labeled ok")
    g.free()


@pytest.mark.parametrize("p", [0.9, 0.5, 0.15])
def test_batched_labeled(K, g0, g0_gpu, g0_oracle, p):
    """Batched label-filtered counts, mixed k, seeds labeled or not, equal to the oracle and to the plain form."""
    el, seeds = g0
    rng = np.random.default_rng(int(p * 1000))
    lab = rng.random(el.n) < p
    every = np.nonzero(g0_oracle.degrees() > 0)[0].astype(np.int32)
    ks = rng.integers(0, 8, size=every.size).astype(np.int32)
    got = g0_gpu.count_batched_labeled(every, ks, lab)
    for i in range(0, every.size, 3):
        assert int(got[i]) == g0_oracle.khop_filtered(int(every[i]), int(ks[i]), lab.astype(np.uint8))[0], \
            (p, int(every[i]), int(ks[i]))
    for k in (1, 3):
        sel = ks == k
        assert np.array_equal(got[sel], g0_gpu.count_labeled(every[sel], k, lab))
    # the mask does not leak into a later unfiltered batch
    assert np.array_equal(g0_gpu.count_batched(seeds, np.full(len(seeds), 3)), g0_oracle.count(seeds, 3)[0])


@pytest.mark.parametrize("directed", [False, True])
def test_batched_labeled_ragged(K, directed):
    rng = np.random.default_rng(29 + directed)
    src, dst, n, d = graphs.random_graph(rng, 70001, 250000, directed)
    g = K.Graph(src, dst, n, d)
    og = oracle.OracleGraph(src, dst, n, d)
    lab = rng.random(n) < 0.6
    seeds = np.concatenate([rng.integers(0, n, size=150), [0, n - 1]]).astype(np.int32)
    ks = rng.integers(1, 9, size=seeds.size).astype(np.int32)
    got = g.count_batched_labeled(seeds, ks, lab)
    for i in range(seeds.size):
        assert int(got[i]) == og.khop_filtered(int(seeds[i]), int(ks[i]), lab.astype(np.uint8))[0], (directed, i)
    g.free()


def test_pipeline_run_lengths_labeled(K, g0, g0_gpu, g0_oracle):
    """Label-filtered runs of 1 to 9 queries at k = 1..3 through the host entry
    point, which runs all of a call's seeds as one pipelined sequence."""
    el, seeds = g0
    rng = np.random.default_rng(55)
    lab = rng.random(el.n) < 0.5
    for k in (1, 2, 3):
        for m in rng.permutation(np.arange(1, 10)):
            s = seeds[rng.integers(0, len(seeds), size=int(m))].astype(np.int32)
            _check_labeled(g0_gpu, g0_oracle, s, k, lab, ("run", k, int(m)))
