"""GPU parity of the breadth-first distances (khop_bfs, khop_bfs_dev) against
the CPU oracle's distances, bit exact: every vertex's distance, the reach
count and the depth, in every direction mode, with and without a depth limit,
on small graphs of every shape, a deep path, random graphs with many
components, directed power-law graphs with split hub rows, and R-MAT scale 21
(the full plain-path workload) from sampled seeds."""
import time

import numpy as np
import pytest

import graphgen
import oracle
from tests import graphs

pytestmark = pytest.mark.gpu

ALL = 2**31 - 1
MODES = ("auto", "push", "pull")


def _say(*a):
    print("[gpu-bfs]", *a, flush=True)


@pytest.fixture(scope="module")
def K():
    import paper_1905_01294_amd as K
    return K


def _set_mode(K, g, mode):
    g.set_option(K.KHOP_OPT_DIRECTION, {"auto": K.KHOP_DIR_AUTO, "push": K.KHOP_DIR_PUSH,
                                        "pull": K.KHOP_DIR_PULL}[mode])


def _check(g, og, seed, max_depth=-1, tag=""):
    dist, count, depth = g.bfs(int(seed), max_depth)
    ref = og.distances(int(seed), ALL if max_depth < 0 else max_depth)
    assert np.array_equal(dist, ref), (tag, seed, max_depth, int((dist != ref).sum()))
    assert count == int((ref > 0).sum()), (tag, seed, max_depth)
    assert depth == int(ref.max()), (tag, seed, max_depth)
    return ref


@pytest.fixture(scope="module")
def g0_gpu(K, g0):
    el, _ = g0
    return K.Graph.from_edgelist(el)


@pytest.mark.parametrize("mode", MODES)
def test_g0_seeds_full_depth(K, g0, g0_gpu, g0_oracle, mode):
    el, seeds = g0
    _set_mode(K, g0_gpu, mode)
    _say("g0 full depth", mode)
    for s in seeds:
        _check(g0_gpu, g0_oracle, s, -1, mode)
    _set_mode(K, g0_gpu, "auto")


@pytest.mark.parametrize("mode", MODES)
def test_g0_depth_limits(K, g0, g0_gpu, g0_oracle, mode):
    el, seeds = g0
    _set_mode(K, g0_gpu, mode)
    _say("g0 depth limits", mode)
    for s in seeds[:8]:
        for d in (0, 1, 2, 3, 6, 40):
            _check(g0_gpu, g0_oracle, s, d, mode)
    # the count at depth k is the k-hop count of the plain path
    for d in (1, 2, 3):
        c = g0_gpu.count(seeds[:8], d)
        assert list(c) == [g0_gpu.bfs(int(s), d)[1] for s in seeds[:8]]
    _set_mode(K, g0_gpu, "auto")


@pytest.mark.parametrize("pam", [0, 2**31 - 1])
def test_g0_claim_modes(K, g0, g0_gpu, g0_oracle, pam):
    """Top-down heads claimed by atomics only, or by byte marks and compaction."""
    el, seeds = g0
    old = g0_gpu.get_option(K.KHOP_OPT_PUSH_ATOMIC)
    _set_mode(K, g0_gpu, "push")
    g0_gpu.set_option(K.KHOP_OPT_PUSH_ATOMIC, pam)
    try:
        for s in seeds[:12]:
            _check(g0_gpu, g0_oracle, s, -1, f"pam={pam}")
    finally:
        g0_gpu.set_option(K.KHOP_OPT_PUSH_ATOMIC, old)
        _set_mode(K, g0_gpu, "auto")


CLOSED = [
    ("path", graphs.path(50)),
    ("cycle_directed", graphs.cycle(17, directed=True)),
    ("grid", graphs.grid(9, 13)),
    ("hypercube", graphs.hypercube(7)),
    ("tree", graphs.binary_tree(8)),
    ("star", graphs.star(300)),
    ("complete", graphs.complete(40)),
]


@pytest.mark.parametrize("name,gr", CLOSED, ids=[c[0] for c in CLOSED])
@pytest.mark.parametrize("mode", MODES)
def test_closed_form_graphs(K, name, gr, mode):
    src, dst, n, directed = gr
    g = K.Graph(src, dst, n, directed)
    og = oracle.OracleGraph(src, dst, n, directed)
    _set_mode(K, g, mode)
    for s in sorted({0, n // 2, n - 1}):
        _check(g, og, s, -1, name)
        _check(g, og, s, 2, name)
    g.free()


def test_deep_path(K):
    """A path of 3000 vertices: 2999 levels, hop groups grown between host checks."""
    src, dst, n, directed = graphs.path(3000)
    g = K.Graph(src, dst, n, directed)
    og = oracle.OracleGraph(src, dst, n, directed)
    t = time.time()
    ref = _check(g, og, 0, -1, "path")
    _say("path 3000 from an end", round(time.time() - t, 3), "s")
    assert ref.max() == 2999
    _check(g, og, 1500, -1, "path")
    _check(g, og, 0, 2500, "path")
    g.free()


@pytest.mark.parametrize("directed", [False, True])
@pytest.mark.parametrize("mode", MODES)
def test_random_graphs(K, directed, mode):
    rng = np.random.default_rng(31 + directed)
    for n, m in ((1, 0), (70, 60), (500, 400), (3000, 9000), (6000, 4000)):
        src, dst, n, d = graphs.random_graph(rng, n, m, directed)
        g = K.Graph(src, dst, n, d)
        og = oracle.OracleGraph(src, dst, n, d)
        _set_mode(K, g, mode)
        for s in rng.integers(0, n, size=6):
            _check(g, og, s, -1, (n, m))
            _check(g, og, s, 1, (n, m))
        g.free()


def test_isolated_seed_and_errors(K):
    src = np.array([1, 2], dtype=np.int32)
    dst = np.array([2, 3], dtype=np.int32)
    g = K.Graph(src, dst, 5)
    dist, count, depth = g.bfs(0)
    assert list(dist) == [0, -1, -1, -1, -1] and count == 0 and depth == 0
    dist, count, depth = g.bfs(1)
    assert list(dist) == [-1, 0, 1, 2, -1] and count == 2 and depth == 2
    dist, count, depth = g.bfs(3, 0)
    assert list(dist) == [-1, -1, -1, 0, -1] and count == 0 and depth == 0
    for bad in (-1, 5):
        with pytest.raises(K.KhopError) as e:
            g.bfs(bad)
        assert e.value.status == K.KHOP_EINVAL
    g.free()


@pytest.mark.parametrize("heavy", [4, 64, 4096])
def test_directed_power_law_heavy_rows(K, heavy):
    el = graphgen.chung_lu(20000, 200000, 2.2, seed=13)
    g = K.Graph.from_edgelist(el)
    og = oracle.OracleGraph.from_edgelist(el)
    g.set_option(K.KHOP_OPT_PULL_HEAVY, heavy)
    for s in graphgen.draw_seeds(el, 8, seed=5):
        _check(g, og, s, -1, heavy)
    g.free()


def test_device_form_and_interleaving_with_counts(K, g0, g0_gpu, g0_oracle):
    import torch
    el, seeds = g0
    d_dist = torch.empty(el.n, dtype=torch.int32, device="cuda")
    d_count = torch.empty(1, dtype=torch.int64, device="cuda")
    d_depth = torch.empty(1, dtype=torch.int32, device="cuda")
    for i, s in enumerate(seeds[:10]):
        md = -1 if i % 2 == 0 else 3
        g0_gpu.bfs_dev(int(s), d_dist, md, d_count, d_depth)
        torch.cuda.synchronize()
        ref = g0_oracle.distances(int(s), ALL if md < 0 else md)
        assert np.array_equal(d_dist.cpu().numpy(), ref)
        assert int(d_count.item()) == int((ref > 0).sum())
        assert int(d_depth.item()) == int(ref.max())
        # a count run between searches shares the pooled query state
        c = g0_gpu.count(seeds[:4], 2)
        assert np.array_equal(c, g0_oracle.count(seeds[:4], 2)[0])


def test_side_stream(K, g0, g0_gpu, g0_oracle):
    import torch
    el, seeds = g0
    st = torch.cuda.Stream()
    d_dist = torch.empty(el.n, dtype=torch.int32, device="cuda")
    with torch.cuda.stream(st):
        g0_gpu.bfs_dev(int(seeds[3]), d_dist, -1, stream=st)
    st.synchronize()
    assert np.array_equal(d_dist.cpu().numpy(), g0_oracle.distances(int(seeds[3]), ALL))


@pytest.fixture(scope="module")
def g1(K):
    t = time.time()
    el = graphgen.rmat(21, 32, seed=1)
    og = oracle.OracleGraph.from_edgelist(el)
    g = K.Graph.from_edgelist(el)
    _say("rmat21 ready in", round(time.time() - t, 1), "s")
    yield el, og, g
    g.free()


@pytest.mark.parametrize("mode", MODES)
def test_rmat21_sampled_seeds(K, g1, mode):
    el, og, g = g1
    _set_mode(K, g, mode)
    seeds = graphgen.draw_seeds(el, 3, seed=7, stream=1)
    for s in seeds:
        t = time.time()
        ref = _check(g, og, s, -1, mode)
        _say("rmat21", mode, "seed", int(s), "depth", int(ref.max()), "reach", int((ref >= 0).sum()),
             round(time.time() - t, 2), "s")
    _check(g, og, seeds[0], 2, mode)
    _set_mode(K, g, "auto")
