"""GPU parity of the plain single-query path against the CPU oracle (bit exact).

Counts are integers, so the bar is equality, for every seed, at every k, in
every direction mode (auto, forced top-down, forced bottom-up); the traversed-
edge credit must match the oracle's too."""
import numpy as np
import pytest

import graphgen
import oracle
from tests import graphs

pytestmark = pytest.mark.gpu

KS = (1, 2, 3, 6)
MODES = ("auto", "push", "pull")


def _say(*a):
    print("[gpu-plain]", *a, flush=True)


@pytest.fixture(scope="module")
def K():
    import paper_1905_01294_amd as K
    return K


def _set_mode(K, g, mode):
    g.set_option(K.KHOP_OPT_DIRECTION, {"auto": K.KHOP_DIR_AUTO, "push": K.KHOP_DIR_PUSH,
                                        "pull": K.KHOP_DIR_PULL}[mode])


@pytest.fixture(scope="module")
def g0_gpu(K, g0):
    el, _ = g0
    return K.Graph.from_edgelist(el)


def test_g0_graph_shape(K, g0, g0_gpu, g0_oracle):
    el, _ = g0
    assert g0_gpu.n == el.n
    assert g0_gpu.num_arcs == g0_oracle.num_arcs
    assert np.array_equal(g0_gpu.degrees(), g0_oracle.degrees())


@pytest.mark.parametrize("mode", MODES)
def test_g0_all_seeds(K, g0, g0_gpu, g0_oracle, mode):
    el, seeds = g0
    _set_mode(K, g0_gpu, mode)
    for k in KS:
        _say("g0 32 seeds", mode, "k", k)
        c, te = g0_gpu.count(seeds, k, with_te=True)
        oc, ote = g0_oracle.count(seeds, k)
        assert np.array_equal(c, oc), (mode, k)
        assert np.array_equal(te, ote), (mode, k)
    _set_mode(K, g0_gpu, "auto")


@pytest.mark.parametrize("mode", MODES)
def test_g0_every_nonisolated_vertex_dev(K, g0_gpu, g0_oracle, mode):
    import torch
    seeds = np.nonzero(g0_oracle.degrees() > 0)[0].astype(np.int32)
    _set_mode(K, g0_gpu, mode)
    d_seeds = torch.from_numpy(seeds).cuda()
    for k in KS:
        _say("g0 every vertex dev", mode, "k", k, "seeds", len(seeds))
        d_c = torch.empty(len(seeds), dtype=torch.int64, device="cuda")
        d_t = torch.empty(len(seeds), dtype=torch.int64, device="cuda")
        g0_gpu.count_dev(d_seeds, k, d_c, d_t)
        torch.cuda.synchronize()
        oc, ote = g0_oracle.count(seeds, k)
        assert np.array_equal(d_c.cpu().numpy(), oc), (mode, k)
        assert np.array_equal(d_t.cpu().numpy(), ote), (mode, k)
    _set_mode(K, g0_gpu, "auto")


def test_g0_regression_fixture(K, g0_gpu):
    import json
    import os
    fx = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "g0_rmat10_counts.json")))
    seeds = np.array(fx["seeds"], np.int32)
    for k, row in fx["counts"].items():
        c, te = g0_gpu.count(seeds, int(k), with_te=True)
        assert c.tolist() == row and te.tolist() == fx["te"][k]


CLOSED = [
    ("path", graphs.path(70), lambda n, s, k: min(k, s) + min(k, n - 1 - s)),
    ("cycle", graphs.cycle(131), lambda n, s, k: min(2 * k, n - 1)),
    ("star", graphs.star(200), lambda n, s, k: (n - 1) * (k >= 1) if s == 0 else (k >= 1) + (n - 2) * (k >= 2)),
    ("complete", graphs.complete(65), lambda n, s, k: (n - 1) * (k >= 1)),
    ("dpath", graphs.path(100, directed=True), lambda n, s, k: min(k, n - 1 - s)),
    ("dcycle", graphs.cycle(129, directed=True), lambda n, s, k: min(k, n - 1)),
]


@pytest.mark.parametrize("name,gr,f", CLOSED, ids=[c[0] for c in CLOSED])
@pytest.mark.parametrize("mode", MODES)
def test_closed_forms(K, name, gr, f, mode):
    src, dst, n, d = gr
    g = K.Graph(src, dst, n, d)
    _set_mode(K, g, mode)
    seeds = np.array(sorted({0, 1, n // 2, n - 2, n - 1}), np.int32)
    for k in (0, 1, 2, 3, 6, 40, 200):
        _say(name, mode, "k", k)
        c = g.count(seeds, k)
        assert c.tolist() == [f(n, int(s), k) for s in seeds], (name, mode, k)
    g.free()


@pytest.mark.parametrize("mode", MODES)
def test_random_graphs_against_oracle(K, mode):
    rng = np.random.default_rng(2024)
    for trial in range(12):
        n = int(rng.integers(1, 700))
        m = int(rng.integers(0, 4 * n + 1))
        directed = bool(trial % 2)
        src, dst, n, d = graphs.random_graph(rng, n, m, directed)
        _say("random", mode, trial, n, m, directed)
        g = K.Graph(src, dst, n, d)
        _set_mode(K, g, mode)
        og = oracle.OracleGraph(src, dst, n, d)
        seeds = rng.integers(0, n, size=min(n, 24)).astype(np.int32)
        for k in (1, 2, 3, 6, 1000):
            c, te = g.count(seeds, k, with_te=True)
            oc, ote = og.count(seeds, k)
            assert np.array_equal(c, oc) and np.array_equal(te, ote), (trial, mode, k)
        g.free()


def test_edge_cases(K):
    # one vertex, no edges
    g = K.Graph(np.zeros(0, np.int32), np.zeros(0, np.int32), 1)
    assert g.count(np.array([0], np.int32), 3).tolist() == [0]
    assert g.count(np.zeros(0, np.int32), 3).tolist() == []
    g.free()
    # isolated seed and the last vertex of a ragged final word
    src, dst = np.array([0, 1, 2], np.int32), np.array([1, 2, 99], np.int32)
    g = K.Graph(src, dst, 100)
    assert g.count(np.array([50, 99, 0], np.int32), 6).tolist() == [0, 3, 3]
    assert g.count(np.array([99], np.int32), 0).tolist() == [0]
    # duplicate seeds answer identically
    assert g.count(np.array([1, 1, 1], np.int32), 1).tolist() == [2, 2, 2]
    with pytest.raises(K.KhopError) as ei:
        g.count(np.array([100], np.int32), 1)
    assert ei.value.status == K.KHOP_EINVAL
    with pytest.raises(K.KhopError):
        g.count(np.array([0], np.int32), -1)
    g.free()


@pytest.mark.parametrize("k", [1, 2])
def test_device_path_marks_bad_seed(K, k):
    import torch
    g = K.Graph(np.array([0], np.int32), np.array([1], np.int32), 3)
    d_s = torch.tensor([0, 7, 1, -1], dtype=torch.int32, device="cuda")
    d_c = torch.zeros(4, dtype=torch.int64, device="cuda")
    d_t = torch.zeros(4, dtype=torch.int64, device="cuda")
    g.count_dev(d_s, k, d_c, d_t)
    torch.cuda.synchronize()
    assert d_c.cpu().tolist() == [1, -1, 1, -1]
    # traversed edges: the out-degrees of levels 0 .. k-1 (one each here)
    assert d_t.cpu().tolist() == [k, -1, k, -1]
    g.free()


def test_input_invariance(K, g0, g0_oracle):
    el, seeds = g0
    rng = np.random.default_rng(3)
    order = rng.permutation(el.m)
    dup = rng.integers(0, el.m, size=el.m // 2)
    loops = rng.integers(0, el.n, size=300).astype(np.int32)
    g2 = K.Graph(np.concatenate([el.src[order], el.src[dup], loops]),
                 np.concatenate([el.dst[order], el.dst[dup], loops]), el.n)
    perm = graphgen.permutation(el.n, seed=5, tag=9)
    g3 = K.Graph(perm[el.src], perm[el.dst], el.n)
    for k in KS:
        oc, _ = g0_oracle.count(seeds, k)
        assert np.array_equal(g2.count(seeds, k), oc)
        assert np.array_equal(g3.count(perm[seeds], k), oc)
    g2.free()
    g3.free()


def test_repeat_runs_bit_identical(K, g0_gpu, g0):
    _, seeds = g0
    first = [g0_gpu.count(seeds, k) for k in KS]
    for _ in range(20):
        for k, ref in zip(KS, first):
            assert np.array_equal(g0_gpu.count(seeds, k), ref)


@pytest.mark.parametrize("heavy", [8, 32, 300, 4096])
def test_directed_power_law_small(K, heavy):
    el = graphgen.chung_lu(60_000, 900_000, 6.0, seed=4)
    g = K.Graph.from_edgelist(el)
    g.set_option(K.KHOP_OPT_PULL_HEAVY, heavy)
    og = oracle.OracleGraph.from_edgelist(el)
    seeds = graphgen.draw_seeds(el, 40, seed=1)
    for mode in MODES:
        _set_mode(K, g, mode)
        for k in KS:
            _say("chung-lu 60k", mode, k, "heavy", heavy)
            c, te = g.count(seeds, k, with_te=True)
            oc, ote = og.count(seeds, k)
            assert np.array_equal(c, oc) and np.array_equal(te, ote), (mode, k)
    g.free()


@pytest.mark.parametrize("grid", [1, 16])
@pytest.mark.parametrize("pam", [0, 2**31 - 1])
def test_top_down_queues_split_over_waves(K, grid, pam):
    """Forced top-down hops over region queues longer than a wave, whose edges are split between few
    (one block per compute unit) or many waves at arbitrary points, with heads claimed by byte marks
    and compaction (pam 0) or by atomics only: counts, traversed edges and BFS distances equal the
    oracle's."""
    el = graphgen.chung_lu(60_000, 900_000, 6.0, seed=8)
    g = K.Graph.from_edgelist(el)
    og = oracle.OracleGraph.from_edgelist(el)
    g.set_option(K.KHOP_OPT_PLAIN_GRID, grid)
    g.set_option(K.KHOP_OPT_PUSH_ATOMIC, pam)
    _set_mode(K, g, "push")
    seeds = graphgen.draw_seeds(el, 24, seed=2)
    for k in KS:
        _say("chung-lu 60k push windows, grid", grid, "pam", pam, "k", k)
        c, te = g.count(seeds, k, with_te=True)
        oc, ote = og.count(seeds, k)
        assert np.array_equal(c, oc) and np.array_equal(te, ote), k
    for s in seeds[:3]:
        dist, count, depth = g.bfs(int(s), -1)
        assert np.array_equal(dist, og.distances(int(s), 2**31 - 1))
    g.free()


@pytest.mark.parametrize("k", [1, 2, 3, 6])
def test_repeated_runs_replay_captured_launches(K, k):
    """A run repeated with the same device pointers, sizes and settings replays its launch sequence as a
    captured HIP graph: every replay, with new seeds written into the same buffer, other work on the
    context in between and a setting changed half way, equals the oracle."""
    import torch
    el = graphgen.chung_lu(60_000, 900_000, 6.0, seed=12)
    g = K.Graph.from_edgelist(el)
    og = oracle.OracleGraph.from_edgelist(el)
    dev = torch.device("cuda:0")
    g.set_option(K.KHOP_OPT_PLAIN_GRAPHS, 1)
    assert g.get_option(K.KHOP_OPT_PLAIN_GRAPHS) == 1
    pool = graphgen.draw_seeds(el, 400, seed=3)
    d_s = torch.empty(64, dtype=torch.int32, device=dev)
    d_c = torch.empty(64, dtype=torch.int64, device=dev)
    d_te = torch.empty(64, dtype=torch.int64, device=dev)
    for rep in range(6):
        seeds = pool[64 * rep:64 * (rep + 1)] if rep < 6 else pool[:64]
        d_s.copy_(torch.from_numpy(seeds))
        d_c.fill_(-7)
        d_te.fill_(-7)
        if rep == 3:
            g.set_option(K.KHOP_OPT_ALPHA, 3)  # new settings: a new launch sequence, seen, then captured
        g.count_dev(d_s, k, d_c, d_te)
        torch.cuda.synchronize()
        oc, ote = og.count(seeds, k)
        assert np.array_equal(d_c.cpu().numpy(), oc) and np.array_equal(d_te.cpu().numpy(), ote), (k, rep)
        # other work on the graph's contexts between the replays
        assert np.array_equal(g.count(pool[300:310], 2), og.count(pool[300:310], 2)[0])
        dist = g.bfs(int(pool[350 + rep]), -1)[0]
        assert np.array_equal(dist, og.distances(int(pool[350 + rep]), 2**31 - 1))
    g.free()


@pytest.mark.parametrize("alpha,beta", [(1, 2), (14, 24), (2, 1000), (1000, 2), (1, 100000)])
def test_direction_switch_points(K, alpha, beta):
    """Automatic direction with thresholds that move the top-down/bottom-up switches to other hops (a
    top-down hop after a bottom-up one walks the queue that hop appended).  Counts, traversed edges and
    full-depth distances equal the oracle's."""
    el = graphgen.chung_lu(120_000, 900_000, 3.0, seed=17)
    g = K.Graph.from_edgelist(el)
    og = oracle.OracleGraph.from_edgelist(el)
    g.set_option(K.KHOP_OPT_ALPHA, alpha)
    g.set_option(K.KHOP_OPT_BETA, beta)
    seeds = graphgen.draw_seeds(el, 24, seed=4)
    for k in (2, 3, 4, 6, 9):
        c, te = g.count(seeds, k, with_te=True)
        oc, ote = og.count(seeds, k)
        assert np.array_equal(c, oc) and np.array_equal(te, ote), (alpha, beta, k)
    for s in seeds[:4]:
        assert np.array_equal(g.bfs(int(s), -1)[0], og.distances(int(s), 2**31 - 1)), (alpha, beta, s)
    g.free()


@pytest.mark.parametrize("mode", MODES)
def test_context_reuse_across_entry_points(K, mode):
    """One graph's pooled query context serves, in turn, pipelined counts at several k, breadth-first
    searches, label-filtered counts, level sizes, neighborhood listings and one-at-a-time counts: a query's
    set-up rewrites only the blocks of its state that earlier uses set bits in, so each result must equal
    the oracle's whatever ran on the context before it."""
    el = graphgen.chung_lu(300_000, 2_400_000, 4.0, seed=21)
    g = K.Graph.from_edgelist(el)
    og = oracle.OracleGraph.from_edgelist(el)
    _set_mode(K, g, mode)
    rng = np.random.default_rng(5)
    lab = rng.random(el.n) < 0.6
    deg = og.degrees()
    hub = int(np.argmax(deg))
    for rnd in range(2):
        seeds = graphgen.draw_seeds(el, 40, seed=30 + rnd)
        _say("context reuse", mode, "round", rnd)
        for k in (3, 1, 2, 6):
            c, te = g.count(seeds, k, with_te=True)
            oc, ote = og.count(seeds, k)
            assert np.array_equal(c, oc) and np.array_equal(te, ote), (rnd, "count", k)
        s0 = int(seeds[rnd])
        dist, cnt, depth = g.bfs(s0, -1)
        assert np.array_equal(dist, og.distances(s0, 2**31 - 1)), (rnd, "bfs")
        lc = g.count_labeled(seeds[:12], 2, lab)
        assert list(lc) == [og.khop_filtered(int(x), 2, lab)[0] for x in seeds[:12]], (rnd, "labeled")
        assert np.array_equal(g.count(np.array([hub, s0, hub], np.int32), 2), og.count(np.array([hub, s0, hub]), 2)[0])
        assert list(g.levels(s0, 6)) == list(og.khop(s0, 6)[2]), (rnd, "levels")
        ref = og.distances(s0, 2)
        assert np.array_equal(g.neighborhood(s0, 2), np.nonzero(ref > 0)[0]), (rnd, "neighborhood")
        g.set_option(K.KHOP_OPT_PLAIN_PIPELINE, 0)
        try:
            assert np.array_equal(g.count(seeds[:16], 3), og.count(seeds[:16], 3)[0]), (rnd, "sequential")
        finally:
            g.set_option(K.KHOP_OPT_PLAIN_PIPELINE, 1)
        lc = g.count_labeled(seeds[:12], 3, lab)
        assert list(lc) == [og.khop_filtered(int(x), 3, lab)[0] for x in seeds[:12]], (rnd, "labeled 3")
    g.free()


@pytest.mark.parametrize("heavy", [1, 4, 64, 128])
def test_g0_pull_heavy_chunks(K, g0, g0_oracle, heavy):
    """Low chunk thresholds send many scale-10 vertices through the chunk kernel."""
    el, seeds = g0
    g = K.Graph.from_edgelist(el)
    g.set_option(K.KHOP_OPT_PULL_HEAVY, heavy)
    seeds_all = np.nonzero(g0_oracle.degrees() > 0)[0].astype(np.int32)
    for mode in ("auto", "pull"):
        _set_mode(K, g, mode)
        for k in KS:
            c, te = g.count(seeds_all, k, with_te=True)
            oc, ote = g0_oracle.count(seeds_all, k)
            assert np.array_equal(c, oc) and np.array_equal(te, ote), (mode, k)
    g.free()


def test_torch_side_stream(K, g0, g0_gpu, g0_oracle):
    """Device tensors and a non-default stream from PyTorch drive the library directly."""
    import torch
    _, seeds = g0
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        d_seeds = torch.from_numpy(seeds).cuda()
        d_c = torch.empty(len(seeds), dtype=torch.int64, device="cuda")
        g0_gpu.count_dev(d_seeds, 3, d_c, stream=s)
        d_b = torch.empty(len(seeds), dtype=torch.int64, device="cuda")
        g0_gpu.count_batched_dev(d_seeds, torch.full_like(d_seeds, 3), d_b, stream=s)
    s.synchronize()
    expect = g0_oracle.count(seeds, 3)[0]
    assert np.array_equal(d_c.cpu().numpy(), expect)
    assert np.array_equal(d_b.cpu().numpy(), expect)


def test_profile_reports_kernels_and_event_cost(K, g0, g0_gpu, g0_oracle):
    """khop_profile: per-kind launch counts and algorithmic bytes of a profiled
    run, the empty launches that price the event bracket, and unchanged counts."""
    el, _ = g0
    seeds = graphgen.draw_seeds(el, 16, seed=5)
    g0_gpu.profile(True)
    c = g0_gpu.count(seeds, 2)
    b = g0_gpu.count_batched(seeds, np.full(16, 3))
    stats = g0_gpu.profile_read()
    g0_gpu.profile(False)
    assert np.array_equal(c, g0_oracle.count(seeds, 2)[0])
    assert np.array_equal(b, g0_oracle.count(seeds, 3)[0])
    assert stats["empty_launch"]["launches"] == 16
    assert stats["empty_launch"]["algorithmic_bytes"] == 0
    # one query per call: hop 1 in one step launch, the last hop in the next
    assert stats["plain_step"]["launches"] == 2 * 16
    assert stats["plain_step"]["algorithmic_bytes"] > 0 and stats["plain_step"]["total_ms"] > 0
    assert "plain_hop_push" not in stats and "plain_hop_pull" not in stats
    assert stats["batch_pull"]["launches"] >= 2 and stats["batch_pull"]["algorithmic_bytes"] > 0
    assert "batch_count" in stats and "batch_push" in stats
    # k = 1, no vertex mask: one degree launch per query and no step launch
    g0_gpu.profile(True)
    c1 = g0_gpu.count(seeds, 1)
    s1 = g0_gpu.profile_read()
    g0_gpu.profile(False)
    assert np.array_equal(c1, g0_oracle.count(seeds, 1)[0])
    assert s1["plain_degree"]["launches"] == 16 and "plain_step" not in s1
    # k = 3: hop 2 runs on its own, counted by the direction it took; forced bottom-up, all pull
    for mode, kind in ((K.KHOP_DIR_PUSH, "plain_hop_push"), (K.KHOP_DIR_PULL, "plain_hop_pull")):
        g0_gpu.set_option(K.KHOP_OPT_DIRECTION, mode)
        g0_gpu.profile(True)
        c3 = g0_gpu.count(seeds, 3)
        s3 = g0_gpu.profile_read()
        g0_gpu.profile(False)
        g0_gpu.set_option(K.KHOP_OPT_DIRECTION, K.KHOP_DIR_AUTO)
        assert np.array_equal(c3, g0_oracle.count(seeds, 3)[0])
        assert s3[kind]["launches"] == 16 and s3["plain_compact"]["launches"] == 16


@pytest.mark.parametrize("mode", MODES)
def test_hub_seed_takes_the_claiming_hop1(K, mode):
    """A seed with more neighbors than the regions hold in 64-entry chunks
    (40 000 > 64 * 256) takes hop 1's claiming form; its leaves take the
    claim-free one.  A few leaf-to-leaf edges make hop 2 find something."""
    n = 40000
    src = np.concatenate([np.zeros(n - 1, np.int32), np.arange(1, 2001, 2, dtype=np.int32)])
    dst = np.concatenate([np.arange(1, n, dtype=np.int32), np.arange(2, 2002, 2, dtype=np.int32)])
    extra_s = np.arange(n, n + 500, dtype=np.int32)  # a tail hanging off leaf 7: depth up to 502
    extra_d = extra_s + 1
    src = np.concatenate([src, [7], extra_s[:-1]]).astype(np.int32)
    dst = np.concatenate([dst, [n], extra_d[:-1]]).astype(np.int32)
    N = n + 500
    g = K.Graph(src, dst, N)
    og = oracle.OracleGraph(src, dst, N, False)
    _set_mode(K, g, mode)
    for s in (0, 7, 1999, n - 1, n + 250):
        for k in (1, 2, 3, 6):
            c, te = g.count(np.array([s], np.int32), k, with_te=True)
            oc, ote = og.count(np.array([s], np.int32), k)
            assert (int(c[0]), int(te[0])) == (int(oc[0]), int(ote[0])), (mode, s, k)
        dist, count, depth = g.bfs(s)
        assert np.array_equal(dist, og.distances(s, 2**31 - 1)), (mode, s)
    g.free()


@pytest.mark.parametrize("mode", MODES)
def test_pipeline_run_lengths(K, g0, g0_gpu, g0_oracle, mode):
    """Device runs of 1 to 9 queries at k = 1..4, back to back on one context.
    Consecutive queries share launches: a query's last hop runs beside the
    next one's hop 1, and bitmaps, control records and queues rotate over
    three, four and two sets.  Every length puts the run's end at a different
    phase of that rotation, and each run starts from the first set again."""
    import torch
    el, seeds = g0
    _set_mode(K, g0_gpu, mode)
    rng = np.random.default_rng(77)
    for k in (1, 2, 3, 4):
        for m in rng.permutation(np.arange(1, 10)):
            s = seeds[rng.integers(0, len(seeds), size=int(m))].astype(np.int32)
            d_s = torch.from_numpy(s).cuda()
            d_c = torch.full((int(m),), -7, dtype=torch.int64, device="cuda")
            d_t = torch.full((int(m),), -7, dtype=torch.int64, device="cuda")
            g0_gpu.count_dev(d_s, k, d_c, d_t)
            torch.cuda.synchronize()
            oc, ote = g0_oracle.count(s, k)
            assert np.array_equal(d_c.cpu().numpy(), oc), (mode, k, int(m))
            assert np.array_equal(d_t.cpu().numpy(), ote), (mode, k, int(m))
    _set_mode(K, g0_gpu, "auto")


@pytest.mark.parametrize("mode", MODES)
def test_pipeline_hub_and_leaf_seeds(K, mode):
    """Hub seeds (40 000 neighbors: the claiming hop 1) between leaf seeds in
    one device run, so the hub's hop 1 shares its launch with a leaf query's
    last hop and the other way round; invalid seeds in between answer -1."""
    import torch
    n = 40000
    src = np.concatenate([np.zeros(n - 1, np.int32), np.arange(1, 4001, 2, dtype=np.int32)])
    dst = np.concatenate([np.arange(1, n, dtype=np.int32), np.arange(2, 4002, 2, dtype=np.int32)])
    g = K.Graph(src, dst, n)
    og = oracle.OracleGraph(src, dst, n, False)
    _set_mode(K, g, mode)
    s = np.array([0, 5, 0, 0, 3001, -1, 0, 12, n, 39999, 0], np.int32)
    ok = (s >= 0) & (s < n)
    d_s = torch.from_numpy(s).cuda()
    for k in (1, 2, 3):
        d_c = torch.zeros(len(s), dtype=torch.int64, device="cuda")
        d_t = torch.zeros(len(s), dtype=torch.int64, device="cuda")
        g.count_dev(d_s, k, d_c, d_t)
        torch.cuda.synchronize()
        c, t = d_c.cpu().numpy(), d_t.cpu().numpy()
        oc, ote = og.count(s[ok], k)
        assert np.array_equal(c[ok], oc) and np.array_equal(t[ok], ote), (mode, k)
        assert (c[~ok] == -1).all() and (t[~ok] == -1).all(), (mode, k)
    g.free()


@pytest.mark.parametrize("heavy", [2, 65536])
@pytest.mark.parametrize("mode", MODES)
def test_bottom_up_probe_hits_and_misses(K, mode, heavy):
    # Each target t has two in-neighbors: the hub H (out-degree 200, so H is
    # every target's probe) and its own low-degree vertex l_t.  From seed S1
    # hop 1 reaches every l_t and H only at hop 3, so a bottom-up hop 2 finds
    # the targets past a probe that is not in the frontier; from seed S2 hop 1
    # reaches H, and the probe finds them.  Extra in-edges of low out-degree
    # give some targets longer rows (past the reordered first four), and a
    # small chunk threshold sends those to the chunk table instead.
    H, T = 0, 200
    tg = np.arange(1, T + 1)
    lo = tg + T
    s1, s2, c1, c2 = 2 * T + 1, 2 * T + 2, 2 * T + 3, 2 * T + 4
    n = 2 * T + 5
    src = [np.full(T, H), lo, np.full(T, s1), [s1, c1, c2, s2]]
    dst = [tg, tg, lo, [c1, c2, H, H]]
    rng = np.random.default_rng(7)
    extra_t = rng.choice(tg, size=60, replace=False)
    for t in extra_t:
        src.append(rng.choice(lo, size=5, replace=False))
        dst.append(np.full(5, t))
    src = np.concatenate([np.asarray(x) for x in src]).astype(np.int32)
    dst = np.concatenate([np.asarray(x) for x in dst]).astype(np.int32)
    g = K.Graph(src, dst, n, True)
    _set_mode(K, g, mode)
    g.set_option(K.KHOP_OPT_PULL_HEAVY, heavy)
    og = oracle.OracleGraph(src, dst, n, True)
    seeds = np.array([s1, s2, H, c1, int(lo[0]), int(tg[0])], np.int32)
    _say("probe graph", mode, "heavy", heavy)
    for k in (1, 2, 3, 4, 6):
        c, te = g.count(seeds, k, with_te=True)
        oc, ote = og.count(seeds, k)
        assert np.array_equal(c, oc) and np.array_equal(te, ote), (mode, heavy, k)
    g.free()
