"""GPU tests of the continuous-batching server: every served count equals the
oracle's (tolerance 0: counts are integers), alone and in a mix of seeds, k and
graphs, with admissions while other queries are in flight, under tight memory
budgets and with deadlines."""
import threading
import time

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-server]", *a, flush=True)


@pytest.fixture(scope="module")
def K():
    import paper_1905_01294_amd as K
    return K


@pytest.fixture(scope="module")
def graphs(K, g0):
    el0, _ = g0
    el1 = graphgen.chung_lu(20_000, 200_000, 4.0, seed=3)
    g = [K.Graph.from_edgelist(el0), K.Graph.from_edgelist(el1)]
    o = [oracle.OracleGraph.from_edgelist(el0), oracle.OracleGraph.from_edgelist(el1)]
    yield (el0, el1), g, o
    for x in g:
        x.free()


def _collect(srv, expect_n, timeout=60.0):
    got = {}
    t0 = time.time()
    while len(got) < expect_n:
        for r in srv.poll():
            got[r.ticket] = r
        if time.time() - t0 > timeout:
            raise AssertionError(f"only {len(got)} of {expect_n} results")
        time.sleep(0.001)
    return got


def test_mixed_batch_matches_oracle(K, graphs):
    (el0, el1), g, o = graphs
    srv = K.Server(1 << 30, 1024)
    ids = [srv.add_graph(x) for x in g]
    rng = np.random.default_rng(1)
    reqs = []
    for i in range(1500):
        gi = int(rng.integers(0, 2))
        el = (el0, el1)[gi]
        s = int(rng.integers(0, el.n))
        k = int(rng.choice([0, 1, 2, 3, 6]))
        reqs.append((srv.submit(ids[gi], s, k), gi, s, k))
    srv.drain(120000)
    got = _collect(srv, len(reqs))
    for t, gi, s, k in reqs:
        r = got[t]
        assert r.status == K.KHOP_OK
        assert (r.graph_id, r.seed, r.k) == (ids[gi], s, k)
        assert r.count == o[gi].khop(s, k)[0], (gi, s, k)
        assert r.t_submit_ns <= r.t_done_ns
    srv.close()


def test_alone_equals_in_mix(K, graphs):
    (el0, el1), g, o = graphs
    srv = K.Server(1 << 30, 256)
    gid = srv.add_graph(g[1])
    seeds = graphgen.draw_seeds(el1, 40, seed=9)
    alone = {}
    for s in seeds[:10]:
        t = srv.submit(gid, int(s), 3)
        srv.drain(30000)
        alone[int(s)] = _collect(srv, 1)[t].count
    ticks = [(srv.submit(gid, int(s), 3), int(s)) for s in seeds]
    srv.drain(30000)
    mix = _collect(srv, len(ticks))
    for t, s in ticks:
        if s in alone:
            assert mix[t].count == alone[s]
        assert mix[t].count == o[1].khop(s, 3)[0]
    srv.close()


def test_open_loop_arrivals_while_running(K, graphs):
    """Requests arrive from another thread while batches run; all are admitted and correct."""
    (el0, el1), g, o = graphs
    srv = K.Server(1 << 30, 128)
    ids = [srv.add_graph(x) for x in g]
    rng = np.random.default_rng(5)
    plan = [(int(rng.integers(0, 2)), int(rng.choice([1, 2, 3, 6]))) for _ in range(600)]
    plan = [(gi, int(rng.integers(0, (el0, el1)[gi].n)), k) for gi, k in plan]
    gaps = rng.exponential(50e-6, size=len(plan))
    tickets = []

    def producer():
        for (gi, s, k), gap in zip(plan, gaps):
            tickets.append((srv.submit(ids[gi], s, k), gi, s, k))
            time.sleep(gap)

    th = threading.Thread(target=producer)
    th.start()
    th.join()
    srv.drain(60000)
    got = _collect(srv, len(tickets))
    admitted_late = 0
    for t, gi, s, k in tickets:
        r = got[t]
        assert r.status == K.KHOP_OK
        assert r.count == o[gi].khop(s, k)[0]
        admitted_late += r.t_admit_ns > r.t_submit_ns
    assert admitted_late > 0
    srv.close()


def test_small_budget_one_word(K, graphs):
    (el0, _), g, o = graphs
    # room for exactly one one-word batch context of the scale-10 graph: the
    # lanes' slots take turns with it
    budget = K.khop_server_batch_bytes(g[0].handle, 1)
    assert K.khop_server_batch_bytes(g[0].handle, 2) > budget
    srv = K.Server(budget, 1024)
    gid = srv.add_graph(g[0])
    seeds = np.nonzero(o[0].degrees() > 0)[0][:300]
    ticks = [(srv.submit(gid, int(s), 2), int(s)) for s in seeds]
    srv.drain(60000)
    got = _collect(srv, len(ticks))
    for t, s in ticks:
        assert got[t].count == o[0].khop(s, 2)[0]
    st = srv.stats()
    assert max(x["words"] for x in st) <= 1
    srv.close()


def test_one_word_budget_both_lanes(K, graphs):
    """Short and deep queries compete for one one-word context; both lanes finish, all equal the oracle."""
    (el0, _), g, o = graphs
    srv = K.Server(K.khop_server_batch_bytes(g[0].handle, 1), 1024)
    srv.set_option(K.KHOP_SERVER_ROUTE, K.KHOP_ROUTE_BATCH)
    gid = srv.add_graph(g[0])
    seeds = np.nonzero(o[0].degrees() > 0)[0][:400]
    ticks = [(srv.submit(gid, int(s), (1, 2, 3, 6)[i % 4]), int(s), (1, 2, 3, 6)[i % 4]) for i, s in enumerate(seeds)]
    srv.drain(60000)
    got = _collect(srv, len(ticks))
    for t, s, k in ticks:
        assert got[t].status == K.KHOP_OK and got[t].count == o[0].khop(s, k)[0]
    lanes = {x["lane"]: x for x in srv.stats() if x["graph_id"] == gid}
    assert lanes["batch_k_le_2"]["queries"] == 200 and lanes["batch_k_gt_2"]["queries"] == 200
    srv.close()


def test_deep_k_is_answered(K, graphs):
    """k far past every eccentricity, on both paths: the count of everything within reach."""
    (el0, el1), g, o = graphs
    for route in (K.KHOP_ROUTE_BATCH, K.KHOP_ROUTE_PLAIN):
        srv = K.Server(1 << 30, 256)
        srv.set_option(K.KHOP_SERVER_ROUTE, route)
        ids = [srv.add_graph(x) for x in g]
        ticks = []
        for gi, el in enumerate((el0, el1)):
            for s in graphgen.draw_seeds(el, 6, seed=gi + 40):
                for k in (40, 10**6, 2**31 - 1):
                    ticks.append((srv.submit(ids[gi], int(s), k), gi, int(s), k))
        srv.drain(60000)
        got = _collect(srv, len(ticks))
        for t, gi, s, k in ticks:
            assert got[t].status == K.KHOP_OK
            assert got[t].count == o[gi].count(np.array([s], np.int32), k)[0][0], (route, gi, s, k)
        srv.close()


def test_deadlines_when_no_memory(K, graphs):
    (el0, _), g, o = graphs
    srv = K.Server(1024, 64)  # too small for any batch: requests wait, then time out
    srv.set_option(K.KHOP_SERVER_ROUTE, K.KHOP_ROUTE_BATCH)  # (the single-query lane is outside the budget)
    gid = srv.add_graph(g[0])
    t = srv.submit(gid, 1, 2, deadline_ns=K.monotonic_ns() + 20_000_000)
    srv.drain(5000)
    r = _collect(srv, 1)[t]
    assert r.status == K.KHOP_ETIMEDOUT
    srv.close()


def test_k0_and_invalid(K, graphs):
    (el0, _), g, o = graphs
    srv = K.Server(1 << 28, 64)
    gid = srv.add_graph(g[0])
    t = srv.submit(gid, 3, 0)
    srv.drain(5000)
    r = _collect(srv, 1)[t]
    assert r.status == K.KHOP_OK and r.count == 0
    with pytest.raises(K.KhopError):
        srv.submit(gid, el0.n, 1)
    with pytest.raises(K.KhopError):
        srv.submit(gid, 0, -1)
    srv.close()


@pytest.mark.parametrize("route", ["ROUTE_BATCH", "ROUTE_PLAIN", "ROUTE_AUTO"])
def test_each_route_matches_oracle(K, graphs, route):
    """Every query through the batches only, the single-query lanes only, or the
    automatic choice between them, with arrivals spread over time."""
    (el0, el1), g, o = graphs
    srv = K.Server(1 << 30, 256)
    srv.set_option(K.KHOP_SERVER_ROUTE, getattr(K, "KHOP_" + route))
    ids = [srv.add_graph(x) for x in g]
    rng = np.random.default_rng(77)
    reqs = []
    for i in range(900):
        gi = int(rng.integers(0, 2))
        s = int(rng.integers(0, (el0, el1)[gi].n))
        k = int(rng.choice([0, 1, 2, 3, 6, 9]))
        reqs.append((srv.submit(ids[gi], s, k), gi, s, k))
        if i % 100 == 99:
            time.sleep(0.002)
    srv.drain(120000)
    got = _collect(srv, len(reqs))
    for t, gi, s, k in reqs:
        r = got[t]
        assert r.status == K.KHOP_OK
        assert r.count == o[gi].khop(s, k)[0], (route, gi, s, k)
        assert r.t_submit_ns <= r.t_admit_ns <= r.t_done_ns or k == 0
        if route == "ROUTE_PLAIN" and k > 0:
            assert r.path == K.KHOP_PATH_SINGLE
        if route == "ROUTE_BATCH":
            assert r.path == K.KHOP_PATH_BATCH
    srv.close()


def test_plain_lane_takes_light_load(K, graphs):
    """At a trickle of queries the automatic route answers from the single-query lane in well under a millisecond."""
    (el0, _), g, o = graphs
    srv = K.Server(1 << 30, 1024)
    gid = srv.add_graph(g[0])
    seeds = np.nonzero(o[0].degrees() > 0)[0][:60]
    lat = []
    for s in seeds:
        t = srv.submit(gid, int(s), 2)
        srv.drain(10000)
        r = _collect(srv, 1)[t]
        assert r.count == o[0].khop(int(s), 2)[0]
        assert r.path == K.KHOP_PATH_SINGLE
        lat.append((r.t_done_ns - r.t_submit_ns) / 1e6)
    _say("trickle latency ms p50", float(np.median(lat)))
    assert float(np.median(lat)) < 2.0
    srv.close()


@pytest.mark.parametrize("route", ["ROUTE_PLAIN", "ROUTE_BATCH"])
def test_expired_deadline_on_each_path(K, graphs, route):
    """A request whose deadline has already passed times out on either path; the rest are answered."""
    (el0, _), g, o = graphs
    srv = K.Server(1 << 28, 64)
    srv.set_option(K.KHOP_SERVER_ROUTE, getattr(K, "KHOP_" + route))
    gid = srv.add_graph(g[0])
    past = K.monotonic_ns() - 1_000_000
    t_late = srv.submit(gid, 5, 2, deadline_ns=past)
    t_ok = srv.submit(gid, 5, 2)
    srv.drain(10000)
    got = _collect(srv, 2)
    assert got[t_late].status == K.KHOP_ETIMEDOUT
    assert got[t_ok].status == K.KHOP_OK and got[t_ok].count == o[0].khop(5, 2)[0]
    srv.close()
