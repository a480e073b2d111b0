"""Host-side checks of the server's scheduling rules (csrc/serve_policy.h),
compiled with the host compiler and driven with a simulated clock
(tests/serve_policy_sim.cpp): FIFO admission per lane, deadlines, the memory
budget, slot reuse and context release, and the slot order of a batch."""
import json
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
RUNS = 2  # run slots per lane (kRunsPerLane)


def ctx_bytes(w):
    return 1000 + 300 * w  # the simulator's context size


@pytest.fixture(scope="module")
def sim(tmp_path_factory):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path_factory.mktemp("policy") / "serve_policy_sim")
    subprocess.run([cxx, "-std=c++17", "-O1", "-Wall", "-I", os.path.join(ROOT, "paper_1905_01294_amd", "csrc"),
                    os.path.join(ROOT, "tests", "serve_policy_sim.cpp"), "-o", exe], check=True)
    return exe


def run(sim, seed, budget, max_words, lanes, arrivals):
    out = subprocess.run([sim, str(seed), str(budget), str(max_words), str(lanes), str(arrivals)], check=True,
                         capture_output=True, text=True).stdout
    return [json.loads(line) for line in out.splitlines()]


CONFIGS = [
    # (seed, budget, max_words, lanes)
    (1, 10**9, 16, 4),
    (2, 10**9, 1, 2),
    (3, ctx_bytes(1), 16, 4),   # one one-word context at a time
    (4, ctx_bytes(4) + ctx_bytes(1), 4, 3),
    (5, 3 * ctx_bytes(2), 8, 4),
]


@pytest.mark.parametrize("seed,budget,max_words,lanes", CONFIGS)
def test_policy_invariants(sim, seed, budget, max_words, lanes):
    ev = run(sim, seed, budget, max_words, lanes, 400)
    arrive = {e["ticket"]: e for e in ev if e["ev"] == "arrive"}
    launched, late = {}, {}
    last_ticket = {}
    busy = {}
    held = {}  # (lane, run) -> bytes
    queued = {}  # lane -> tickets waiting
    for e in ev:
        if e["ev"] == "arrive":
            queued.setdefault(e["lane"], set()).add(e["ticket"])
        if e["ev"] == "launch":
            key = (e["lane"], e["run"])
            assert not busy.get(key), "a slot launched while busy"
            others = sum(v for (l, r), v in busy.items() if l == e["lane"] and r != e["run"])
            if others:  # beside a running launch only for a backlog of a quarter of its width
                assert len(queued[e["lane"]]) >= 16 * e["words"], (len(queued[e["lane"]]), e)
            busy[key] = True
            w = e["words"]
            assert w & (w - 1) == 0 and 1 <= w <= max_words
            assert 1 <= len(e["tickets"]) <= 64 * w
            if e["alloc"]:
                assert key not in held, "allocated over a held context"
                avail_before = budget - sum(held.values())
                assert ctx_bytes(w) <= avail_before
                assert 2 * w > max_words or ctx_bytes(2 * w) > avail_before, "not the widest context that fits"
                held[key] = e["bytes"]
            else:
                assert key in held, "launched without a context"
            assert sum(held.values()) <= budget
            for t in e["tickets"]:
                assert t not in launched and t not in late
                launched[t] = e["t"]
                queued[e["lane"]].discard(t)
                a = arrive[t]
                assert a["lane"] == e["lane"]
                assert a["deadline"] == 0 or e["t"] <= a["deadline"], "launched after its deadline"
                # FIFO within a lane
                assert t > last_ticket.get(e["lane"], 0)
                last_ticket[e["lane"]] = t
        elif e["ev"] == "done":
            busy[(e["lane"], e["run"])] = False
        elif e["ev"] == "release":
            key = (e["lane"], e["run"])
            assert not busy.get(key) and key in held
            del held[key]
        elif e["ev"] == "late":
            t = e["ticket"]
            assert t not in launched and t not in late
            queued[e["lane"]].discard(t)
            assert 0 < arrive[t]["deadline"] < e["t"], "timed out before its deadline"
            late[t] = e["t"]
        elif e["ev"] == "pass":
            assert e["avail"] == budget - sum(held.values())
    assert set(launched) | set(late) == set(arrive)
    assert ev[-1]["ev"] == "end" and ev[-1]["avail"] == budget and not held


def test_tight_budget_one_context_at_a_time(sim):
    ev = run(sim, 7, ctx_bytes(1), 16, 4, 300)
    held = 0
    for e in ev:
        if e["ev"] == "launch" and e["alloc"]:
            held += 1
            assert held == 1
        elif e["ev"] == "release":
            held -= 1
    assert any(e["ev"] == "pass" and e["waiting"] for e in ev), "other lanes never waited for memory"


def test_no_memory_only_deadlines(sim):
    """With a budget below one context nothing launches: requests with a deadline time out, the others wait."""
    ev = run(sim, 8, ctx_bytes(1) - 1, 4, 2, 80)
    assert ev[-1]["ev"] == "end" and ev[-1]["cut"] == 1
    assert not any(e["ev"] == "launch" for e in ev)
    arrive = {e["ticket"]: e for e in ev if e["ev"] == "arrive"}
    late = {e["ticket"]: e for e in ev if e["ev"] == "late"}
    assert set(late) == {t for t, a in arrive.items() if a["deadline"] > 0} and late
    for t, e in late.items():
        assert e["t"] > arrive[t]["deadline"]
    assert any(e["ev"] == "pass" and e["waiting"] for e in ev)


@pytest.mark.parametrize("ks", [[3, 1, 2, 1, 6, 0, 2, 3], [1, 1, 1], [0, 2, 0, 1], [5], [2, 2, 2, 2]])
def test_batch_order(sim, ks):
    out = subprocess.run([sim, "order"] + [str(k) for k in ks], check=True, capture_output=True, text=True).stdout
    order = [int(x) for x in out.split()]
    assert sorted(order) == list(range(len(ks)))
    key = [-1 if ks[i] == 1 else ks[i] for i in order]
    assert key == sorted(key, reverse=True)  # largest k first, one-hop queries last
    for a, b in zip(order, order[1:]):
        if key[order.index(a)] == key[order.index(b)]:
            assert a < b  # stable


def route(sim, route_opt, gap_ns, floor_ms, cost_ms, batch_ms, n=2000):
    out = subprocess.run([sim, "route", str(route_opt), str(gap_ns), str(floor_ms), str(cost_ms), str(batch_ms),
                          str(n)], check=True, capture_output=True, text=True).stdout
    rows = [line.split() for line in out.splitlines()]
    return [int(a) for a, _ in rows], [float(b) for _, b in rows]


MAX_BACKLOG_MS = 3.0  # SingleRouter::kMaxBacklogMs


def test_router_forced_routes(sim):
    assert route(sim, 1, 1000, 0.01, 0.01, 50)[0] == [0] * 2000  # ROUTE_BATCH
    assert route(sim, 2, 1000, 5.0, 5.0, 0.1)[0] == [1] * 2000   # ROUTE_PLAIN


def test_router_light_load_takes_everything(sim):
    """A trickle of cheap queries (0.01 ms each, one every 100 us) all go to the single-query lane."""
    taken, backlog = route(sim, 0, 100_000, 0.01, 0.01, 5.0)
    assert all(taken) and max(backlog) < 0.1


def test_router_backlog_is_bounded(sim):
    """Cheap by their uncontended cost but slow in practice (0.3 ms each under contention), arriving every
    20 us: the lane keeps at most its backlog bound and sends the rest to the batches."""
    taken, backlog = route(sim, 0, 20_000, 0.01, 0.3, 200.0)
    assert 0 < sum(taken) < len(taken)
    assert max(backlog) <= MAX_BACKLOG_MS + 1e-9


def test_router_heavy_demand_goes_to_batches(sim):
    """Dear queries (2 ms uncontended) arriving faster than one device can answer them: once the decayed
    demand passes the device, none is taken until it falls back below 0.8."""
    taken, _ = route(sim, 0, 500_000, 2.0, 2.0, 1000.0, n=4000)
    assert sum(taken[-1000:]) < 0.5 * 1000 * 0.5  # at most about what one device keeps up with
    taken2, _ = route(sim, 0, 10_000_000, 2.0, 2.0, 1000.0, n=200)
    assert all(taken2)  # one every 10 ms: well under the device
