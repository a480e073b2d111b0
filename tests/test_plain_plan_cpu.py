"""Host-side check of the plain path's query pipeline schedule
(csrc/plain_plan.h), compiled with the host compiler.

Each step launch runs the last hop of one query beside hop 1 of the next and,
on other blocks, counts an earlier query's byte marks, writes a finished
count and sets up the next query.  Query q runs on bitmap state q % 3,
control slot q % 5 and queue set q % 2.  For runs of 1..13 queries at
k = 1..7 the schedule must give every query each of its events exactly once
and in order, never hand one resource to two pieces of a launch, and reuse a
state, slot or queue set only after its previous query is done with it.
"""
import json
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _plan_constant(name):
    """A constant of the schedule header (kPlanStates, kPlanSlots, kPlanQueueSets)."""
    text = open(os.path.join(ROOT, "paper_1905_01294_amd", "csrc", "plain_plan.h")).read()
    return int(re.search(r"constexpr int %s = (\d+);" % name, text).group(1))


STATES, SLOTS, QSETS = (_plan_constant(n) for n in ("kPlanStates", "kPlanSlots", "kPlanQueueSets"))
INIT, MID = -1.0, 0.5  # the init launch; hops 2..k-1 of a query run between its step and the next


@pytest.fixture(scope="module")
def plans(tmp_path_factory):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path_factory.mktemp("plan") / "plan_dump")
    subprocess.run([cxx, "-std=c++17", "-O1", "-I", os.path.join(ROOT, "paper_1905_01294_amd", "csrc"),
                    os.path.join(ROOT, "tests", "plan_dump.cpp"), "-o", exe], check=True)
    args = [str(x) for k in range(1, 8) for m in range(1, 14) for x in (k, m)]
    out = subprocess.run([exe] + args, check=True, capture_output=True, text=True).stdout
    return [json.loads(line) for line in out.splitlines()]


def events(plan):
    """Times of each query's events: set-up, hop 1, last hop, marks count, count written."""
    k, m, steps = plan["k"], plan["m"], plan["steps"]
    S = len(steps)
    ev = {name: {} for name in ("setup", "h1", "last", "marks", "fin")}

    def put(name, q, t):
        assert q not in ev[name], (plan["k"], m, name, q)
        ev[name][q] = t

    put("setup", 0, INIT)
    for j, (last, h1, marks, fin, setup) in enumerate(steps):
        assert last >= 0 or h1 >= 0, ("a step with no hop", k, m, j)
        for name, q in (("last", last), ("h1", h1), ("marks", marks), ("fin", fin), ("setup", setup)):
            if q >= 0:
                put(name, q, float(j))
        if k == 1 and h1 >= 0:
            put("last", h1, float(j))
    _, _, marks, fin, _ = plan["close"]
    put("marks", marks, float(S))
    if fin >= 0:
        put("fin", fin, float(S))
    put("fin", m - 1, float(S + 1))  # the final launch
    for name in ev:
        assert sorted(ev[name]) == list(range(m)), (k, m, name, sorted(ev[name]))
    return ev


def test_plan_sizes(plans):
    for p in plans:
        assert len(p["steps"]) == (p["m"] + 1 if p["k"] >= 2 else p["m"])


def test_each_query_in_order(plans):
    for p in plans:
        k, m = p["k"], p["m"]
        ev = events(p)
        for q in range(m):
            assert ev["setup"][q] < ev["h1"][q] <= ev["last"][q] < ev["marks"][q] < ev["fin"][q], (k, m, q)
            if k >= 2:
                # hops 2..k-1 run between a query's step and the next, so the last hop is the next step
                assert ev["last"][q] == ev["h1"][q] + 1, (k, m, q)


def test_no_resource_shared_within_a_launch(plans):
    for p in plans:
        k, m = p["k"], p["m"]
        for j, (last, h1, marks, fin, setup) in enumerate(p["steps"]):
            st = {name: q % STATES for name, q in (("last", last), ("h1", h1), ("marks", marks), ("setup", setup))
                  if q >= 0}
            # the marks of a state may be counted in the launch that resets it: each word is
            # counted before it is reset, by the same thread
            for a in ("last", "h1"):
                for b in st:
                    if a != b and a in st:
                        assert st[a] != st[b], ("state", k, m, j, a, b)
            if "marks" in st and "setup" in st and st["marks"] == st["setup"]:
                assert marks == setup - STATES
            sl = {name: q % SLOTS for name, q in (("last", last), ("h1", h1), ("marks", marks), ("fin", fin),
                                                  ("setup", setup)) if q >= 0}
            names = list(sl)
            for i, a in enumerate(names):
                for b in names[i + 1:]:
                    # the count and the set-up run on blocks of their own, concurrently
                    assert sl[a] != sl[b], ("slot", k, m, j, a, b)
            if last >= 0 and h1 >= 0:
                assert last % QSETS != h1 % QSETS, ("queues", k, m, j)


def test_resources_reused_only_when_free(plans):
    for p in plans:
        k, m = p["k"], p["m"]
        ev = events(p)
        for q in range(m):
            r = q + STATES  # the next query on q's bitmap state resets it when it is set up
            if r < m:
                assert ev["last"][q] + (MID if k >= 3 else 0) < ev["setup"][r], ("state", k, m, q)
                assert ev["marks"][q] <= ev["setup"][r], ("state marks", k, m, q)
            r = q + SLOTS  # the next query on q's control slot
            if r < m:
                assert ev["fin"][q] < ev["setup"][r], ("slot", k, m, q)
            r = q + QSETS  # the next query on q's queue set writes it in its hop 1
            if r < m:
                assert ev["last"][q] < ev["h1"][r], ("queues", k, m, q)
