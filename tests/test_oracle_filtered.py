"""Pins of the oracle's label-filtered search (oracle_khop_filtered): a
vertex other than the seed is entered only if it is allowed, so every path
runs through allowed vertices.  Pinned by
  * brute force: boolean powers of the dense adjacency with the columns of
    vertices that may not be entered cleared (a step may only land on an
    allowed vertex);
  * closed forms: a path cut by a blocked vertex, a star with some leaves
    blocked, a cycle blocked on one side;
  * the unfiltered count when every vertex is allowed.
"""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
from tests import graphs


def og(src, dst, n, directed):
    return oracle.OracleGraph(src, dst, n, directed)


def brute(src, dst, n, directed, s, k, allowed):
    a = graphs.dense_adjacency(src, dst, n, directed).astype(np.int64)
    np.fill_diagonal(a, 0)
    outdeg = (a > 0).sum(axis=1)
    step = a * allowed.astype(np.int64)[None, :]  # columns of blocked vertices cleared
    reach = np.zeros(n, dtype=bool)
    reach[s] = True
    sets = [reach.copy()]
    for _ in range(k):
        reach = reach | ((reach.astype(np.int64) @ step) > 0)
        sets.append(reach.copy())
    te = int(outdeg[sets[k - 1]].sum()) if k >= 1 else 0
    return int(sets[k].sum()) - 1, te


@settings(max_examples=800, deadline=None)
@given(n=st.integers(1, 36), m=st.integers(0, 120), directed=st.booleans(), k=st.integers(0, 7),
       rseed=st.integers(0, 2**32 - 1), p=st.floats(0.0, 1.0))
def test_brute_force_random(n, m, directed, k, rseed, p):
    rng = np.random.default_rng(rseed)
    src, dst, n, directed = graphs.random_graph(rng, n, m, directed)
    allowed = (rng.random(n) < p).astype(np.uint8)
    s = int(rng.integers(0, n))
    g = og(src, dst, n, directed)
    assert g.khop_filtered(s, k, allowed) == brute(src, dst, n, directed, s, k, allowed)


def test_all_allowed_is_the_plain_count():
    rng = np.random.default_rng(4)
    src, dst, n, d = graphs.random_graph(rng, 300, 900, True)
    g = og(src, dst, n, d)
    ones = np.ones(n, np.uint8)
    for s in rng.integers(0, n, size=10):
        for k in (1, 2, 3, 6):
            c, te, _ = g.khop(int(s), k)
            assert g.khop_filtered(int(s), k, ones) == (c, te)


@pytest.mark.parametrize("n,m", [(10, 4), (30, 1), (30, 29)])
def test_path_cut(n, m):
    g = og(*graphs.path(n))
    allowed = np.ones(n, np.uint8)
    allowed[m] = 0
    for k in (0, 1, 2, 5, 40):
        assert g.khop_filtered(0, k, allowed)[0] == min(k, m - 1)
        if m < n - 1:
            # from the far side the cut vertex, and what lies past it, stay out of reach
            assert g.khop_filtered(n - 1, k, allowed)[0] == min(k, n - 2 - m)


def test_star_with_blocked_leaves():
    n = 50
    g = og(*graphs.star(n))
    allowed = np.zeros(n, np.uint8)
    allowed[[0, 3, 4, 9, 20]] = 1
    for k in (1, 2, 5):
        assert g.khop_filtered(0, k, allowed)[0] == 4
        # a blocked leaf is still a seed; it reaches the centre, then the allowed leaves
        assert g.khop_filtered(7, k, allowed)[0] == 1 + 4 * (k >= 2)
    allowed[0] = 0
    assert g.khop_filtered(3, 6, allowed)[0] == 0


def test_cycle_blocked_on_one_side():
    n = 20
    g = og(*graphs.cycle(n))
    allowed = np.ones(n, np.uint8)
    allowed[1] = 0
    for k in (1, 3, 10, 30):
        # only the direction through n - 1, n - 2, ... stays open: n - 2 vertices at most
        assert g.khop_filtered(0, k, allowed)[0] == min(k, n - 2)
