"""Checks of the seeded input generator (statistics only: its realisations are
not pinned to any external graph, since the paper's datasets are not at hand)."""
import hashlib
import os
import subprocess
import sys

import numpy as np

import graphgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_rmat_sizes_and_range():
    el = graphgen.rmat(12, 8, seed=2)
    assert el.n == 4096 and el.m == 8 * 4096 and not el.directed
    assert el.src.min() >= 0 and el.src.max() < el.n and el.dst.max() < el.n


def test_rmat_quadrant_frequencies():
    el = graphgen.rmat(14, 16, seed=3, relabel=False)
    top = 1 << 13
    r = el.src >= top
    c = el.dst >= top
    freq = np.array([(~r & ~c).mean(), (~r & c).mean(), (r & ~c).mean(), (r & c).mean()])
    assert np.allclose(freq, [0.57, 0.19, 0.19, 0.05], atol=0.005)
    # the lowest recursion level follows the same split
    r0 = (el.src & 1) == 1
    c0 = (el.dst & 1) == 1
    assert abs((r0 & c0).mean() - 0.05) < 0.005


def test_relabel_is_a_permutation_of_labels():
    a = graphgen.rmat(10, 4, seed=5, relabel=False)
    b = graphgen.rmat(10, 4, seed=5, relabel=True)
    # same tuples up to one relabelling: the label mapping must be consistent
    mapping = {}
    for u, v in zip(np.concatenate([a.src, a.dst]).tolist(), np.concatenate([b.src, b.dst]).tolist()):
        assert mapping.setdefault(u, v) == v
    assert len(set(mapping.values())) == len(mapping)


def test_deterministic_and_seed_sensitive():
    a = graphgen.rmat(11, 8, seed=4)
    b = graphgen.rmat(11, 8, seed=4)
    c = graphgen.rmat(11, 8, seed=5)
    assert np.array_equal(a.src, b.src) and np.array_equal(a.dst, b.dst)
    assert not np.array_equal(a.src, c.src)


def _digest_with_threads(threads):
    code = ("import sys; sys.path.insert(0, %r); import graphgen, hashlib;"
            "e = graphgen.rmat(15, 8, seed=9); c = graphgen.chung_lu(20000, 300000, 5.0, seed=9);"
            "print(hashlib.sha256(e.src.tobytes() + e.dst.tobytes() + c.src.tobytes() + c.dst.tobytes()).hexdigest())"
            % ROOT)
    env = dict(os.environ, OMP_NUM_THREADS=str(threads))
    return subprocess.check_output([sys.executable, "-c", code], env=env).decode().strip()


def test_same_bytes_at_any_thread_count():
    assert _digest_with_threads(1) == _digest_with_threads(4)


def test_chung_lu_shape():
    n, m, x = 200_000, 2_000_000, 20.0
    el = graphgen.chung_lu(n, m, x, seed=1)
    assert el.directed and el.m == m
    outdeg = np.bincount(el.src, minlength=n)
    expect_max = m * np.log1p(1 / x) / np.log((n + x) / x)
    assert abs(outdeg.max() - expect_max) < 6 * np.sqrt(expect_max)
    # rank-size slope about -1 (degree exponent 2) over the mid ranks
    d = np.sort(outdeg)[::-1].astype(float)
    ranks = np.arange(1, n + 1, dtype=float)
    sel = slice(100, 10_000)
    slope = np.polyfit(np.log(ranks[sel]), np.log(d[sel]), 1)[0]
    assert -1.15 < slope < -0.85


def test_twitter_parameters_give_three_million_hub():
    n, m, x = graphgen.TWITTER_N, graphgen.TWITTER_M, graphgen.TWITTER_X
    expect_max = m * np.log1p(1 / x) / np.log((n + x) / x)
    assert 2.8e6 < expect_max < 3.1e6


def test_seed_draws():
    el = graphgen.rmat(10, 16, seed=1)
    s = graphgen.draw_seeds(el, 300, seed=7)
    assert len(s) == len(set(s.tolist())) == 300
    touched = set(el.src[el.src != el.dst].tolist()) | set(el.dst[el.src != el.dst].tolist())
    assert set(s.tolist()) <= touched
    assert np.array_equal(s, graphgen.draw_seeds(el, 300, seed=7))
    assert not np.array_equal(s, graphgen.draw_seeds(el, 300, seed=8))
    # more than the candidates: every candidate exactly once
    allc = graphgen.draw_seeds(el, 10**6, seed=1)
    assert sorted(allc.tolist()) == sorted(touched)
