"""The no-allocation entry point, khop_count_dev_noalloc, called through the C
ABI: its counts and traversed edges equal khop_count_dev's (and the oracle's)
bit for bit, on consecutive calls whose inputs shrink and change graphs, so
that each call works on scratch an earlier call left behind; it rejects what
its fixed scratch cannot hold and leaves device memory as it was."""
import ctypes

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-noalloc]", *a, flush=True)


@pytest.fixture(scope="module")
def K():
    import paper_1905_01294_amd as K
    return K


def _run(K, fn, g, seeds, k):
    """One call of fn (a C entry point) on device copies of seeds; returns host counts and traversed edges."""
    import torch
    d_s = torch.from_numpy(np.ascontiguousarray(seeds, np.int32)).cuda()
    d_c = torch.full((len(seeds),), -7, dtype=torch.int64, device="cuda")
    d_t = torch.full((len(seeds),), -7, dtype=torch.int64, device="cuda")
    st = torch.cuda.current_stream()
    rc = fn(g.handle, ctypes.c_void_p(d_s.data_ptr()), len(seeds), int(k), ctypes.c_void_p(d_c.data_ptr()),
            ctypes.c_void_p(d_t.data_ptr()), ctypes.c_void_p(st.cuda_stream))
    assert rc == K.KHOP_OK, K.khop_last_error()
    torch.cuda.synchronize()
    return d_c.cpu().numpy(), d_t.cpu().numpy()


def test_noalloc_equals_count_dev_consecutive_calls(K):
    """Two calls in a row, the second with fewer seeds, then another graph, then the first again."""
    el0 = graphgen.rmat(10, 16, seed=1)
    el1 = graphgen.rmat(16, 8, seed=5)
    g0, g1 = K.Graph.from_edgelist(el0), K.Graph.from_edgelist(el1)
    o0, o1 = oracle.OracleGraph.from_edgelist(el0), oracle.OracleGraph.from_edgelist(el1)
    try:
        s0 = np.nonzero(o0.degrees() > 0)[0].astype(np.int32)
        s1 = graphgen.draw_seeds(el1, 200, seed=3)
        plan = [(g0, o0, s0, 3), (g0, o0, s0[:37], 3), (g1, o1, s1, 2), (g1, o1, s1[:9], 6),
                (g0, o0, s0[:100], 1), (g0, o0, s0[5:6], 32), (g1, o1, s1[:50], 0)]
        for g, o, seeds, k in plan:
            _say("noalloc", g.n, len(seeds), k)
            got = _run(K, K._lib.khop_count_dev_noalloc, g, seeds, k)
            ref = _run(K, K._lib.khop_count_dev, g, seeds, k)
            assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
            oc, ote = o.count(seeds, k)
            assert np.array_equal(got[0], oc) and np.array_equal(got[1], ote)
    finally:
        g0.free()
        g1.free()


def test_noalloc_invalid_seeds_and_limits(K):
    import torch
    el = graphgen.rmat(10, 16, seed=1)
    g = K.Graph.from_edgelist(el)
    o = oracle.OracleGraph.from_edgelist(el)
    try:
        seeds = np.array([3, -1, el.n, 5, 3], np.int32)
        c, t = _run(K, K._lib.khop_count_dev_noalloc, g, seeds, 2)
        oc, ote = o.count(np.array([3, 5], np.int32), 2)
        assert list(c) == [oc[0], -1, -1, oc[1], oc[0]] and list(t) == [ote[0], -1, -1, ote[1], ote[0]]
        d_s = torch.zeros(4, dtype=torch.int32, device="cuda")
        d_c = torch.zeros(4, dtype=torch.int64, device="cuda")
        args = (ctypes.c_void_p(d_s.data_ptr()), 4)
        rc = K._lib.khop_count_dev_noalloc(g.handle, *args, 33, ctypes.c_void_p(d_c.data_ptr()), None, None)
        assert rc == K.KHOP_ERANGE
        assert K._lib.khop_count_dev_noalloc(g.handle, *args, -1, ctypes.c_void_p(d_c.data_ptr()), None,
                                             None) == K.KHOP_EINVAL
    finally:
        g.free()
    # a graph whose query context exceeds the scratch
    big = K.Graph(np.array([0, 1], np.int32), np.array([1, 2], np.int32), 3_000_000)
    try:
        d_s = torch.zeros(1, dtype=torch.int32, device="cuda")
        d_c = torch.zeros(1, dtype=torch.int64, device="cuda")
        rc = K._lib.khop_count_dev_noalloc(big.handle, ctypes.c_void_p(d_s.data_ptr()), 1, 2,
                                           ctypes.c_void_p(d_c.data_ptr()), None, None)
        assert rc == K.KHOP_ERANGE and "scratch" in K.khop_last_error()
    finally:
        big.free()


def test_noalloc_takes_no_device_memory(K):
    """Free device memory is the same before and after a call (outputs allocated beforehand)."""
    import torch
    el = graphgen.rmat(12, 16, seed=2)
    g = K.Graph.from_edgelist(el)
    try:
        seeds = graphgen.draw_seeds(el, 64, seed=1)
        d_s = torch.from_numpy(seeds).cuda()
        d_c = torch.empty(64, dtype=torch.int64, device="cuda")
        d_t = torch.empty(64, dtype=torch.int64, device="cuda")
        g.count_dev_noalloc(d_s, 3, d_c, d_t)  # first use on this device
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        for k in (1, 2, 3, 6):
            g.count_dev_noalloc(d_s, k, d_c, d_t)
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0
    finally:
        g.free()
