"""Serving entry points that need no GPU: argument checks and an empty server."""
import ctypes

import pytest

import paper_1905_01294_amd as K


def test_create_validation():
    lib = K._lib
    h = ctypes.c_void_p()
    assert lib.khop_server_create(0, 1024, ctypes.byref(h)) == K.KHOP_EINVAL
    assert lib.khop_server_create(1 << 30, 100, ctypes.byref(h)) == K.KHOP_EINVAL
    assert lib.khop_server_create(1 << 30, 2048, ctypes.byref(h)) == K.KHOP_EINVAL
    assert lib.khop_server_create(1 << 30, 1024, None) == K.KHOP_EINVAL
    assert h.value is None


def test_empty_server_lifecycle():
    s = K.Server(1 << 30, 256)
    assert s.poll() == []
    s.drain(100)  # nothing pending
    with pytest.raises(K.KhopError) as ei:
        s.submit(0, 0, 1)  # no graph registered
    assert ei.value.status == K.KHOP_EINVAL
    s.close()
    s.close()


def test_null_handles():
    lib = K._lib
    t = ctypes.c_uint64()
    n = ctypes.c_int64()
    assert lib.khop_server_submit(None, 0, 0, 1, 0, ctypes.byref(t)) == K.KHOP_EINVAL
    assert lib.khop_server_poll(None, None, 0, ctypes.byref(n)) == K.KHOP_EINVAL
    assert lib.khop_server_drain(None, 0) == K.KHOP_EINVAL
    assert lib.khop_server_add_graph(None, None, None) == K.KHOP_EINVAL
    assert lib.khop_server_destroy(None) == K.KHOP_OK


def test_route_option_validation():
    s = K.Server(1 << 30, 256)
    for v in (K.KHOP_ROUTE_AUTO, K.KHOP_ROUTE_BATCH, K.KHOP_ROUTE_PLAIN):
        s.set_option(K.KHOP_SERVER_ROUTE, v)
    for opt, v in ((K.KHOP_SERVER_ROUTE, 3), (K.KHOP_SERVER_ROUTE, -1), (99, 0)):
        with pytest.raises(K.KhopError) as ei:
            s.set_option(opt, v)
        assert ei.value.status == K.KHOP_EINVAL
    assert K._lib.khop_server_set_option(None, K.KHOP_SERVER_ROUTE, 0) == K.KHOP_EINVAL
    s.close()
