"""C-ABI checks that need no GPU: the library loads, exports every entry point
that include/khop.h declares, and validates arguments before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1905_01294_amd as K

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _gpu_present():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def declared_functions():
    text = open(os.path.join(ROOT, "include", "khop.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "return")))


def test_header_declares_the_binding_exports():
    assert set(declared_functions()) == set(K.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(K.library_path())
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_version_and_empty_error():
    assert "gfx950" in K.khop_version()


def _rc(fn, *args):
    return fn(*args)


def test_graph_free_null_is_ok():
    assert K._lib.graph_free(None) == K.KHOP_OK


def test_load_validation_before_device():
    lib = K._lib
    src = np.array([0, 1], np.int32)
    dst = np.array([1, 5], np.int32)
    h = ctypes.c_void_p()
    p = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    # out NULL
    assert lib.graph_load_csr(p(src), p(dst), 2, 4, 0, None) == K.KHOP_EINVAL
    # endpoint 5 outside [0, 4)
    assert lib.graph_load_csr(p(src), p(dst), 2, 4, 0, ctypes.byref(h)) == K.KHOP_EINVAL
    assert "outside" in K.khop_last_error()
    assert h.value is None  # untouched on error
    # NULL arrays with edges
    assert lib.graph_load_csr(None, None, 2, 8, 0, ctypes.byref(h)) == K.KHOP_EINVAL
    # bad vertex counts and flags
    assert lib.graph_load_csr(p(src), p(dst), 2, 0, 0, ctypes.byref(h)) == K.KHOP_EINVAL
    assert lib.graph_load_csr(p(src), p(dst), 2, 2**31, 0, ctypes.byref(h)) == K.KHOP_ERANGE
    assert lib.graph_load_csr(p(src), p(dst), 2, 8, 7, ctypes.byref(h)) == K.KHOP_EINVAL
    assert lib.graph_load_csr(p(src), p(dst), -1, 8, 0, ctypes.byref(h)) == K.KHOP_EINVAL
    assert h.value is None


@pytest.mark.skipif(_gpu_present(), reason="checks the no-device path")
def test_valid_load_without_device_is_edevice():
    with pytest.raises(K.KhopError) as ei:
        K.graph_load_csr(np.array([0], np.int32), np.array([1], np.int32), 2)
    assert ei.value.status == K.KHOP_EDEVICE


def test_null_graph_calls():
    lib = K._lib
    c = (ctypes.c_int64 * 4)()
    s = (ctypes.c_int32 * 4)()
    assert lib.khop_count(None, s, 1, 1, c, None) == K.KHOP_EINVAL
    assert lib.khop_count_dev(None, None, 1, 1, None, None, None) == K.KHOP_EINVAL
    assert lib.khop_count_dev_noalloc(None, None, 1, 1, None, None, None) == K.KHOP_EINVAL
    assert lib.khop_count_batched(None, s, s, 1, c) == K.KHOP_EINVAL
    assert lib.khop_count_batched_dev(None, None, None, 1, None, None) == K.KHOP_EINVAL
    assert lib.graph_info(None, None, None, None) == K.KHOP_EINVAL
    assert lib.graph_degrees(None, None) == K.KHOP_EINVAL
    assert lib.khop_set_option(None, 1, 0) == K.KHOP_EINVAL
    assert lib.khop_get_option(None, 1, None) == K.KHOP_EINVAL
    assert lib.khop_autotune(None, 0) == K.KHOP_EINVAL
    assert lib.khop_profile(None, 1) == K.KHOP_EINVAL
    assert lib.khop_profile_read(None, None, 0, None) == K.KHOP_EINVAL
    assert "NULL" in K.khop_last_error()


def test_binding_rejects_mismatched_arrays():
    with pytest.raises(ValueError):
        K.graph_load_csr(np.zeros(3, np.int32), np.zeros(2, np.int32), 4)


def test_one_hip_runtime_in_process():
    """The binding loads PyTorch's HIP runtime first, so libkhop shares it."""
    paths = set()
    with open("/proc/self/maps") as f:
        for line in f:
            if "libamdhip64" in line:
                paths.add(line.split()[-1])
    assert len(paths) <= 1, paths


def test_label_bits_layout():
    """Bit v % 64 of word v // 64 is vertex v's label; bits past n are clear."""
    rng = np.random.default_rng(3)
    for n in (1, 63, 64, 65, 200):
        lab = rng.random(n) < 0.5
        words = K.label_bits(lab, n)
        assert words.dtype == np.uint64 and words.shape == ((n + 63) // 64,)
        for v in range(((n + 63) // 64) * 64):
            bit = (int(words[v // 64]) >> (v % 64)) & 1
            assert bit == (int(lab[v]) if v < n else 0)


def test_typed_and_labeled_validation_without_gpu():
    lib = K._lib
    h = ctypes.c_void_p()
    assert lib.graph_load_csr_typed(None, None, None, 3, 4, 0, 1, ctypes.byref(h)) == K.KHOP_EINVAL
    assert lib.khop_count_labeled(None, None, 1, 1, None, None, None) == K.KHOP_EINVAL
