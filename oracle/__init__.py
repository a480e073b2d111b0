"""ORACLE -- test infrastructure only.

Plain single-threaded CPU k-hop neighborhood count (the breadth-first-search
definition of the count the paper benchmarks in Section III), written in C in
`oracle.c` and wrapped here with ctypes.  Only the tests, the smoke check and
the benchmark's CPU-baseline leg use it; the library never imports it and it
imports nothing from the library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (single-threaded, -O2); returns its path."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.oracle_build.argtypes = [_i32p, _i32p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int,
                                     ctypes.POINTER(ctypes.c_void_p)]
        lib.oracle_build.restype = ctypes.c_int
        lib.oracle_free.argtypes = [ctypes.c_void_p]
        lib.oracle_free.restype = None
        lib.oracle_num_vertices.argtypes = [ctypes.c_void_p]
        lib.oracle_num_vertices.restype = ctypes.c_int64
        lib.oracle_num_arcs.argtypes = [ctypes.c_void_p]
        lib.oracle_num_arcs.restype = ctypes.c_int64
        lib.oracle_degrees.argtypes = [ctypes.c_void_p, _i64p]
        lib.oracle_degrees.restype = ctypes.c_int
        lib.oracle_khop.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, _i64p, _i64p, _i32p]
        lib.oracle_khop.restype = ctypes.c_int64
        lib.oracle_khop_many.argtypes = [ctypes.c_void_p, _i32p, ctypes.c_int64, ctypes.c_int32, _i64p,
                                         _i64p]
        lib.oracle_khop_many.restype = ctypes.c_int
        lib.oracle_khop_filtered.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                             ctypes.POINTER(ctypes.c_uint8), _i64p]
        lib.oracle_khop_filtered.restype = ctypes.c_int64
        _lib = lib
    return _lib


class OracleGraph:
    """The oracle's own adjacency of a tuple list (self-loops and duplicates dropped)."""

    def __init__(self, src, dst, n: int, directed: bool):
        lib = _load()
        src = np.ascontiguousarray(src, dtype=np.int32)
        dst = np.ascontiguousarray(dst, dtype=np.int32)
        if src.shape != dst.shape:
            raise ValueError("src and dst differ in length")
        h = ctypes.c_void_p()
        rc = lib.oracle_build(src.ctypes.data_as(_i32p), dst.ctypes.data_as(_i32p), src.shape[0], int(n),
                              1 if directed else 0, ctypes.byref(h))
        if rc != 0:
            raise ValueError(f"oracle_build failed ({rc})")
        self._h = h
        self.n = int(n)
        self.directed = bool(directed)

    @classmethod
    def from_edgelist(cls, el) -> "OracleGraph":
        return cls(el.src, el.dst, el.n, el.directed)

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.oracle_free(self._h)
            self._h = None

    @property
    def num_arcs(self) -> int:
        return int(_lib.oracle_num_arcs(self._h))

    def degrees(self) -> np.ndarray:
        out = np.empty(self.n, dtype=np.int64)
        _lib.oracle_degrees(self._h, out.ctypes.data_as(_i64p))
        return out

    def khop(self, seed: int, k: int):
        """(count, te, level_counts[k]) for one seed."""
        lv = np.zeros(max(k, 1), dtype=np.int64)
        te = ctypes.c_int64(0)
        c = _lib.oracle_khop(self._h, int(seed), int(k), lv.ctypes.data_as(_i64p), ctypes.byref(te), None)
        if c < 0:
            raise ValueError(f"oracle_khop failed ({c})")
        return int(c), int(te.value), lv[:k].copy()

    def distances(self, seed: int, k: int) -> np.ndarray:
        """dist(seed, v) for every v when it is at most k, else -1."""
        d = np.empty(self.n, dtype=np.int32)
        c = _lib.oracle_khop(self._h, int(seed), int(k), None, None, d.ctypes.data_as(_i32p))
        if c < 0:
            raise ValueError(f"oracle_khop failed ({c})")
        return d

    def khop_filtered(self, seed: int, k: int, allowed):
        """(count, te) of the search that enters only vertices with allowed[v] (the seed exempt)."""
        a = np.ascontiguousarray(allowed, dtype=np.uint8)
        if a.shape != (self.n,):
            raise ValueError("allowed must have one entry per vertex")
        te = ctypes.c_int64(0)
        c = _lib.oracle_khop_filtered(self._h, int(seed), int(k), a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                      ctypes.byref(te))
        if c < 0:
            raise ValueError(f"oracle_khop_filtered failed ({c})")
        return int(c), int(te.value)

    def count(self, seeds, k: int):
        """(counts, te) arrays for many seeds at one k."""
        seeds = np.ascontiguousarray(seeds, dtype=np.int32)
        counts = np.empty(seeds.shape[0], dtype=np.int64)
        te = np.empty(seeds.shape[0], dtype=np.int64)
        rc = _lib.oracle_khop_many(self._h, seeds.ctypes.data_as(_i32p), seeds.shape[0], int(k),
                                   counts.ctypes.data_as(_i64p), te.ctypes.data_as(_i64p))
        if rc != 0:
            raise ValueError(f"oracle_khop_many failed ({rc})")
        return counts, te
