"""Seeded synthetic inputs for the k-hop neighborhood count.

Raw edge tuples (R-MAT and a directed Chung-Lu power-law graph, shaped like
the paper's Graph500 and Twitter datasets of Section III) and seed draws
(uniform over non-isolated vertices, without replacement, as in the paper's
300/10-seed protocol of Section III).  Tuples keep their self-loops and
duplicates: each consumer builds its own adjacency.  Nothing here computes a
neighborhood; the module only feeds both the library and the oracle.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB_PATH = os.path.join(_HERE, "libgraphgen.so")
_lib = None

RMAT_A, RMAT_B, RMAT_C = 0.57, 0.19, 0.19

# Chung-Lu parameters for the 41.6M-vertex / 1.47B-edge Twitter-shaped graph:
# with x = 35 the top-ranked vertex expects m*ln(1+1/x)/ln((n+x)/x) ~ 2.96M edges.
TWITTER_N = 41_600_000
TWITTER_M = 1_470_000_000
TWITTER_X = 35.0


def build(force: bool = False) -> str:
    """Compile libgraphgen.so with gcc and OpenMP; returns its path."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        i32p = ctypes.POINTER(ctypes.c_int32)
        lib.gg_rmat.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, ctypes.c_uint64, ctypes.c_int, i32p, i32p]
        lib.gg_rmat.restype = ctypes.c_int
        lib.gg_chung_lu.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64,
                                    i32p, i32p]
        lib.gg_chung_lu.restype = ctypes.c_int
        lib.gg_permutation.argtypes = [ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint64, i32p]
        lib.gg_permutation.restype = ctypes.c_int
        lib.gg_draw_seeds.argtypes = [i32p, i32p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                      ctypes.c_uint64, ctypes.c_uint64, i32p,
                                      ctypes.POINTER(ctypes.c_int64)]
        lib.gg_draw_seeds.restype = ctypes.c_int64
        lib.gg_u64.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
        lib.gg_u64.restype = ctypes.c_uint64
        _lib = lib
    return _lib


def _p32(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


class EdgeList:
    """Raw tuples (src[i], dst[i]) over vertices [0, n); `directed` tells how they are read."""

    def __init__(self, src: np.ndarray, dst: np.ndarray, n: int, directed: bool, name: str = ""):
        self.src = np.ascontiguousarray(src, dtype=np.int32)
        self.dst = np.ascontiguousarray(dst, dtype=np.int32)
        self.n = int(n)
        self.directed = bool(directed)
        self.name = name

    @property
    def m(self) -> int:
        return int(self.src.shape[0])


def rmat(scale: int, edge_factor: int, seed: int = 1, a: float = RMAT_A, b: float = RMAT_B,
         c: float = RMAT_C, relabel: bool = True) -> EdgeList:
    """Undirected R-MAT tuples: m = edge_factor * 2**scale, Graph500-style relabelling."""
    n = 1 << scale
    m = edge_factor * n
    src = np.empty(m, dtype=np.int32)
    dst = np.empty(m, dtype=np.int32)
    rc = _load().gg_rmat(scale, edge_factor, a, b, c, seed, 1 if relabel else 0, _p32(src), _p32(dst))
    if rc != 0:
        raise ValueError(f"gg_rmat failed ({rc})")
    return EdgeList(src, dst, n, directed=False, name=f"rmat{scale}_ef{edge_factor}_s{seed}")


def chung_lu(n: int, m: int, x: float, seed: int = 1) -> EdgeList:
    """Directed Chung-Lu tuples with weights proportional to 1/(rank + x)."""
    src = np.empty(m, dtype=np.int32)
    dst = np.empty(m, dtype=np.int32)
    rc = _load().gg_chung_lu(n, m, x, seed, _p32(src), _p32(dst))
    if rc != 0:
        raise ValueError(f"gg_chung_lu failed ({rc})")
    return EdgeList(src, dst, n, directed=True, name=f"chunglu_n{n}_m{m}_x{x}_s{seed}")


def twitter_like(seed: int = 1) -> EdgeList:
    """The 41.6M-vertex, 1.47B-tuple directed power-law graph (about 11.8 GB of tuples)."""
    return chung_lu(TWITTER_N, TWITTER_M, TWITTER_X, seed)


def permutation(n: int, seed: int, tag: int) -> np.ndarray:
    out = np.empty(n, dtype=np.int32)
    if _load().gg_permutation(n, seed, tag, _p32(out)) != 0:
        raise ValueError("gg_permutation failed")
    return out


def draw_seeds(el: EdgeList, count: int, seed: int = 7, stream: int = 0) -> np.ndarray:
    """`count` distinct seeds, uniform over vertices with a non-self-loop tuple."""
    out = np.empty(max(count, 1), dtype=np.int32)
    nc = ctypes.c_int64(0)
    got = _load().gg_draw_seeds(_p32(el.src), _p32(el.dst), el.m, el.n, count, seed, stream,
                                _p32(out), ctypes.byref(nc))
    if got < 0:
        raise ValueError("gg_draw_seeds failed")
    return out[:got].copy()


def u64(seed: int, tag: int, i: int) -> int:
    return int(_load().gg_u64(seed, tag, i))
