"""Python binding of libkhop.so, the MI355X k-hop neighborhood-count engine.

Argument marshalling only: every step of the computation runs in the HIP
library.  The functions keep the C names (graph_load_csr, khop_count, ...);
`Graph` and `Server` wrap them for convenience.  Device arrays are passed as
torch tensors (device memory and streams only), host arrays as numpy arrays.

The library must be built (`python -m paper_1905_01294_amd.build`); importing
the binding without it raises ImportError -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkhop.so")

KHOP_OK = 0
KHOP_EINVAL = -1
KHOP_ERANGE = -2
KHOP_ENOMEM = -3
KHOP_EDEVICE = -4
KHOP_EBUSY = -5
KHOP_ETIMEDOUT = -6
KHOP_EINTERNAL = -7
STATUS_NAMES = {0: "KHOP_OK", -1: "KHOP_EINVAL", -2: "KHOP_ERANGE", -3: "KHOP_ENOMEM", -4: "KHOP_EDEVICE",
                -5: "KHOP_EBUSY", -6: "KHOP_ETIMEDOUT", -7: "KHOP_EINTERNAL"}

KHOP_UNDIRECTED = 0
KHOP_DIRECTED = 1

KHOP_OPT_DIRECTION = 1
KHOP_OPT_ALPHA = 2
KHOP_OPT_BETA = 3
KHOP_OPT_PULL_LIGHT = 4
KHOP_OPT_BATCH_SEEDS = 5
KHOP_OPT_BATCH_HEAVY = 6
KHOP_OPT_BATCH_PUSH = 7
KHOP_OPT_PULL_HEAVY = 8
KHOP_OPT_PUSH_ATOMIC = 9
KHOP_OPT_PLAIN_GRID = 10
KHOP_OPT_BATCH_GRID = 11
KHOP_OPT_PLAIN_PIPELINE = 12
KHOP_OPT_PLAIN_GRAPHS = 13
KHOP_DIR_AUTO = 0
KHOP_DIR_PUSH = 1
KHOP_DIR_PULL = 2
KHOP_SERVER_ROUTE = 1
KHOP_ROUTE_AUTO = 0
KHOP_ROUTE_BATCH = 1
KHOP_ROUTE_PLAIN = 2
KHOP_PATH_BATCH = 0
KHOP_PATH_SINGLE = 1
KHOP_LANE_SHORT = 0
KHOP_LANE_DEEP = 1
KHOP_LANE_SINGLE = 2
LANE_NAMES = {KHOP_LANE_SHORT: "batch_k_le_2", KHOP_LANE_DEEP: "batch_k_gt_2", KHOP_LANE_SINGLE: "single"}

# Every entry point declared in include/khop.h.
EXPORTS = ("graph_load_csr", "graph_load_csr_typed", "graph_free", "graph_info", "graph_degrees",
           "khop_count", "khop_count_dev", "khop_count_dev_noalloc", "khop_count_labeled", "khop_count_labeled_dev",
           "khop_count_batched", "khop_count_batched_dev", "khop_count_batched_labeled",
           "khop_bfs", "khop_bfs_dev", "khop_levels", "khop_levels_dev", "khop_neighborhood", "khop_neighborhood_dev",
           "khop_set_option", "khop_get_option", "khop_autotune", "khop_profile", "khop_profile_read",
           "khop_server_create", "khop_server_add_graph", "khop_server_set_option", "khop_server_submit",
           "khop_server_poll", "khop_server_drain", "khop_server_destroy", "khop_last_error", "khop_version",
           "khop_autotune_seconds", "khop_server_batch_bytes", "khop_server_stats")


class KhopError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double),
                ("algorithmic_bytes", ctypes.c_double)]


class ServerStat(ctypes.Structure):
    _fields_ = [("graph_id", ctypes.c_int32), ("lane", ctypes.c_int32), ("launches", ctypes.c_int64),
                ("queries", ctypes.c_int64), ("busy_ms", ctypes.c_double), ("max_ms", ctypes.c_double),
                ("words", ctypes.c_int32), ("queued", ctypes.c_int32)]


class Result(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("status", ctypes.c_int32), ("graph_id", ctypes.c_int32),
                ("seed", ctypes.c_int32), ("k", ctypes.c_int32), ("count", ctypes.c_int64),
                ("t_submit_ns", ctypes.c_int64), ("t_admit_ns", ctypes.c_int64), ("t_done_ns", ctypes.c_int64),
                ("path", ctypes.c_int32), ("reserved", ctypes.c_int32)]


_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_vp = ctypes.c_void_p


def _share_torch_runtime():
    """Load PyTorch's HIP runtime first when PyTorch is installed.

    PyTorch ships its own libamdhip64 with the same soname as the system one;
    whichever is loaded first serves the whole process.  Loading PyTorch's
    first makes libkhop bind to it too, so device pointers and streams handed
    over from PyTorch belong to the runtime that launches the kernels."""
    try:
        import torch  # noqa: F401
    except ImportError:
        pass


def _load():
    _share_torch_runtime()
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1905_01294_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    sig = {
        "graph_load_csr": ([_i32p, _i32p, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint32, ctypes.POINTER(_vp)],),
        "graph_load_csr_typed": ([_i32p, _i32p, ctypes.POINTER(ctypes.c_uint8), ctypes.c_int64, ctypes.c_int64,
                                  ctypes.c_uint32, ctypes.c_uint64, ctypes.POINTER(_vp)],),
        "graph_free": ([_vp],),
        "graph_info": ([_vp, _i64p, _i64p, _i32p],),
        "graph_degrees": ([_vp, _i64p],),
        "khop_count": ([_vp, _i32p, ctypes.c_int64, ctypes.c_int32, _i64p, _i64p],),
        "khop_count_dev": ([_vp, _vp, ctypes.c_int64, ctypes.c_int32, _vp, _vp, _vp],),
        "khop_count_dev_noalloc": ([_vp, _vp, ctypes.c_int64, ctypes.c_int32, _vp, _vp, _vp],),
        "khop_count_labeled": ([_vp, _i32p, ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(ctypes.c_uint64), _i64p,
                                _i64p],),
        "khop_count_labeled_dev": ([_vp, _vp, ctypes.c_int64, ctypes.c_int32, _vp, _vp, _vp, _vp],),
        "khop_count_batched": ([_vp, _i32p, _i32p, ctypes.c_int64, _i64p],),
        "khop_count_batched_dev": ([_vp, _vp, _vp, ctypes.c_int64, _vp, _vp],),
        "khop_count_batched_labeled": ([_vp, _i32p, _i32p, ctypes.c_int64, ctypes.POINTER(ctypes.c_uint64), _i64p],),
        "khop_bfs": ([_vp, ctypes.c_int32, ctypes.c_int32, _i32p, _i64p, _i32p],),
        "khop_bfs_dev": ([_vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp, _vp],),
        "khop_levels": ([_vp, ctypes.c_int32, ctypes.c_int32, _i64p],),
        "khop_levels_dev": ([_vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp],),
        "khop_neighborhood": ([_vp, ctypes.c_int32, ctypes.c_int32, _i32p, ctypes.c_int64, _i64p],),
        "khop_neighborhood_dev": ([_vp, ctypes.c_int32, ctypes.c_int32, _vp, ctypes.c_int64, _vp, _vp],),
        "khop_set_option": ([_vp, ctypes.c_int32, ctypes.c_int64],),
        "khop_get_option": ([_vp, ctypes.c_int32, _i64p],),
        "khop_autotune": ([_vp, ctypes.c_int32],),
        "khop_profile": ([_vp, ctypes.c_int32],),
        "khop_profile_read": ([_vp, ctypes.POINTER(KernelStat), ctypes.c_int32, _i32p],),
        "khop_server_create": ([ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(_vp)],),
        "khop_server_add_graph": ([_vp, _vp, _i32p],),
        "khop_server_set_option": ([_vp, ctypes.c_int32, ctypes.c_int64],),
        "khop_server_submit": ([_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                ctypes.POINTER(ctypes.c_uint64)],),
        "khop_server_poll": ([_vp, ctypes.POINTER(Result), ctypes.c_int64, _i64p],),
        "khop_server_stats": ([_vp, ctypes.POINTER(ServerStat), ctypes.c_int32, _i32p],),
        "khop_server_batch_bytes": ([_vp, ctypes.c_int32, _i64p],),
        "khop_server_drain": ([_vp, ctypes.c_int64],),
        "khop_server_destroy": ([_vp],),
    }
    for name, (args,) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.khop_last_error.argtypes = []
    lib.khop_last_error.restype = ctypes.c_char_p
    lib.khop_version.argtypes = []
    lib.khop_version.restype = ctypes.c_char_p
    lib.khop_autotune_seconds.argtypes = []
    lib.khop_autotune_seconds.restype = ctypes.c_double
    return lib


_lib = _load()


def library_path() -> str:
    return LIB_PATH


def _check(rc: int):
    if rc != KHOP_OK:
        raise KhopError(rc, (_lib.khop_last_error() or b"").decode())


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_i32p)


def _stream_ptr(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(getattr(stream, "cuda_stream", stream)))


def _dev_ptr(t, dtype_name):
    if t is None:
        return None
    if not t.is_cuda or str(t.dtype) != dtype_name or not t.is_contiguous():
        raise ValueError(f"expected a contiguous {dtype_name} device tensor")
    return ctypes.c_void_p(t.data_ptr())


# ------------------------------------------------------------------ C-named functions

def khop_version() -> str:
    return _lib.khop_version().decode()


def khop_autotune_seconds() -> float:
    """Seconds the last khop_autotune call spent searching (0 when served from the cache)."""
    return float(_lib.khop_autotune_seconds())


def khop_last_error() -> str:
    return (_lib.khop_last_error() or b"").decode()


def graph_load_csr(src, dst, num_vertices: int, flags: int = KHOP_UNDIRECTED):
    """Returns an opaque graph handle (ctypes.c_void_p)."""
    s, sp = _i32(src)
    d, dp = _i32(dst)
    if s.shape != d.shape:
        raise ValueError("src and dst differ in length")
    h = _vp()
    _check(_lib.graph_load_csr(sp, dp, s.shape[0], int(num_vertices), int(flags), ctypes.byref(h)))
    return h


def graph_load_csr_typed(src, dst, rel, num_vertices: int, rel_mask: int, flags: int = KHOP_UNDIRECTED):
    """A graph of the tuples whose relation type rel[i] (< 64) has its bit set in rel_mask."""
    s, sp = _i32(src)
    d, dp = _i32(dst)
    r = np.ascontiguousarray(rel, dtype=np.uint8)
    if s.shape != d.shape or s.shape != r.shape:
        raise ValueError("src, dst and rel differ in length")
    h = _vp()
    _check(_lib.graph_load_csr_typed(sp, dp, r.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), s.shape[0],
                                     int(num_vertices), int(flags), ctypes.c_uint64(int(rel_mask)), ctypes.byref(h)))
    return h


def label_bits(labeled, n: int) -> np.ndarray:
    """The vertex mask words (bit v % 64 of word v // 64) of a boolean array of n entries."""
    a = np.zeros(((int(n) + 63) // 64) * 64, dtype=bool)
    a[:int(n)] = np.asarray(labeled, dtype=bool)
    return np.packbits(a.reshape(-1, 8)[:, ::-1], axis=1).reshape(-1).view(np.uint64).copy()


def graph_free(h) -> None:
    _check(_lib.graph_free(h))


def graph_info(h):
    n, m, d = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
    _check(_lib.graph_info(h, ctypes.byref(n), ctypes.byref(m), ctypes.byref(d)))
    return int(n.value), int(m.value), bool(d.value)


def graph_degrees(h, n: int) -> np.ndarray:
    out = np.empty(n, dtype=np.int64)
    _check(_lib.graph_degrees(h, out.ctypes.data_as(_i64p)))
    return out


def khop_count(h, seeds, k: int, with_te: bool = False):
    s, sp = _i32(seeds)
    counts = np.empty(s.shape[0], dtype=np.int64)
    te = np.empty(s.shape[0], dtype=np.int64) if with_te else None
    _check(_lib.khop_count(h, sp, s.shape[0], int(k), counts.ctypes.data_as(_i64p),
                           te.ctypes.data_as(_i64p) if te is not None else None))
    return (counts, te) if with_te else counts


def khop_count_dev_noalloc(h, d_seeds, k: int, d_counts, d_te=None, stream=None) -> None:
    """khop_count_dev with the query context in the library's static scratch (no allocation)."""
    n = int(d_seeds.numel())
    if int(d_counts.numel()) < n or (d_te is not None and int(d_te.numel()) < n):
        raise ValueError("output tensors shorter than the seed tensor")
    _check(_lib.khop_count_dev_noalloc(h, _dev_ptr(d_seeds, "torch.int32"), n, int(k),
                                       _dev_ptr(d_counts, "torch.int64"), _dev_ptr(d_te, "torch.int64"),
                                       _stream_ptr(stream)))


def khop_count_dev(h, d_seeds, k: int, d_counts, d_te=None, stream=None) -> None:
    n = int(d_seeds.numel())
    if int(d_counts.numel()) < n or (d_te is not None and int(d_te.numel()) < n):
        raise ValueError("output tensors shorter than the seed tensor")
    _check(_lib.khop_count_dev(h, _dev_ptr(d_seeds, "torch.int32"), n, int(k), _dev_ptr(d_counts, "torch.int64"),
                               _dev_ptr(d_te, "torch.int64"), _stream_ptr(stream)))


def khop_count_labeled(h, seeds, k: int, bits, with_te: bool = False):
    s, sp = _i32(seeds)
    b = np.ascontiguousarray(bits, dtype=np.uint64)
    counts = np.empty(s.shape[0], dtype=np.int64)
    te = np.empty(s.shape[0], dtype=np.int64) if with_te else None
    _check(_lib.khop_count_labeled(h, sp, s.shape[0], int(k), b.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                   counts.ctypes.data_as(_i64p), te.ctypes.data_as(_i64p) if te is not None else None))
    return (counts, te) if with_te else counts


def khop_count_labeled_dev(h, d_seeds, k: int, d_bits, d_counts, d_te=None, stream=None) -> None:
    n = int(d_seeds.numel())
    if int(d_counts.numel()) < n or (d_te is not None and int(d_te.numel()) < n):
        raise ValueError("output tensors shorter than the seed tensor")
    _check(_lib.khop_count_labeled_dev(h, _dev_ptr(d_seeds, "torch.int32"), n, int(k), _dev_ptr(d_bits, "torch.int64"),
                                       _dev_ptr(d_counts, "torch.int64"), _dev_ptr(d_te, "torch.int64"),
                                       _stream_ptr(stream)))


def khop_count_batched(h, seeds, ks) -> np.ndarray:
    s, sp = _i32(seeds)
    kk, kp = _i32(np.broadcast_to(np.asarray(ks, dtype=np.int32), s.shape))
    counts = np.empty(s.shape[0], dtype=np.int64)
    _check(_lib.khop_count_batched(h, sp, kp, s.shape[0], counts.ctypes.data_as(_i64p)))
    return counts


def khop_count_batched_labeled(h, seeds, ks, bits) -> np.ndarray:
    s, sp = _i32(seeds)
    kk, kp = _i32(np.broadcast_to(np.asarray(ks, dtype=np.int32), s.shape))
    b = np.ascontiguousarray(bits, dtype=np.uint64)
    counts = np.empty(s.shape[0], dtype=np.int64)
    _check(_lib.khop_count_batched_labeled(h, sp, kp, s.shape[0], b.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                           counts.ctypes.data_as(_i64p)))
    return counts


def khop_count_batched_dev(h, d_seeds, d_ks, d_counts, stream=None) -> None:
    n = int(d_seeds.numel())
    if int(d_ks.numel()) < n or int(d_counts.numel()) < n:
        raise ValueError("tensors shorter than the seed tensor")
    _check(_lib.khop_count_batched_dev(h, _dev_ptr(d_seeds, "torch.int32"), _dev_ptr(d_ks, "torch.int32"), n,
                                       _dev_ptr(d_counts, "torch.int64"), _stream_ptr(stream)))


def khop_bfs(h, seed: int, n: int, max_depth: int = -1):
    """(dist int32[n], count, depth) of a breadth-first search from seed."""
    dist = np.empty(int(n), dtype=np.int32)
    c, d = ctypes.c_int64(), ctypes.c_int32()
    _check(_lib.khop_bfs(h, int(seed), int(max_depth), dist.ctypes.data_as(_i32p), ctypes.byref(c),
                         ctypes.byref(d)))
    return dist, int(c.value), int(d.value)


def khop_bfs_dev(h, seed: int, d_dist, max_depth: int = -1, d_count=None, d_depth=None, stream=None) -> None:
    _check(_lib.khop_bfs_dev(h, int(seed), int(max_depth), _dev_ptr(d_dist, "torch.int32"),
                             _dev_ptr(d_count, "torch.int64"), _dev_ptr(d_depth, "torch.int32"),
                             _stream_ptr(stream)))


def khop_levels(h, seed: int, k: int) -> np.ndarray:
    """int64[k]: the number of vertices at distance exactly 1..k."""
    out = np.zeros(max(int(k), 0), dtype=np.int64)
    _check(_lib.khop_levels(h, int(seed), int(k), out.ctypes.data_as(_i64p) if k > 0 else None))
    return out


def khop_levels_dev(h, seed: int, k: int, d_levels, stream=None) -> None:
    if k > 0 and int(d_levels.numel()) < k:
        raise ValueError("level tensor shorter than k")
    _check(_lib.khop_levels_dev(h, int(seed), int(k), _dev_ptr(d_levels, "torch.int64"), _stream_ptr(stream)))


def khop_neighborhood(h, seed: int, k: int, capacity: int):
    """(ascending ids of the k-hop neighborhood, at most `capacity` of them; its full size)."""
    ids = np.empty(max(int(capacity), 1), dtype=np.int32)
    c = ctypes.c_int64()
    _check(_lib.khop_neighborhood(h, int(seed), int(k), ids.ctypes.data_as(_i32p), int(capacity), ctypes.byref(c)))
    return ids[:min(int(c.value), int(capacity))].copy(), int(c.value)


def khop_neighborhood_dev(h, seed: int, k: int, d_ids, d_count, stream=None) -> None:
    _check(_lib.khop_neighborhood_dev(h, int(seed), int(k), _dev_ptr(d_ids, "torch.int32"), int(d_ids.numel()),
                                      _dev_ptr(d_count, "torch.int64"), _stream_ptr(stream)))


def khop_set_option(h, option: int, value: int) -> None:
    _check(_lib.khop_set_option(h, int(option), int(value)))


def khop_get_option(h, option: int) -> int:
    v = ctypes.c_int64()
    _check(_lib.khop_get_option(h, int(option), ctypes.byref(v)))
    return int(v.value)


def khop_autotune(h, seeds_per_launch: int = 0) -> None:
    _check(_lib.khop_autotune(h, int(seeds_per_launch)))


def khop_profile(h, enable: bool) -> None:
    _check(_lib.khop_profile(h, 1 if enable else 0))


def khop_profile_read(h):
    buf = (KernelStat * 32)()
    n = ctypes.c_int32()
    _check(_lib.khop_profile_read(h, buf, 32, ctypes.byref(n)))
    return {buf[i].name.decode(): {"launches": int(buf[i].launches), "total_ms": float(buf[i].total_ms),
                                   "algorithmic_bytes": float(buf[i].algorithmic_bytes)} for i in range(n.value)}


def khop_server_create(mem_budget_bytes: int, max_batch_seeds: int = 1024):
    h = _vp()
    _check(_lib.khop_server_create(int(mem_budget_bytes), int(max_batch_seeds), ctypes.byref(h)))
    return h


def khop_server_add_graph(server, graph) -> int:
    gid = ctypes.c_int32()
    _check(_lib.khop_server_add_graph(server, graph, ctypes.byref(gid)))
    return int(gid.value)


def khop_server_set_option(server, option: int, value: int) -> None:
    _check(_lib.khop_server_set_option(server, int(option), int(value)))


def khop_server_submit(server, graph_id: int, seed: int, k: int, deadline_ns: int = 0) -> int:
    t = ctypes.c_uint64()
    _check(_lib.khop_server_submit(server, int(graph_id), int(seed), int(k), int(deadline_ns), ctypes.byref(t)))
    return int(t.value)


def khop_server_poll(server, max_results: int = 4096):
    buf = (Result * max_results)()
    n = ctypes.c_int64()
    _check(_lib.khop_server_poll(server, buf, max_results, ctypes.byref(n)))
    return [buf[i] for i in range(n.value)]


def khop_server_drain(server, timeout_ms: int = 60000) -> None:
    _check(_lib.khop_server_drain(server, int(timeout_ms)))


def khop_server_destroy(server) -> None:
    _check(_lib.khop_server_destroy(server))


# ------------------------------------------------------------------ convenience wrappers

class Graph:
    """A device-resident graph built from raw edge tuples."""

    def __init__(self, src, dst, num_vertices: int, directed: bool = False):
        self._h = graph_load_csr(src, dst, num_vertices, KHOP_DIRECTED if directed else KHOP_UNDIRECTED)
        self.n, self.num_arcs, self.directed = graph_info(self._h)

    @classmethod
    def typed(cls, src, dst, rel, num_vertices: int, rel_mask: int, directed: bool = False) -> "Graph":
        """The graph of the tuples whose relation type rel[i] has its bit set in rel_mask."""
        self = cls.__new__(cls)
        self._h = graph_load_csr_typed(src, dst, rel, num_vertices, rel_mask,
                                       KHOP_DIRECTED if directed else KHOP_UNDIRECTED)
        self.n, self.num_arcs, self.directed = graph_info(self._h)
        return self

    @classmethod
    def from_edgelist(cls, el) -> "Graph":
        return cls(el.src, el.dst, el.n, el.directed)

    @property
    def handle(self):
        return self._h

    def free(self):
        if self._h is not None:
            graph_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def degrees(self) -> np.ndarray:
        return graph_degrees(self._h, self.n)

    def count(self, seeds, k: int, with_te: bool = False):
        return khop_count(self._h, seeds, k, with_te)

    def count_dev(self, d_seeds, k: int, d_counts, d_te=None, stream=None):
        khop_count_dev(self._h, d_seeds, k, d_counts, d_te, stream)

    def count_dev_noalloc(self, d_seeds, k: int, d_counts, d_te=None, stream=None):
        khop_count_dev_noalloc(self._h, d_seeds, k, d_counts, d_te, stream)

    def count_labeled(self, seeds, k: int, labeled, with_te: bool = False):
        """Counts in the subgraph of the vertices with labeled[v] true (the seeds exempt)."""
        return khop_count_labeled(self._h, seeds, k, label_bits(labeled, self.n), with_te)

    def count_labeled_dev(self, d_seeds, k: int, d_bits, d_counts, d_te=None, stream=None):
        if int(d_bits.numel()) < (self.n + 63) // 64:
            raise ValueError("mask tensor shorter than ceil(n / 64) words")
        khop_count_labeled_dev(self._h, d_seeds, k, d_bits, d_counts, d_te, stream)

    def count_batched(self, seeds, ks):
        return khop_count_batched(self._h, seeds, ks)

    def count_batched_labeled(self, seeds, ks, labeled):
        """Batched counts in the subgraph of the vertices with labeled[v] true (the seeds exempt)."""
        return khop_count_batched_labeled(self._h, seeds, ks, label_bits(labeled, self.n))

    def count_batched_dev(self, d_seeds, d_ks, d_counts, stream=None):
        khop_count_batched_dev(self._h, d_seeds, d_ks, d_counts, stream)

    def bfs(self, seed: int, max_depth: int = -1):
        return khop_bfs(self._h, seed, self.n, max_depth)

    def bfs_dev(self, seed: int, d_dist, max_depth: int = -1, d_count=None, d_depth=None, stream=None):
        if int(d_dist.numel()) < self.n:
            raise ValueError("distance tensor shorter than the vertex count")
        khop_bfs_dev(self._h, seed, d_dist, max_depth, d_count, d_depth, stream)

    def levels(self, seed: int, k: int) -> np.ndarray:
        return khop_levels(self._h, seed, k)

    def levels_dev(self, seed: int, k: int, d_levels, stream=None):
        khop_levels_dev(self._h, seed, k, d_levels, stream)

    def neighborhood(self, seed: int, k: int, capacity: int = None):
        """Ascending ids of { v : 1 <= dist(seed, v) <= k } (k < 0: the whole reach)."""
        ids, c = khop_neighborhood(self._h, seed, k, self.n if capacity is None else capacity)
        return ids if capacity is None else (ids, c)

    def neighborhood_dev(self, seed: int, k: int, d_ids, d_count, stream=None):
        khop_neighborhood_dev(self._h, seed, k, d_ids, d_count, stream)

    def set_option(self, option: int, value: int):
        khop_set_option(self._h, option, value)

    def get_option(self, option: int) -> int:
        return khop_get_option(self._h, option)

    def autotune(self, seeds_per_launch: int = 0):
        khop_autotune(self._h, seeds_per_launch)

    def profile(self, enable: bool):
        khop_profile(self._h, enable)

    def profile_read(self):
        return khop_profile_read(self._h)


class Server:
    """Continuous-batching k-hop server over resident graphs (see khop_server_* in include/khop.h)."""

    def __init__(self, mem_budget_bytes: int, max_batch_seeds: int = 1024):
        self._h = khop_server_create(mem_budget_bytes, max_batch_seeds)
        self._graphs = []

    def add_graph(self, graph: "Graph") -> int:
        gid = khop_server_add_graph(self._h, graph.handle)
        self._graphs.append(graph)  # keep the graph alive while served
        return gid

    def set_option(self, option: int, value: int):
        khop_server_set_option(self._h, option, value)

    def submit(self, graph_id: int, seed: int, k: int, deadline_ns: int = 0) -> int:
        return khop_server_submit(self._h, graph_id, seed, k, deadline_ns)

    def poll(self, max_results: int = 4096):
        return khop_server_poll(self._h, max_results)

    def drain(self, timeout_ms: int = 60000):
        khop_server_drain(self._h, timeout_ms)

    def stats(self):
        """Per-lane counters: a list of dicts (graph_id, lane name, launches, queries, busy_ms, max_ms, words,
        queued)."""
        return khop_server_stats(self._h)

    def close(self):
        if self._h is not None:
            khop_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def khop_server_stats(h, max_lanes: int = 256):
    buf = (ServerStat * max_lanes)()
    n = ctypes.c_int32(0)
    _check(_lib.khop_server_stats(h, buf, max_lanes, ctypes.byref(n)))
    return [{"graph_id": x.graph_id, "lane": LANE_NAMES.get(x.lane, x.lane), "launches": x.launches,
             "queries": x.queries, "busy_ms": x.busy_ms, "max_ms": x.max_ms, "words": x.words, "queued": x.queued}
            for x in buf[:n.value]]


def khop_server_batch_bytes(graph_handle, words: int) -> int:
    """Device bytes of one server batch context of `words` 64-query words for the graph."""
    b = ctypes.c_int64(0)
    _check(_lib.khop_server_batch_bytes(graph_handle, int(words), ctypes.byref(b)))
    return int(b.value)


def monotonic_ns() -> int:
    """CLOCK_MONOTONIC in nanoseconds, the clock of the server's time stamps and deadlines."""
    import time
    return time.clock_gettime_ns(time.CLOCK_MONOTONIC)
