"""Python binding of the evq C ABI (include/evq.h): argument marshalling only.

Every step of a query runs in the HIP library (libevq.so, gfx950).  Device
buffers are torch tensors (uint32 values held in int32 tensors) and the
stream is torch's current stream.  Importing this package fails loudly when
the library has not been built: there is no fallback path.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("EVQ_LIBRARY") or os.path.join(_HERE, "libevq.so")

SSSP, BFS, SSWP, SSNP, VITERBI = 0, 1, 2, 3, 4
ALGOS = {"sssp": SSSP, "bfs": BFS, "sswp": SSWP, "ssnp": SSNP, "viterbi": VITERBI}
INF = 0xFFFFFFFF
BUCKET_WIDTH_AUTO = 0xFFFFFFFF  # evq_tuning.bucket_width: derived from the graph

EVQ_OK, EVQ_EINVAL, EVQ_ERANGE, EVQ_ENOMEM, EVQ_EDEVICE, EVQ_ENOCONV = 0, -1, -2, -3, -4, -5
EVQ_ECANCELED, EVQ_EBUSY = -6, -7
_STATUS = {EVQ_EINVAL: "EINVAL", EVQ_ERANGE: "ERANGE", EVQ_ENOMEM: "ENOMEM", EVQ_EDEVICE: "EDEVICE",
           EVQ_ENOCONV: "ENOCONV", EVQ_ECANCELED: "ECANCELED", EVQ_EBUSY: "EBUSY"}

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it first (python paper_2502_10579_amd/_build.py)")


class Edge(ctypes.Structure):
    _fields_ = [("src", ctypes.c_uint32), ("dst", ctypes.c_uint32), ("w", ctypes.c_uint32)]


class Batch(ctypes.Structure):
    _fields_ = [("dels", ctypes.POINTER(Edge)), ("n_del", ctypes.c_uint64),
                ("adds", ctypes.POINTER(Edge)), ("n_add", ctypes.c_uint64)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Allocator(ctypes.Structure):
    """evq_allocator: the caller's device allocator for a graph's arrays."""
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", ctypes.c_void_p)]


class GraphInfo(ctypes.Structure):
    _fields_ = [("num_vertices", ctypes.c_uint32), ("num_snapshots", ctypes.c_uint32),
                ("mask_words", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("num_edges", ctypes.c_uint64), ("num_partial", ctypes.c_uint64),
                ("device_bytes", ctypes.c_uint64), ("build_ms", ctypes.c_double),
                ("first_snapshot", ctypes.c_uint64)]


class QueryStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("ms_total", "ms_cap", "ms_cup", "ms_compact", "ms_relax",
                                               "ms_writeback")] + \
               [(n, ctypes.c_uint64) for n in ("n_unstable", "n_seed_edges", "n_relax_edges", "iters_cap",
                                               "iters_cup", "iters_relax", "edges_cap", "edges_cup",
                                               "edge_visits_relax", "lane_relaxations", "updates_cap",
                                               "updates_cup", "items_cap", "items_cup", "seed_visits_cup",
                                               "subwindows")]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class QueryDesc(ctypes.Structure):
    _fields_ = [("algo", ctypes.c_uint32), ("source", ctypes.c_uint32), ("win_begin", ctypes.c_uint32),
                ("win_len", ctypes.c_uint32)]


class ResultC(ctypes.Structure):
    _fields_ = [("algo", ctypes.c_uint32), ("source", ctypes.c_uint32), ("win_begin", ctypes.c_uint32),
                ("win_len", ctypes.c_uint32), ("num_vertices", ctypes.c_uint32), ("n_unstable", ctypes.c_uint32),
                ("row_stride", ctypes.c_uint32), ("reserved", ctypes.c_uint32), ("d_rcap", ctypes.c_void_p),
                ("d_unstable", ctypes.c_void_p), ("d_x", ctypes.c_void_p)]


class BatchConfig(ctypes.Structure):
    _fields_ = [("lanes", ctypes.c_uint32), ("chunk", ctypes.c_uint32), ("blocks", ctypes.c_uint32),
                ("group", ctypes.c_uint32)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_uint32), ("max_batch", ctypes.c_uint32), ("max_inflight", ctypes.c_uint32),
                ("max_groups", ctypes.c_uint32), ("mem_budget", ctypes.c_uint64), ("max_queued", ctypes.c_uint32),
                ("queue_hi", ctypes.c_uint32)]


class Completion(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("status", ctypes.c_int32), ("group_size", ctypes.c_uint32),
                ("t_arrival_ms", ctypes.c_double), ("t_admit_ms", ctypes.c_double), ("t_bounds_ms", ctypes.c_double),
                ("t_done_ms", ctypes.c_double),
                ("n_unstable", ctypes.c_uint64), ("iters_relax", ctypes.c_uint64), ("result", ResultC)]


class Tuning(ctypes.Structure):
    _fields_ = [("pull_frac", ctypes.c_double), ("split_frac", ctypes.c_double), ("split_min", ctypes.c_uint32),
                ("launch_depth", ctypes.c_uint32), ("direct_tasks", ctypes.c_uint32),
                ("append_rebuild", ctypes.c_uint32), ("trace_loops", ctypes.c_uint32),
                ("delta", ctypes.c_uint32 * 5), ("heavy", ctypes.c_uint32 * 5), ("append_edges", ctypes.c_uint32),
                ("relax_staged", ctypes.c_uint32), ("append_items", ctypes.c_uint32),
                ("bucket_width", ctypes.c_uint32), ("vertex_order", ctypes.c_uint32)]


class KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_uint64), ("total_ms", ctypes.c_double)]


_lib = ctypes.CDLL(LIB_PATH)
_P = ctypes.c_void_p
_lib.evq_build.restype = ctypes.c_int32
_lib.evq_build.argtypes = [ctypes.c_uint32, ctypes.POINTER(Edge), ctypes.c_uint64, ctypes.POINTER(Batch),
                           ctypes.c_uint32, ctypes.POINTER(Allocator), _P, ctypes.POINTER(_P)]
_lib.evq_graph_info_get.restype = ctypes.c_int32
_lib.evq_graph_info_get.argtypes = [_P, ctypes.POINTER(GraphInfo)]
_lib.evq_graph_export.restype = ctypes.c_int32
_lib.evq_graph_export.argtypes = [_P, _P, _P, _P, _P, _P, _P]
for _name in ("evq_query", "evq_query_plain", "evq_query_sequential"):
    getattr(_lib, _name).restype = ctypes.c_int32
    getattr(_lib, _name).argtypes = [_P, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, _P,
                                     ctypes.POINTER(QueryStats), _P]
_lib.evq_query_noalloc.restype = ctypes.c_int32
_lib.evq_query_noalloc.argtypes = [_P, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, _P, _P]
_lib.evq_query_bounds.restype = ctypes.c_int32
_lib.evq_query_bounds.argtypes = [_P, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, _P, _P,
                                  _P]
_lib.evq_query_batch.restype = ctypes.c_int32
_lib.evq_query_batch.argtypes = [_P, ctypes.POINTER(QueryDesc), ctypes.c_uint32, ctypes.POINTER(ResultC),
                                 ctypes.POINTER(QueryStats), _P]
for _name in ("evq_result_expand", "evq_expand"):
    getattr(_lib, _name).restype = ctypes.c_int32
    getattr(_lib, _name).argtypes = [ctypes.POINTER(ResultC), _P, _P]
_lib.evq_result_free.restype = ctypes.c_int32
_lib.evq_result_free.argtypes = [ctypes.POINTER(ResultC), _P]
_lib.evq_batch_config_get.restype = ctypes.c_int32
_lib.evq_batch_config_get.argtypes = [ctypes.POINTER(BatchConfig)]
_lib.evq_batch_config_set.restype = ctypes.c_int32
_lib.evq_batch_config_set.argtypes = [ctypes.POINTER(BatchConfig)]
_lib.evq_append.restype = ctypes.c_int32
_lib.evq_append.argtypes = [_P, ctypes.POINTER(Batch), _P]
_lib.evq_server_create.restype = ctypes.c_int32
_lib.evq_server_create.argtypes = [_P, ctypes.POINTER(ServerConfig), ctypes.POINTER(_P)]
_lib.evq_server_submit.restype = ctypes.c_int32
_lib.evq_server_submit.argtypes = [_P, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                   ctypes.POINTER(ctypes.c_uint64)]
_lib.evq_server_poll.restype = ctypes.c_int
_lib.evq_server_poll.argtypes = [_P, ctypes.POINTER(Completion), ctypes.c_int, ctypes.c_int]
_lib.evq_server_pending.restype = ctypes.c_int32
_lib.evq_server_pending.argtypes = [_P, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint32)]
_lib.evq_server_destroy.restype = ctypes.c_int32
_lib.evq_server_destroy.argtypes = [_P]
_lib.evq_batch_autotune.restype = ctypes.c_int32
_lib.evq_batch_autotune.argtypes = [_P, ctypes.POINTER(QueryDesc), ctypes.c_uint32, ctypes.POINTER(BatchConfig),
                                    ctypes.POINTER(ctypes.c_double), _P]
_lib.evq_free.restype = None
_lib.evq_free.argtypes = [_P]
_lib.evq_last_error.restype = ctypes.c_char_p
_lib.evq_last_error.argtypes = []
_lib.evq_timing_enable.restype = None
_lib.evq_timing_enable.argtypes = [ctypes.c_int]
_lib.evq_timing_reset.restype = None
_lib.evq_timing_reset.argtypes = []
_lib.evq_timing_report.restype = ctypes.c_int
_lib.evq_timing_report.argtypes = [ctypes.POINTER(KernelTime), ctypes.c_int]
_lib.evq_tuning_get.restype = ctypes.c_int32
_lib.evq_tuning_get.argtypes = [ctypes.POINTER(Tuning)]
_lib.evq_tuning_set.restype = ctypes.c_int32
_lib.evq_tuning_set.argtypes = [ctypes.POINTER(Tuning)]
_lib.evq_gather_ceiling.restype = ctypes.c_int32
_lib.evq_gather_ceiling.argtypes = [_P, ctypes.c_uint32, ctypes.POINTER(ctypes.c_double), _P]

EXPORTED = ["evq_build", "evq_graph_info_get", "evq_graph_export", "evq_query", "evq_query_bounds",
            "evq_query_plain", "evq_query_sequential", "evq_query_batch", "evq_result_expand", "evq_result_free",
            "evq_batch_config_get", "evq_batch_config_set", "evq_batch_autotune", "evq_expand", "evq_append", "evq_server_create",
            "evq_server_submit", "evq_server_poll", "evq_server_pending", "evq_server_destroy", "evq_free", "evq_last_error", "evq_timing_enable",
            "evq_timing_reset", "evq_timing_report", "evq_gather_ceiling", "evq_tuning_get", "evq_tuning_set", "evq_query_noalloc"]


class EvqError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


def _check(rc):
    if rc != EVQ_OK:
        raise EvqError(rc, _lib.evq_last_error().decode(errors="replace"))


def last_error() -> str:
    return _lib.evq_last_error().decode(errors="replace")


def _edges(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.uint32).reshape(-1, 3))
    return a, (a.ctypes.data_as(ctypes.POINTER(Edge)) if len(a) else None)


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    import torch
    if torch.cuda.is_available():
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(0)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class Graph:
    """Versioned graph of K snapshots resident on the current device (evq_build)."""

    def __init__(self, num_vertices, base, dels, adds, stream=None, allocator=None):
        """allocator: None, or an Allocator whose callbacks stay referenced by the caller for the
        graph's whole life (evq_build's `alloc`)."""
        if len(dels) != len(adds):
            raise ValueError("dels and adds must have one entry per batch")
        keep = []
        b, bp = _edges(base)
        keep.append(b)
        batches = (Batch * max(len(dels), 1))()
        for i, (d, a) in enumerate(zip(dels, adds)):
            d, dp = _edges(d)
            a, ap = _edges(a)
            keep += [d, a]
            batches[i] = Batch(dp, len(d), ap, len(a))
        h = ctypes.c_void_p()
        _check(_lib.evq_build(num_vertices, bp, len(b), batches, len(dels),
                              ctypes.byref(allocator) if allocator is not None else None, _stream(stream),
                              ctypes.byref(h)))
        self._h = h
        self._allocator = allocator
        self.num_vertices = num_vertices
        self.K = len(dels)

    def append(self, dels, adds, stream=None):
        """Advance the held snapshots by one batch (evq_append)."""
        d, dp = _edges(dels)
        a, ap = _edges(adds)
        b = Batch(dp, len(d), ap, len(a))
        _check(_lib.evq_append(self._h, ctypes.byref(b), _stream(stream)))

    @property
    def first(self) -> int:
        """Global id of the oldest snapshot held."""
        return self.info["first_snapshot"]

    @classmethod
    def from_instance(cls, inst, stream=None):
        return cls(inst.num_vertices, inst.base, inst.dels, inst.adds, stream)

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.evq_free(self._h)
            self._h = None

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def info(self) -> dict:
        gi = GraphInfo()
        _check(_lib.evq_graph_info_get(self._h, ctypes.byref(gi)))
        return {k: getattr(gi, k) for k, _ in GraphInfo._fields_ if k != "reserved"}

    def export(self, stream=None) -> dict:
        """Host copy of the versioned graph: row_ptr, row_split, col, w, mask (E, mask_words)."""
        inf = self.info
        V, E, MW = inf["num_vertices"], inf["num_edges"], inf["mask_words"]
        out = dict(row_ptr=np.empty(V + 1, np.uint32), row_split=np.empty(V, np.uint32),
                   col=np.empty(max(E, 1), np.uint32), w=np.empty(max(E, 1), np.uint32),
                   mask=np.empty((max(E, 1), MW), np.uint64))
        _check(_lib.evq_graph_export(self._h, *(ctypes.c_void_p(out[k].ctypes.data)
                                               for k in ("row_ptr", "row_split", "col", "w", "mask")),
                                     _stream(stream)))
        for k in ("col", "w", "mask"):
            out[k] = out[k][:E]
        return out

    def gather_ceiling(self, launches: int = 5, stream=None) -> float:
        """Edges/s of the expansion's per-edge memory operations alone over this graph (measurement only)."""
        r = ctypes.c_double(0.0)
        _check(_lib.evq_gather_ceiling(self._h, launches, ctypes.byref(r), _stream(stream)))
        return r.value

    def _alloc(self, L, out):
        import torch
        if out is None:
            out = torch.empty((self.num_vertices, L), dtype=torch.int32, device="cuda")
        if out.dtype != torch.int32 or not out.is_cuda or not out.is_contiguous() or \
                out.numel() != self.num_vertices * L:
            raise ValueError("out must be a contiguous int32 CUDA tensor of V * L elements")
        return out

    def _window(self, win_begin, win_len):
        """Default window: from the oldest held snapshot (win_begin None) to the newest (win_len None)."""
        if win_begin is None:
            win_begin = self.first
        if win_len is None:
            win_len = self.first + self.K - win_begin
        return win_begin, win_len

    def query(self, algo, source, win_begin=None, win_len=None, out=None, stats=False, stream=None):
        """values (V, L) int32 tensor holding uint32 values (evq_query)."""
        algo = ALGOS.get(algo, algo)
        win_begin, L = self._window(win_begin, win_len)
        out = self._alloc(L, out)
        st = QueryStats() if stats else None
        _check(_lib.evq_query(self._h, algo, source, win_begin, L, _ptr(out),
                              ctypes.byref(st) if st is not None else None, _stream(stream)))
        return (out, st.as_dict()) if stats else out

    def query_noalloc(self, algo, source, win_begin=None, win_len=None, out=None, stream=None):
        """Same output as query(), from a call that allocates nothing (evq_query_noalloc); it returns
        once the values are complete.  `out` should be allocated beforehand by callers that cannot
        allocate."""
        algo = ALGOS.get(algo, algo)
        win_begin, L = self._window(win_begin, win_len)
        out = self._alloc(L, out)
        _check(_lib.evq_query_noalloc(self._h, algo, source, win_begin, L, _ptr(out), _stream(stream)))
        return out

    def query_plain(self, algo, source, win_begin=None, win_len=None, out=None, stats=False, stream=None):
        """Same output as query(), without the intersection-union analysis (evq_query_plain)."""
        algo = ALGOS.get(algo, algo)
        win_begin, L = self._window(win_begin, win_len)
        out = self._alloc(L, out)
        st = QueryStats() if stats else None
        _check(_lib.evq_query_plain(self._h, algo, source, win_begin, L, _ptr(out),
                                    ctypes.byref(st) if st is not None else None, _stream(stream)))
        return (out, st.as_dict()) if stats else out

    def query_sequential(self, algo, source, win_begin=None, win_len=None, out=None, stats=False, stream=None):
        """Same output as query(), relaxing the window's snapshots one after another (evq_query_sequential)."""
        algo = ALGOS.get(algo, algo)
        win_begin, L = self._window(win_begin, win_len)
        out = self._alloc(L, out)
        st = QueryStats() if stats else None
        _check(_lib.evq_query_sequential(self._h, algo, source, win_begin, L, _ptr(out),
                                         ctypes.byref(st) if st is not None else None, _stream(stream)))
        return (out, st.as_dict()) if stats else out

    def query_bounds(self, algo, source, win_begin=None, win_len=None, stream=None):
        """(R_cap, R_cup) int32 tensors of V values (evq_query_bounds)."""
        import torch
        algo = ALGOS.get(algo, algo)
        win_begin, L = self._window(win_begin, win_len)
        rcap = torch.empty(self.num_vertices, dtype=torch.int32, device="cuda")
        rcup = torch.empty(self.num_vertices, dtype=torch.int32, device="cuda")
        _check(_lib.evq_query_bounds(self._h, algo, source, win_begin, L, _ptr(rcap), _ptr(rcup), _stream(stream)))
        return rcap, rcup

    def query_batch(self, queries, stats=False, stream=None):
        """Answer many queries (evq_query_batch).  queries: iterable of (algo, source, win_begin, win_len).
        Returns a list of Result (compact, device-resident), and per-query stats dicts if asked."""
        qs = list(queries)
        n = len(qs)
        descs = (QueryDesc * max(n, 1))()
        for i, (a, src, b, L) in enumerate(qs):
            descs[i] = QueryDesc(ALGOS.get(a, a), src, b, L)
        res = (ResultC * max(n, 1))()
        st = (QueryStats * max(n, 1))() if stats else None
        _check(_lib.evq_query_batch(self._h, descs, n, res, st, _stream(stream)))
        out = [Result(res[i]) for i in range(n)]
        return (out, [st[i].as_dict() for i in range(n)]) if stats else out


    def autotune_batch(self, queries, stream=None):
        """Time query_batch's execution choices on these queries and install the fastest (evq_batch_autotune).
        Returns (config dict, best milliseconds)."""
        qs = list(queries)
        descs = (QueryDesc * max(len(qs), 1))()
        for i, (a, src, b, L) in enumerate(qs):
            descs[i] = QueryDesc(ALGOS.get(a, a), src, b, L)
        c = BatchConfig()
        ms = ctypes.c_double()
        _check(_lib.evq_batch_autotune(self._h, descs, len(qs), ctypes.byref(c), ctypes.byref(ms), _stream(stream)))
        return {"lanes": c.lanes, "chunk": c.chunk, "blocks": c.blocks, "group": c.group}, ms.value


class Result:
    """Compact result of one batched query (evq_result); device memory is released by free() or on deletion."""

    def __init__(self, c):
        self._c = ResultC()
        ctypes.memmove(ctypes.byref(self._c), ctypes.byref(c), ctypes.sizeof(ResultC))

    @property
    def info(self) -> dict:
        return {k: getattr(self._c, k) for k in ("algo", "source", "win_begin", "win_len", "num_vertices",
                                                  "n_unstable", "row_stride")}

    def expand(self, out=None, stream=None):
        """values (V, win_len) int32 tensor (evq_result_expand)."""
        import torch
        V, L = self._c.num_vertices, self._c.win_len
        if out is None:
            out = torch.empty((V, L), dtype=torch.int32, device="cuda")
        if out.dtype != torch.int32 or not out.is_cuda or not out.is_contiguous() or out.numel() != V * L:
            raise ValueError("out must be a contiguous int32 CUDA tensor of V * L elements")
        _check(_lib.evq_expand(ctypes.byref(self._c), _ptr(out), _stream(stream)))
        return out

    def free(self, stream=None):
        if self._c.d_rcap and _lib is not None:
            _check(_lib.evq_result_free(ctypes.byref(self._c), _stream(stream)))

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Server:
    """Query server over a graph (evq_server_*): mode "batch" (continuous batching) or "plain" (one at a time)."""

    def __init__(self, graph, mode="batch", max_batch=0, max_inflight=0, max_groups=0, mem_budget=0, max_queued=0,
                 queue_hi=0):
        cfg = ServerConfig({"batch": 0, "plain": 1}[mode], max_batch, max_inflight, max_groups, mem_budget,
                           max_queued, queue_hi)
        h = ctypes.c_void_p()
        _check(_lib.evq_server_create(graph._h, ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self.graph = graph  # the handle must outlive the server

    def submit(self, algo, source, win_len) -> int:
        t = ctypes.c_uint64()
        _check(_lib.evq_server_submit(self._h, ALGOS.get(algo, algo), source, win_len, ctypes.byref(t)))
        return t.value

    def poll(self, cap=256, wait_ms=0) -> list:
        """Completed queries: dicts with ticket, status, times (ms), window and a Result (None on failure)."""
        arr = (Completion * cap)()
        n = _lib.evq_server_poll(self._h, arr, cap, wait_ms)
        out = []
        for i in range(n):
            c = arr[i]
            r = c.result
            out.append({"ticket": c.ticket, "status": c.status, "group_size": c.group_size,
                        "t_arrival_ms": c.t_arrival_ms, "t_admit_ms": c.t_admit_ms, "t_bounds_ms": c.t_bounds_ms,
                        "t_done_ms": c.t_done_ms, "n_unstable": c.n_unstable,
                        "iters_relax": c.iters_relax, "algo": r.algo, "source": r.source,
                        "win_begin": r.win_begin, "win_len": r.win_len,
                        "result": Result(r) if c.status == EVQ_OK and r.d_rcap else None})
        return out

    def pending(self):
        q, f = ctypes.c_uint32(), ctypes.c_uint32()
        _check(_lib.evq_server_pending(self._h, ctypes.byref(q), ctypes.byref(f)))
        return q.value, f.value

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.evq_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def batch_config() -> dict:
    c = BatchConfig()
    _check(_lib.evq_batch_config_get(ctypes.byref(c)))
    return {"lanes": c.lanes, "chunk": c.chunk, "blocks": c.blocks, "group": c.group}


def set_batch_config(lanes=0, chunk=0, blocks=0, group=0):
    """Execution choices of query_batch (0 keeps the current value)."""
    _check(_lib.evq_batch_config_set(ctypes.byref(BatchConfig(lanes, chunk, blocks, group))))


def get_tuning() -> dict:
    """Scheduling knobs of single queries, appends and frontier loops (evq_tuning_get)."""
    t = Tuning()
    _check(_lib.evq_tuning_get(ctypes.byref(t)))
    d = {k: getattr(t, k) for k, _ in Tuning._fields_ if k != "reserved"}
    d["delta"], d["heavy"] = list(t.delta), list(t.heavy)
    return d


def set_tuning(**kw):
    """Replace some scheduling knobs (evq_tuning_set); the others keep their values.
    delta / heavy may be one number (every algorithm) or five."""
    cur = get_tuning()
    for k, v in kw.items():
        if k not in cur:
            raise KeyError(k)
        if k in ("delta", "heavy") and not isinstance(v, (list, tuple)):
            v = [v] * 5
        cur[k] = v
    t = Tuning()
    for k, v in cur.items():
        if k in ("delta", "heavy"):
            getattr(t, k)[:] = [int(x) for x in v]
        else:
            setattr(t, k, v)
    _check(_lib.evq_tuning_set(ctypes.byref(t)))


class tuning:
    """Context manager: set scheduling knobs for the block, restore them after."""

    def __init__(self, **kw):
        self.kw = kw

    def __enter__(self):
        self.prev = get_tuning()
        set_tuning(**self.kw)
        return self

    def __exit__(self, *a):
        set_tuning(**self.prev)


def to_u32(t) -> np.ndarray:
    """Host uint32 view of an int32 device tensor."""
    return t.detach().cpu().numpy().view(np.uint32)


def to_f32(t) -> np.ndarray:
    """Host float32 view of Viterbi values (IEEE single bit patterns in an int32 device tensor)."""
    return t.detach().cpu().numpy().view(np.float32)


def timing_enable(on=True):
    _lib.evq_timing_enable(1 if on else 0)


def timing_reset():
    _lib.evq_timing_reset()


def timing_report() -> dict:
    n = _lib.evq_timing_report(None, 0)
    arr = (KernelTime * max(n, 1))()
    n = _lib.evq_timing_report(arr, n)
    return {arr[i].name.decode(): (arr[i].launches, arr[i].total_ms) for i in range(n)}


lib = _lib
