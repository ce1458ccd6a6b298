"""Python binding of libbqsssp.so (the C ABI declared in include/bq.h).

Argument marshalling only: every step of the queue and of the solver runs in
the library's HIP kernels. PyTorch supplies device memory and streams. If the
shared library is missing the import of a function fails loudly; there is no
CPU fallback.

Entry points mirror the C names: ``sssp_bf``, ``Queue`` (bq_create,
bq_enqueue, bq_dequeue, bq_reset, bq_bench_mixed, bq_bench_enqdeq, bq_counters), ``SsspContext``
(sssp_ctx_create, sssp_bf, sssp_autotune, sssp_last_stats), ``SsspBatch``
(the batched form), ``Server`` and ``Arena`` (the served form),
``RoundsContext`` (sssp_bf_rounds, the round form over an edge queue).
"""
from __future__ import annotations

import ctypes
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbqsssp.so")

BQ_OK, BQ_EINVAL, BQ_ENOMEM, BQ_EHIP, BQ_ERANGE, BQ_ETIMEOUT, BQ_EBUSY = 0, -1, -2, -3, -4, -5, -6
BQ_EOVERFLOW = -7
BQ_F_VALIDATE = 1
BQ_F_TRACE = 2
BQ_F_GRAPH = 4
BQ_F_BWD = 8
BQ_F_NEGINF = 16
BQ_F_NOREMAP = 32

# every symbol include/bq.h declares
EXPORTS = [
    "bq_create", "bq_destroy", "bq_reset", "bq_enqueue", "bq_dequeue", "bq_counters",
    "bq_bench_mixed", "bq_bench_enqdeq", "sssp_ctx_create", "sssp_ctx_destroy", "sssp_bf", "sssp_last_stats",
    "sssp_last_trace", "sssp_autotune", "sssp_batch_create", "sssp_batch_destroy",
    "sssp_bf_batched", "sssp_batch_last_stats", "sssp_batch_autotune",
    "sssp_bf_batched_start", "sssp_batch_finish", "bq_server_create", "bq_server_destroy",
    "bq_server_set_small_lanes", "bq_server_set_graph_launch", "bq_server_add_graph", "bq_server_run", "bq_arena_create", "bq_arena_destroy",
    "bq_arena_alloc", "bq_arena_free", "bq_arena_usage",
    "bq_strerror", "bq_device_cus", "bq_probe",
    "sssp_rounds_create", "sssp_rounds_destroy", "sssp_bf_rounds", "sssp_rounds_last_stats",
    "sssp_bf_noalloc",
]


class BQError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {strerror(status)} ({status})")


class Launch(ctypes.Structure):
    _fields_ = [("wg_size", ctypes.c_int32), ("wg_count", ctypes.c_int32),
                ("ticket_batch", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("timeout_us", ctypes.c_uint64), ("row_chunk", ctypes.c_int32),
                ("queue_scale", ctypes.c_int32), ("segments", ctypes.c_int32),
                ("bucket_width", ctypes.c_int32)]


class BenchStats(ctypes.Structure):
    _fields_ = [("enq_ok", ctypes.c_uint64), ("deq_ok", ctypes.c_uint64),
                ("enq_full", ctypes.c_uint64), ("deq_empty", ctypes.c_uint64),
                ("ms", ctypes.c_double)]


class SsspStats(ctypes.Structure):
    _fields_ = [("dequeued", ctypes.c_uint64), ("relaxations", ctypes.c_uint64),
                ("pushes", ctypes.c_uint64), ("fanout", ctypes.c_uint64),
                ("batches", ctypes.c_uint64), ("walks", ctypes.c_uint64),
                ("improvements", ctypes.c_uint64), ("idle_polls", ctypes.c_uint64),
                ("ticket_spins", ctypes.c_uint64), ("ms", ctypes.c_double),
                ("solve_ms", ctypes.c_double), ("grid", ctypes.c_int32),
                ("wg_size", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class RoundsStats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_uint64), ("changes", ctypes.c_uint64),
                ("relaxations", ctypes.c_uint64), ("ticket_spins", ctypes.c_uint64),
                ("ms", ctypes.c_double), ("solve_ms", ctypes.c_double),
                ("grid", ctypes.c_int32), ("wg_size", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Instance(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("src", ctypes.c_int32), ("m", ctypes.c_int64),
                ("offsets", ctypes.c_void_p), ("cols", ctypes.c_void_p), ("w", ctypes.c_void_p),
                ("dist", ctypes.c_void_p), ("pred", ctypes.c_void_p)]


class Request(ctypes.Structure):
    _fields_ = [("arrival_us", ctypes.c_double), ("graph", ctypes.c_int32),
                ("src", ctypes.c_int32), ("n", ctypes.c_int32), ("m", ctypes.c_int64),
                ("h_offsets", ctypes.c_void_p), ("h_cols", ctypes.c_void_p),
                ("h_w", ctypes.c_void_p), ("d_dist", ctypes.c_void_p),
                ("d_pred", ctypes.c_void_p)]


class Response(ctypes.Structure):
    _fields_ = [("latency_us", ctypes.c_double), ("wait_us", ctypes.c_double),
                ("service_us", ctypes.c_double), ("reached_edges", ctypes.c_int64),
                ("neg_cycle", ctypes.c_int32), ("status", ctypes.c_int32),
                ("lane", ctypes.c_int32), ("reserved_", ctypes.c_int32)]


class ServerStats(ctypes.Structure):
    _fields_ = [("wall_ms", ctypes.c_double), ("launches", ctypes.c_uint64),
                ("max_inflight", ctypes.c_uint64), ("max_lanes_busy", ctypes.c_uint64),
                ("arena_peak_bytes", ctypes.c_uint64), ("upload_bytes", ctypes.c_uint64)]


_lib = None


def lib(path: str | None = None):
    """Load libbqsssp.so (raises if it was not built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(f"{p} not found: build it with __graft_entry__.build() "
                          "(python -m paper_2608_21826_amd._build)")
    L = ctypes.CDLL(p)
    vp, i32, i64, u32, u64 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                              ctypes.c_uint64)
    P = ctypes.POINTER
    sig = {
        "bq_create": ([u32, u32, vp, P(vp)], i32),
        "bq_destroy": ([vp], i32),
        "bq_reset": ([vp, vp], i32),
        "bq_enqueue": ([vp, vp, u64, vp, P(Launch), vp], i32),
        "bq_dequeue": ([vp, vp, u64, vp, P(Launch), vp], i32),
        "bq_counters": ([vp, vp, P(u64), P(u64), P(i64)], i32),
        "bq_bench_mixed": ([vp, u64, P(Launch), vp, vp, P(BenchStats), P(i32), vp], i32),
        "bq_bench_enqdeq": ([vp, u64, P(Launch), P(BenchStats), P(BenchStats), vp], i32),
        "sssp_ctx_create": ([i32, i64, P(vp)], i32),
        "sssp_ctx_destroy": ([vp], i32),
        "sssp_bf": ([vp, i32, i64, vp, vp, vp, i32, vp, vp, P(i32), P(Launch), vp], i32),
        "sssp_last_stats": ([vp, P(SsspStats)], i32),
        "sssp_bf_noalloc": ([i32, i64, vp, vp, vp, i32, vp, vp, P(i32), P(Launch), vp], i32),
        "sssp_last_trace": ([vp, P(u64), i32], i32),
        "sssp_autotune": ([vp, i32, i64, vp, vp, vp, i32, vp, P(Launch), i32, P(Launch),
                           P(ctypes.c_double), vp], i32),
        "bq_strerror": ([i32], ctypes.c_char_p),
        "bq_device_cus": ([], i32),
        "bq_probe": ([i32, vp, vp, u64, u64, i32, i32, P(ctypes.c_double), vp], i32),
        "sssp_batch_create": ([i32, i64, i64, P(vp)], i32),
        "sssp_batch_destroy": ([vp], i32),
        "sssp_bf_batched": ([vp, i32, P(Instance), P(i32), P(Launch), vp], i32),
        "sssp_batch_last_stats": ([vp, P(SsspStats)], i32),
        "sssp_batch_autotune": ([vp, i32, P(Instance), P(Launch), i32, P(Launch),
                                 P(ctypes.c_double), vp], i32),
        "sssp_bf_batched_start": ([vp, i32, P(Instance), P(Launch), vp], i32),
        "sssp_batch_finish": ([vp, P(i32), P(i64), i32], i32),
        "bq_server_create": ([i32, i32, i64, i64, i64, P(Launch), P(vp)], i32),
        "bq_server_destroy": ([vp], i32),
        "bq_server_set_small_lanes": ([vp, i32], i32),
        "bq_server_add_graph": ([vp, i32, i64, vp, vp, vp, P(i32)], i32),
        "bq_server_set_graph_launch": ([vp, i32, P(Launch)], i32),
        "bq_server_run": ([vp, i32, P(Request), P(Response), P(ServerStats)], i32),
        "bq_arena_create": ([u64, u64, P(vp)], i32),
        "bq_arena_destroy": ([vp], i32),
        "bq_arena_alloc": ([vp, u64, P(u64)], i32),
        "bq_arena_free": ([vp, u64], i32),
        "bq_arena_usage": ([vp, P(u64), P(u64), P(u64)], i32),
        "sssp_rounds_create": ([i32, i64, P(vp)], i32),
        "sssp_rounds_destroy": ([vp], i32),
        "sssp_bf_rounds": ([vp, i32, i64, vp, vp, vp, i32, vp, vp, P(i32), P(Launch), vp], i32),
        "sssp_rounds_last_stats": ([vp, P(RoundsStats)], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    if path is None:
        _lib = L
    return L


def strerror(status: int) -> str:
    try:
        return lib().bq_strerror(int(status)).decode()
    except ImportError:
        return f"status {status}"


def _check(status: int, what: str):
    if status != BQ_OK:
        raise BQError(status, what)


def _release(self):
    """__del__ of the handle classes: close, except while the interpreter
    shuts down. Then the process is ending, the device frees everything, and
    HIP calls from module teardown could run after the runtime (or a
    profiler attached to it) has finished. Call close() to free earlier."""
    if not sys.is_finalizing():
        self.close()


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _launch(launch):
    if launch is None:
        return None
    if isinstance(launch, Launch):
        return ctypes.byref(launch)
    return ctypes.byref(Launch(**launch))


def _need(t, dtype, name, n=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (ROCm) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} must have {n} elements, got {t.numel()}")


# ---------------------------------------------------------------------------
# queue
# ---------------------------------------------------------------------------
class Queue:
    """A Broker Queue of `capacity` int32 slots on the current device."""

    def __init__(self, capacity: int, stream=None):
        h = ctypes.c_void_p()
        _check(lib().bq_create(capacity, 0, _stream(stream), ctypes.byref(h)), "bq_create")
        self.handle = h
        self.capacity = capacity

    def close(self):
        if self.handle:
            lib().bq_destroy(self.handle)
            self.handle = None

    __del__ = _release

    def reset(self, stream=None):
        _check(lib().bq_reset(self.handle, _stream(stream)), "bq_reset")

    def enqueue(self, vals, launch=None, stream=None) -> int:
        import torch
        _need(vals, torch.int32, "vals")
        ok = torch.zeros(1, dtype=torch.int64, device=vals.device)
        _check(lib().bq_enqueue(self.handle, _ptr(vals), vals.numel(), _ptr(ok), _launch(launch),
                                _stream(stream)), "bq_enqueue")
        return int(ok.item())

    def dequeue(self, n: int, launch=None, stream=None, device="cuda"):
        import torch
        out = torch.empty(max(n, 1), dtype=torch.int32, device=device)
        ok = torch.zeros(1, dtype=torch.int64, device=device)
        _check(lib().bq_dequeue(self.handle, _ptr(out), n, _ptr(ok), _launch(launch),
                                _stream(stream)), "bq_dequeue")
        k = int(ok.item())
        return out[:k]

    def bench_enqdeq(self, n_ops: int, launch=None, stream=None):
        """Section IV "Global Enqueue-Dequeue": returns (enqueue stats, dequeue stats)."""
        e, d = BenchStats(), BenchStats()
        _check(lib().bq_bench_enqdeq(self.handle, n_ops, _launch(launch), ctypes.byref(e),
                                     ctypes.byref(d), _stream(stream)), "bq_bench_enqdeq")
        return ({k: getattr(e, k) for k, _ in e._fields_},
                {k: getattr(d, k) for k, _ in d._fields_})

    def counters(self, stream=None):
        h, t, c = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_int64()
        _check(lib().bq_counters(self.handle, _stream(stream), ctypes.byref(h), ctypes.byref(t),
                                 ctypes.byref(c)), "bq_counters")
        return h.value, t.value, c.value

    def bench_mixed(self, n_ops: int, launch=None, log: bool = False, stream=None,
                    device="cuda"):
        """Section IV "Global Mixed" run; returns (stats dict, enq_log, deq_log)."""
        import torch
        el = dl = None
        if log:
            el = torch.full((n_ops // 2,), -1, dtype=torch.int32, device=device)
            dl = torch.full((n_ops // 2,), -1, dtype=torch.int32, device=device)
        st = BenchStats()
        w = ctypes.c_int32()
        _check(lib().bq_bench_mixed(self.handle, n_ops, _launch(launch), _ptr(el), _ptr(dl),
                                    ctypes.byref(st), ctypes.byref(w), _stream(stream)),
               "bq_bench_mixed")
        d = {k: getattr(st, k) for k, _ in st._fields_}
        d["enq_waves"] = w.value
        return d, el, dl


# ---------------------------------------------------------------------------
# SSSP
# ---------------------------------------------------------------------------
def _solve_args(offsets, cols, w, dist, pred, want_pred, launch, flags):
    import torch
    n = offsets.numel() - 1
    m = cols.numel()
    _need(offsets, torch.int64, "offsets", n + 1)
    _need(cols, torch.int32, "cols")
    _need(w, torch.int32, "w", m)
    dev = offsets.device
    if dist is None:
        dist = torch.empty(n, dtype=torch.int64, device=dev)
    _need(dist, torch.int64, "dist", n)
    if want_pred and pred is None:
        pred = torch.empty(n, dtype=torch.int32, device=dev)
    if pred is not None:
        _need(pred, torch.int32, "pred", n)
    L = launch
    if flags:
        L = Launch(**(launch or {})) if not isinstance(launch, Launch) else launch
        L.flags |= flags
    return n, m, dist, pred, L


class SsspContext:
    """Workspace for graphs up to max_n vertices and max_m edges."""

    def __init__(self, max_n: int, max_m: int):
        h = ctypes.c_void_p()
        _check(lib().sssp_ctx_create(int(max_n), int(max_m), ctypes.byref(h)), "sssp_ctx_create")
        self.handle = h
        self.max_n, self.max_m = int(max_n), int(max_m)

    def close(self):
        if self.handle:
            lib().sssp_ctx_destroy(self.handle)
            self.handle = None

    __del__ = _release

    def solve(self, offsets, cols, w, src: int, dist=None, pred=None, want_pred=True,
              launch=None, validate=False, trace=False, neg_inf=False, stream=None):
        """sssp_bf on device tensors; returns (dist int64, pred int32 or None, neg bool).
        With neg_inf, a negative cycle leaves dist = INT64_MIN on the vertices
        it reaches and exact results elsewhere."""
        n, m, dist, pred, L = _solve_args(offsets, cols, w, dist, pred, want_pred, launch,
                                          (BQ_F_VALIDATE if validate else 0) |
                                          (BQ_F_TRACE if trace else 0) |
                                          (BQ_F_NEGINF if neg_inf else 0))
        neg = ctypes.c_int32(0)
        _check(lib().sssp_bf(self.handle, n, m, _ptr(offsets), _ptr(cols), _ptr(w), int(src),
                             _ptr(dist), _ptr(pred), ctypes.byref(neg), _launch(L),
                             _stream(stream)), "sssp_bf")
        return dist, pred, bool(neg.value)

    def autotune(self, offsets, cols, w, src: int, reps: int = 5, base=None, stream=None):
        """sssp_autotune: returns (launch dict, best ms)."""
        import torch
        n = offsets.numel() - 1
        m = cols.numel()
        scratch = torch.empty(n, dtype=torch.int64, device=offsets.device)
        best = Launch()
        ms = ctypes.c_double()
        _check(lib().sssp_autotune(self.handle, n, m, _ptr(offsets), _ptr(cols), _ptr(w), int(src),
                                   _ptr(scratch), _launch(base), int(reps), ctypes.byref(best),
                                   ctypes.byref(ms), _stream(stream)), "sssp_autotune")
        return {k: getattr(best, k) for k, _ in best._fields_}, ms.value

    def trace(self):
        """Timeline of the last solve run with flag BQ_F_TRACE: rows of
        (ticks since start, dequeued so far, queue length, pending)."""
        import numpy as np
        buf = (ctypes.c_uint64 * (4 * 4096))()
        k = lib().sssp_last_trace(self.handle, buf, 4096)
        a = np.frombuffer(buf, dtype=np.uint64).reshape(-1, 4)[:max(k, 0)]
        return a[a[:, 0] != np.iinfo(np.uint64).max]

    def stats(self) -> dict:
        s = SsspStats()
        _check(lib().sssp_last_stats(self.handle, ctypes.byref(s)), "sssp_last_stats")
        return s.as_dict()


def sssp_bf_noalloc(offsets, cols, w, src: int, dist, pred=None, launch=None,
                    validate=False, neg_inf=False, stream=None):
    """sssp_bf_noalloc on device tensors: the solver with its workspace in
    the library's fixed device array (no allocation by the library; the
    caller passes dist and optionally pred). Returns neg (bool)."""
    n, m, dist, pred, L = _solve_args(offsets, cols, w, dist, pred, False, launch,
                                      (BQ_F_VALIDATE if validate else 0) |
                                      (BQ_F_NEGINF if neg_inf else 0))
    neg = ctypes.c_int32(0)
    _check(lib().sssp_bf_noalloc(n, m, _ptr(offsets), _ptr(cols), _ptr(w), int(src), _ptr(dist),
                                 _ptr(pred), ctypes.byref(neg), _launch(L), _stream(stream)),
           "sssp_bf_noalloc")
    return bool(neg.value)


def sssp_bf(offsets, cols, w, src: int, want_pred=True, launch=None, validate=True, ctx=None):
    """One SSSP query on device tensors (allocates a context if none given)."""
    own = ctx is None
    if own:
        ctx = SsspContext(offsets.numel() - 1, cols.numel())
    try:
        return ctx.solve(offsets, cols, w, src, want_pred=want_pred, launch=launch,
                         validate=validate)
    finally:
        if own:
            ctx.close()


class SsspBatch:
    """sssp_bf_batched workspace: up to max_instances queries with at most
    max_total_n vertices and max_total_m edges in total."""

    def __init__(self, max_instances: int, max_total_n: int, max_total_m: int):
        h = ctypes.c_void_p()
        _check(lib().sssp_batch_create(int(max_instances), int(max_total_n), int(max_total_m),
                                       ctypes.byref(h)), "sssp_batch_create")
        self.handle = h

    def close(self):
        if self.handle:
            lib().sssp_batch_destroy(self.handle)
            self.handle = None

    __del__ = _release

    @staticmethod
    def _table(queries):
        """queries: list of (offsets, cols, w, src, dist, pred-or-None)."""
        import torch
        arr = (Instance * len(queries))()
        for i, (off, col, w, src, dist, pred) in enumerate(queries):
            n = off.numel() - 1
            _need(off, torch.int64, "offsets", n + 1)
            _need(col, torch.int32, "cols")
            _need(w, torch.int32, "w", col.numel())
            _need(dist, torch.int64, "dist", n)
            if pred is not None:
                _need(pred, torch.int32, "pred", n)
            arr[i] = Instance(n, int(src), col.numel(), off.data_ptr(), col.data_ptr(),
                              w.data_ptr(), dist.data_ptr(), pred.data_ptr() if pred is not None else 0)
        return arr

    def solve(self, queries, launch=None, graph=False, stream=None):
        """Solve all queries; fills their dist/pred tensors, returns the list of
        negative-cycle flags."""
        arr = self._table(queries)
        neg = (ctypes.c_int32 * len(queries))()
        L = Launch(**(launch or {})) if not isinstance(launch, Launch) else launch
        if graph:
            L.flags |= BQ_F_GRAPH
        _check(lib().sssp_bf_batched(self.handle, len(queries), arr, neg, ctypes.byref(L),
                                     _stream(stream)), "sssp_bf_batched")
        return [bool(x) for x in neg]

    def autotune(self, queries, reps: int = 2, base=None, stream=None):
        arr = self._table(queries)
        best = Launch()
        ms = ctypes.c_double()
        _check(lib().sssp_batch_autotune(self.handle, len(queries), arr, _launch(base), int(reps),
                                         ctypes.byref(best), ctypes.byref(ms), _stream(stream)),
               "sssp_batch_autotune")
        return {k: getattr(best, k) for k, _ in best._fields_}, ms.value

    def stats(self) -> dict:
        s = SsspStats()
        _check(lib().sssp_batch_last_stats(self.handle, ctypes.byref(s)), "sssp_batch_last_stats")
        return s.as_dict()


class Server:
    """bq_server: resident graphs, admission by arena memory, continuous
    batching over `lanes` streams; the last `small_lanes` of them take only
    small requests."""

    def __init__(self, lanes: int, max_batch: int, max_batch_n: int, max_batch_m: int,
                 arena_bytes: int, launch=None, small_lanes: int = 0):
        h = ctypes.c_void_p()
        _check(lib().bq_server_create(int(lanes), int(max_batch), int(max_batch_n),
                                      int(max_batch_m), int(arena_bytes), _launch(launch),
                                      ctypes.byref(h)), "bq_server_create")
        self.handle = h
        self._graphs = []
        if small_lanes:
            _check(lib().bq_server_set_small_lanes(h, int(small_lanes)),
                   "bq_server_set_small_lanes")

    def close(self):
        if self.handle:
            lib().bq_server_destroy(self.handle)
            self.handle = None

    __del__ = _release

    def add_graph(self, offsets, cols, w) -> int:
        import torch
        n = offsets.numel() - 1
        _need(offsets, torch.int64, "offsets", n + 1)
        _need(cols, torch.int32, "cols")
        _need(w, torch.int32, "w", cols.numel())
        gid = ctypes.c_int32()
        _check(lib().bq_server_add_graph(self.handle, n, cols.numel(), _ptr(offsets), _ptr(cols),
                                         _ptr(w), ctypes.byref(gid)), "bq_server_add_graph")
        self._graphs.append((offsets, cols, w))
        return gid.value

    def set_graph_launch(self, graph_id: int, launch=None):
        """bq_server_set_graph_launch: large requests on this resident graph
        run with `launch` (a dict or Launch); None restores the default."""
        _check(lib().bq_server_set_graph_launch(self.handle, int(graph_id), _launch(launch)),
               "bq_server_set_graph_launch")

    def run(self, requests):
        """requests: list of dicts with arrival_us, src, and either graph=<id>
        or upload=(offsets, cols, w) host tensors/arrays (pinned keeps the copy
        asynchronous); optional dist / pred device tensors. Returns (list of
        response dicts, stats dict)."""
        import numpy as np
        arr = (Request * len(requests))()
        keep = []
        for i, r in enumerate(requests):
            q = Request()
            q.arrival_us = float(r["arrival_us"])
            q.src = int(r["src"])
            if r.get("upload") is not None:
                off, col, w = r["upload"]
                keep.append((off, col, w))
                q.graph = -1
                q.n = len(off) - 1
                q.m = len(col)
                q.h_offsets = _host_ptr(off)
                q.h_cols = _host_ptr(col)
                q.h_w = _host_ptr(w)
            else:
                q.graph = int(r["graph"])
            if r.get("dist") is not None:
                q.d_dist = r["dist"].data_ptr()
            if r.get("pred") is not None:
                q.d_pred = r["pred"].data_ptr()
            arr[i] = q
        resp = (Response * len(requests))()
        st = ServerStats()
        _check(lib().bq_server_run(self.handle, len(requests), arr, resp, ctypes.byref(st)),
               "bq_server_run")
        out = [{k: getattr(x, k) for k, _ in x._fields_} for x in resp]
        return out, {k: getattr(st, k) for k, _ in st._fields_}


def _host_ptr(a):
    try:
        return a.data_ptr()
    except AttributeError:
        return a.ctypes.data


class Arena:
    """The engine's host-side first-fit allocator (no device memory)."""

    def __init__(self, size: int, align: int = 256):
        h = ctypes.c_void_p()
        _check(lib().bq_arena_create(int(size), int(align), ctypes.byref(h)), "bq_arena_create")
        self.handle = h

    def close(self):
        if self.handle:
            lib().bq_arena_destroy(self.handle)
            self.handle = None

    __del__ = _release

    def alloc(self, nbytes: int):
        off = ctypes.c_uint64()
        st = lib().bq_arena_alloc(self.handle, int(nbytes), ctypes.byref(off))
        if st == BQ_EBUSY:
            return None
        _check(st, "bq_arena_alloc")
        return off.value

    def free(self, offset: int):
        _check(lib().bq_arena_free(self.handle, int(offset)), "bq_arena_free")

    def usage(self):
        u, p, lf = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().bq_arena_usage(self.handle, ctypes.byref(u), ctypes.byref(p),
                                    ctypes.byref(lf)), "bq_arena_usage")
        return u.value, p.value, lf.value


def device_cus() -> int:
    return int(lib().bq_device_cus())


def probe(kind: int, a, b=None, size: int = 0, ops_per_lane: int = 0, grid: int = 1024,
          block: int = 256, stream=None) -> float:
    """Run one roofline probe kernel (see bq_probe in include/bq.h); returns ms."""
    ms = ctypes.c_double()
    _check(lib().bq_probe(int(kind), _ptr(a), _ptr(b), int(size), int(ops_per_lane), int(grid),
                          int(block), ctypes.byref(ms), _stream(stream)), "bq_probe")
    return ms.value


# ---------------------------------------------------------------------------
# round-based Bellman-Ford over an edge queue
# ---------------------------------------------------------------------------
class RoundsContext:
    """sssp_rounds_create / sssp_bf_rounds: the paper's round form with the
    queue holding edges. Workspace for up to max_n vertices, max_m edges."""

    def __init__(self, max_n: int, max_m: int):
        h = ctypes.c_void_p()
        _check(lib().sssp_rounds_create(int(max_n), int(max_m), ctypes.byref(h)),
               "sssp_rounds_create")
        self.handle = h
        self.max_n, self.max_m = int(max_n), int(max_m)

    def close(self):
        if self.handle:
            lib().sssp_rounds_destroy(self.handle)
            self.handle = None

    __del__ = _release

    def solve(self, offsets, cols, w, src: int, dist=None, pred=None, want_pred=True,
              launch=None, validate=False, neg_inf=False, stream=None):
        """sssp_bf_rounds on device tensors; returns (dist, pred or None, neg).
        With neg_inf, a negative cycle leaves dist = INT64_MIN on the vertices
        it reaches and exact results elsewhere."""
        n, m, dist, pred, L = _solve_args(offsets, cols, w, dist, pred, want_pred, launch,
                                          (BQ_F_VALIDATE if validate else 0) |
                                          (BQ_F_NEGINF if neg_inf else 0))
        neg = ctypes.c_int32(0)
        _check(lib().sssp_bf_rounds(self.handle, n, m, _ptr(offsets), _ptr(cols), _ptr(w),
                                    int(src), _ptr(dist), _ptr(pred), ctypes.byref(neg),
                                    _launch(L), _stream(stream)), "sssp_bf_rounds")
        return dist, pred, bool(neg.value)

    def stats(self) -> dict:
        s = RoundsStats()
        _check(lib().sssp_rounds_last_stats(self.handle, ctypes.byref(s)),
               "sssp_rounds_last_stats")
        return s.as_dict()
