"""CPU oracle for the queue-driven Bellman-Ford path (test infrastructure).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The product path (the HIP library and
its Python binding) never does, and this package imports nothing from it: the
two share no code. Inputs come from ``synth`` only.

Parts and the passages they follow:

- ``bf_rounds``: round-based Bellman-Ford, Alg. 3 on one processing element
  (relax rule of PARALLEL_RELAX_EDGES, change counter, early exit of
  Section III.C, negative cycle when the round indexed n-1 still changes).
- ``bf_fifo``: sequential FIFO Bellman-Ford, the single-thread form of the
  queue-based solver of Section III.C.
- ``pred``: smallest-id tight in-neighbour (a fixed choice among equally
  valid shortest-path trees).
- ``fifo_run``: the sequential bounded FIFO, the specification the concurrent
  queue of Section III.A (Alg. 1) is linearizable to.
- ``history``: checks of concurrent queue histories against that
  specification (see ``oracle/history.py``).
- ``neg_inf``: minus-infinity marking (vertices a reachable negative cycle
  reaches), beyond the paper's detection.
- ``bf_jacobi``: the same rounds as Jacobi rounds on all host cores
  (``cpu_parallel.c``, OpenMP), a multi-core timing baseline only.
- ``ring_mixed`` / ``bq_mixed``: the queue's CPU baselines (``queue_cpu.c``):
  a sequential ring on one core, and Alg. 1's Broker Queue with C11 atomics
  on host threads (checked with the same history checks as the GPU queue).

All values are exact integers; INF = INT64_MAX marks unreached vertices.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

INF = np.iinfo(np.int64).max
_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIBDIR = os.path.join(_HERE, "_build")
_LIB = os.path.join(_LIBDIR, "liboracle.so")
_lock = threading.Lock()
_lib = None
_PSRC = [os.path.join(_HERE, "cpu_parallel.c"), os.path.join(_HERE, "queue_cpu.c")]
_PLIB = os.path.join(_LIBDIR, "libcpupar.so")
_plib = None


def build(force: bool = True, src: str = _SRC, out: str = _LIB) -> str:
    """Compile the C oracle with gcc into a shared library."""
    os.makedirs(os.path.dirname(out), exist_ok=True)
    if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(src):
        return out
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.run(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", tmp, src],
                   check=True)
    os.replace(tmp, out)
    return out


def build_parallel() -> str:
    """Compile the multi-core baseline (OpenMP) into its own library."""
    os.makedirs(_LIBDIR, exist_ok=True)
    tmp = _PLIB + ".tmp%d" % os.getpid()
    subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-pthread", "-shared", "-fPIC",
                    "-D_GNU_SOURCE", "-o", tmp] + _PSRC, check=True)
    os.replace(tmp, _PLIB)
    return _PLIB


def load_parallel():
    global _plib
    if _plib is not None:
        return _plib
    with _lock:
        if not os.path.exists(_PLIB):
            build_parallel()
        lib = ctypes.CDLL(_PLIB)
        i32, i64, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
        lib.cpu_transpose.restype = None
        lib.cpu_transpose.argtypes = [i32, vp, vp, vp, vp, vp, vp]
        lib.cpu_bf_jacobi.restype = i64
        lib.cpu_bf_jacobi.argtypes = [i32, vp, vp, vp, i32, vp, vp, vp]
        f64 = ctypes.c_double
        lib.cpu_ring_mixed.restype = f64
        lib.cpu_ring_mixed.argtypes = [i64, i64, vp]
        lib.cpu_bq_mixed.restype = f64
        lib.cpu_bq_mixed.argtypes = [i64, i64, i32, vp, vp, vp]
        _plib = lib
        return lib


def transpose(g):
    """CSC of g: (toff int64[n+1], tsrc int32[m], tw int32[m])."""
    lib = load_parallel()
    off, col, w = _csr(g)
    toff = np.empty(g.n + 1, dtype=np.int64)
    tsrc = np.empty(col.shape[0], dtype=np.int32)
    tw = np.empty(col.shape[0], dtype=np.int32)
    lib.cpu_transpose(g.n, _ptr(off), _ptr(col), _ptr(w), _ptr(toff), _ptr(tsrc), _ptr(tw))
    return toff, tsrc, tw


def bf_jacobi(g, csc, src: int | None = None):
    """Jacobi rounds on all OpenMP threads over the transposed graph.
    Returns (dist, neg, rounds, threads)."""
    lib = load_parallel()
    toff, tsrc, tw = csc
    s = g.src if src is None else int(src)
    d = np.empty(g.n, dtype=np.int64)
    neg = np.zeros(1, dtype=np.int32)
    thr = np.zeros(1, dtype=np.int32)
    r = lib.cpu_bf_jacobi(g.n, _ptr(toff), _ptr(tsrc), _ptr(tw), s, _ptr(d), _ptr(neg), _ptr(thr))
    return d, bool(neg[0]), int(r), int(thr[0])


def ring_mixed(capacity: int, n_ops: int):
    """Sequential ring, alternating enqueue / dequeue: returns seconds."""
    chk = np.zeros(1, dtype=np.int64)
    return float(load_parallel().cpu_ring_mixed(capacity, n_ops, _ptr(chk)))


def bq_mixed(capacity: int, n_ops: int, threads: int, log: bool = False):
    """Alg. 1's Broker Queue on host threads, Global Mixed: returns
    (seconds, Full/Empty retries, enq_log, deq_log) (logs None unless asked)."""
    el = dl = None
    if log:
        el = np.full(n_ops // 2, -1, dtype=np.int32)
        dl = np.full(n_ops // 2, -1, dtype=np.int32)
    fails = np.zeros(1, dtype=np.int64)
    t = load_parallel().cpu_bq_mixed(capacity, n_ops, threads,
                                     _ptr(el) if log else None, _ptr(dl) if log else None,
                                     _ptr(fails))
    return float(t), int(fails[0]), el, dl


def load(path: str | None = None):
    """Load the oracle library (building it first if it is not there)."""
    global _lib
    if path is None and _lib is not None:
        return _lib
    with _lock:
        p = path or _LIB
        if path is None and not os.path.exists(p):
            build(force=True)
        lib = ctypes.CDLL(p)
        i32, i64 = ctypes.c_int32, ctypes.c_int64
        vp = ctypes.c_void_p
        lib.oracle_bf_rounds.restype = i64
        lib.oracle_bf_rounds.argtypes = [i32, vp, vp, vp, i32, vp, vp]
        lib.oracle_bf_fifo.restype = i64
        lib.oracle_bf_fifo.argtypes = [i32, vp, vp, vp, i32, vp, vp, vp]
        lib.oracle_pred.restype = None
        lib.oracle_pred.argtypes = [i32, vp, vp, vp, i32, vp, vp]
        lib.oracle_neg_inf.restype = i64
        lib.oracle_neg_inf.argtypes = [i32, vp, vp, vp, i32, vp, vp]
        lib.oracle_fifo_run.restype = i64
        lib.oracle_fifo_run.argtypes = [i64, i64, vp, vp, vp]
        if path is None:
            _lib = lib
        return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _csr(g):
    off = np.ascontiguousarray(g.offsets, dtype=np.int64)
    col = np.ascontiguousarray(g.cols, dtype=np.int32)
    w = np.ascontiguousarray(g.w, dtype=np.int32)
    if off.shape[0] != g.n + 1 or off[0] != 0 or off[-1] != col.shape[0]:
        raise ValueError("malformed CSR")
    return off, col, w


def bf_rounds(g, src: int | None = None, lib=None):
    """Round-based BF (Alg. 3, one PE). Returns (dist int64[n], neg bool, rounds)."""
    lib = lib or load()
    off, col, w = _csr(g)
    s = g.src if src is None else int(src)
    d = np.empty(g.n, dtype=np.int64)
    neg = np.zeros(1, dtype=np.int32)
    rounds = lib.oracle_bf_rounds(g.n, _ptr(off), _ptr(col), _ptr(w), s, _ptr(d), _ptr(neg))
    return d, bool(neg[0]), int(rounds)


def bf_fifo(g, src: int | None = None, lib=None):
    """Sequential FIFO BF. Returns (dist, neg, pops, relaxations)."""
    lib = lib or load()
    off, col, w = _csr(g)
    s = g.src if src is None else int(src)
    d = np.empty(g.n, dtype=np.int64)
    neg = np.zeros(1, dtype=np.int32)
    relax = np.zeros(1, dtype=np.int64)
    pops = lib.oracle_bf_fifo(g.n, _ptr(off), _ptr(col), _ptr(w), s, _ptr(d), _ptr(neg),
                              _ptr(relax))
    return d, bool(neg[0]), int(pops), int(relax[0])


def pred(g, dist: np.ndarray, src: int | None = None, lib=None) -> np.ndarray:
    """Smallest-id tight in-neighbour of every reached vertex (-1 for src and
    unreached vertices)."""
    lib = lib or load()
    off, col, w = _csr(g)
    s = g.src if src is None else int(src)
    d = np.ascontiguousarray(dist, dtype=np.int64)
    p = np.empty(g.n, dtype=np.int32)
    lib.oracle_pred(g.n, _ptr(off), _ptr(col), _ptr(w), s, _ptr(d), _ptr(p))
    return p


NEG_INF = np.iinfo(np.int64).min


def neg_inf(g, src: int | None = None, lib=None):
    """Distances with minus infinity: (dist, pred, neg). dist[v] = NEG_INF
    for vertices reachable from a negative cycle that src reaches, INF for
    unreached vertices, the exact distance otherwise; pred = -1 for the
    minus-infinity vertices, the smallest tight in-neighbour otherwise; neg
    = some vertex is minus infinity."""
    lib = lib or load()
    off, col, w = _csr(g)
    s = g.src if src is None else int(src)
    d = np.empty(g.n, dtype=np.int64)
    mark = np.zeros(g.n, dtype=np.int8)
    k = lib.oracle_neg_inf(g.n, _ptr(off), _ptr(col), _ptr(w), s, _ptr(d), _ptr(mark))
    mk = mark.astype(bool)
    # predecessors of the finite vertices: no marked vertex is an in-neighbour
    # of an unmarked one, so the marked ones are left out as unreached
    d_fin = d.copy()
    d_fin[mk] = INF
    p = pred(g, d_fin, s, lib)
    p[mk] = -1
    d[mk] = NEG_INF
    return d, p, bool(k > 0)


def sssp(g, src: int | None = None, method: str = "rounds", lib=None):
    """Distances, predecessors and the negative-cycle flag for (g, src).

    ``method`` = "rounds" (the authority, Alg. 3) or "fifo" (sequential
    queue form, much faster on large graphs). On a negative cycle the
    distances and predecessors are not meaningful and are returned as given.
    """
    if method == "rounds":
        d, neg, _ = bf_rounds(g, src, lib)
    elif method == "fifo":
        d, neg, _, _ = bf_fifo(g, src, lib)
    else:
        raise ValueError(method)
    p = pred(g, d, src, lib) if not neg else np.full(g.n, -1, dtype=np.int32)
    return d, p, neg


def fifo_run(capacity: int, ops, lib=None):
    """Run a sequence of operations on the sequential bounded FIFO.

    ``ops[i] >= 0`` enqueues that value, ``ops[i] < 0`` dequeues once.
    Returns (ok int8[k], out int64[k] (dequeued value or -1), final size).
    """
    lib = lib or load()
    o = np.ascontiguousarray(ops, dtype=np.int64)
    res = np.zeros(o.shape[0], dtype=np.int8)
    out = np.zeros(o.shape[0], dtype=np.int64)
    size = lib.oracle_fifo_run(int(capacity), o.shape[0], _ptr(o), _ptr(res), _ptr(out))
    return res, out, int(size)
