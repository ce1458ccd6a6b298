"""Write the stored expected results for the full-size configurations.

The values come from the CPU oracle only (sequential FIFO Bellman-Ford and
the smallest-id tight predecessor) on graphs from the seeded generators.
Before anything is written, every result is certified by an algorithm that
shares nothing with the oracle:

- potential-shifted graphs (RMAT-20, road2048, the 256 Erdos-Renyi
  instances of the batched workload, their sources): the Johnson
  closed form. With w = w0 + p(u) - p(v) and w0 >= 1, every path P from s
  to v weighs w0(P) + p(s) - p(v), so d(v) = d0(v) + p(s) - p(v) where d0
  comes from a library Dijkstra (scipy) on the non-negative w0;
- the 64x64 grid (weights 1..100): a library Dijkstra on w itself;
- the road mesh with the planted cycle: the three planted edges weigh -3 in
  total, and a breadth-first search from the source reaches them, so a
  negative cycle is reachable (the flag must be 1).

The files hold SHA-256 digests of the inputs and outputs plus a sample of
values, so GPU tests and the benchmark can check bit-exactness at full size
without the CPU solve.

Run from the repository root:  python tests/golden/make_golden.py
"""
import hashlib
import json
import os
import sys
import time

import numpy as np
import scipy.sparse as sp
import scipy.sparse.csgraph as csg

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

INF = oracle.INF
BATCH_SOURCES_SEED = synth.SEED_BASE + 3  # the 64 sources of the batched RMAT-20 workload


def sha(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def graph_digest(g) -> str:
    h = hashlib.sha256()
    for a in (g.offsets, g.cols, g.w):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def _matrix(g, weights):
    """scipy CSR with the minimum weight over parallel edges (csgraph keeps
    only one entry per pair). Self-loops never shorten a path and are
    dropped."""
    s, d, _ = synth.edges_of(g)
    keep = s != d
    s, d, wt = s[keep], d[keep], np.asarray(weights, dtype=np.float64)[keep]
    order = np.lexsort((wt, d, s))
    s, d, wt = s[order], d[order], wt[order]
    first = np.ones(s.size, dtype=bool)
    first[1:] = (s[1:] != s[:-1]) | (d[1:] != d[:-1])
    return sp.csr_matrix((wt[first], (s[first], d[first])), shape=(g.n, g.n))


def _from_float(x):
    out = np.full(x.shape, INF, dtype=np.int64)
    fin = np.isfinite(x)
    out[fin] = np.rint(x[fin]).astype(np.int64)
    return out


def johnson(g, sources):
    """Closed-form distances for potential-shifted weights, one row per source."""
    s, d, w = synth.edges_of(g)
    p = g.meta["potential"].astype(np.int64)
    w0 = w - p[s] + p[d]
    assert w0.min() >= 1, "not a potential-shifted graph with w0 >= 1"
    d0 = csg.dijkstra(_matrix(g, w0), directed=True, indices=np.asarray(sources))
    rows = []
    for i, src in enumerate(sources):
        r = _from_float(d0[i])
        fin = r != INF
        r[fin] = r[fin] + p[src] - p[np.nonzero(fin)[0]]
        rows.append(r)
    return rows


def dijkstra(g, src):
    s, d, w = synth.edges_of(g)
    assert w.min() >= 0
    return _from_float(csg.dijkstra(_matrix(g, w), directed=True, indices=src))


def planted_cycle_reachable(g) -> bool:
    a, b, c = g.meta["cycle"]
    s, d, w = synth.edges_of(g)
    total = 0
    for x, y in ((a, b), (b, c), (c, a)):
        sel = (s == x) & (d == y)
        assert sel.any()
        total += int(w[sel].min())
    A = sp.csr_matrix((np.ones(g.m), (s, d)), shape=(g.n, g.n))
    reach = csg.breadth_first_order(A, g.src, directed=True, return_predecessors=False)
    return total < 0 and a in set(reach.tolist())


def smallest_tight_in_neighbour(g, d, src):
    """pred by its definition, vectorized over the edge list: the smallest u
    with d[u] + w(u, v) = d[v], -1 for src and unreached vertices."""
    s, t, w = synth.edges_of(g)
    fin = d[s] != INF
    tight = np.zeros(s.size, dtype=bool)
    tight[fin] = d[s[fin]] + w[fin] == d[t[fin]]
    best = np.full(g.n, np.iinfo(np.int64).max, dtype=np.int64)
    np.minimum.at(best, t[tight], s[tight])
    out = np.where(best == np.iinfo(np.int64).max, -1, best).astype(np.int32)
    out[src] = -1
    out[d == INF] = -1
    return out


def solve_record(g, src, expected, samples=256, seed=12345):
    """Oracle result for (g, src), asserted equal to `expected` (distances)
    and to the predecessor definition applied to those distances."""
    t0 = time.time()
    d, neg, pops, relax = oracle.bf_fifo(g, src)
    assert not neg, f"{g.name} src={src}: oracle reports a negative cycle"
    assert np.array_equal(d, expected), f"{g.name} src={src}: oracle differs from certificate"
    p = oracle.pred(g, d, src)
    assert np.array_equal(p, smallest_tight_in_neighbour(g, expected, src)), \
        f"{g.name} src={src}: oracle pred differs from its definition"
    reached = d != INF
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(g.n, size=min(samples, g.n), replace=False))
    rec = {"src": int(src), "dist_sha256": sha(d), "pred_sha256": sha(p),
           "reached": int(np.count_nonzero(reached)),
           "m_reached": int(np.diff(g.offsets)[reached].sum()),
           "oracle": "bf_fifo", "pops": int(pops), "relaxations": int(relax),
           "sample_idx": idx.tolist(), "sample_dist": d[idx].tolist(),
           "sample_pred": p[idx].tolist()}
    print(f"  {g.name} src={src}: reached {rec['reached']}, {time.time() - t0:.1f}s",
          flush=True)
    return rec


def road_golden():
    out = {}
    g = synth.config_graph("road2048")
    exp = johnson(g, [g.src])[0]
    rec = solve_record(g, g.src, exp, samples=2000)
    rec.update({"n": g.n, "m": g.m, "graph_sha256": graph_digest(g), "neg_cycle": False,
                "certified_by": "johnson_closed_form"})
    out["road2048"] = rec
    g = synth.config_graph("road2048_negcycle")
    assert planted_cycle_reachable(g)
    d, neg, pops, relax = oracle.bf_fifo(g)
    assert neg, "oracle misses the planted cycle"
    out["road2048_negcycle"] = {"n": g.n, "m": g.m, "src": g.src,
                                "graph_sha256": graph_digest(g), "neg_cycle": True,
                                "oracle": "bf_fifo", "pops": int(pops),
                                "relaxations": int(relax),
                                "certified_by": "planted_cycle_weight_and_bfs"}
    return out


def rmat_golden():
    g = synth.config_graph("rmat20")
    srcs = [int(x) for x in synth.random_sources(g, 64, seed=BATCH_SOURCES_SEED)]
    allsrc = [g.src] + srcs
    print(f"  johnson closed form for {len(allsrc)} sources ...", flush=True)
    exp = johnson(g, allsrc)
    rec = solve_record(g, g.src, exp[0], samples=2000)
    rec.update({"n": g.n, "m": g.m, "graph_sha256": graph_digest(g),
                "certified_by": "johnson_closed_form"})
    batch = []
    for i, src in enumerate(srcs):
        r = solve_record(g, src, exp[1 + i], samples=64, seed=i)
        batch.append(r)
    return {"rmat20": rec,
            "rmat20_x64_sources": {"n": g.n, "m": g.m, "graph_sha256": graph_digest(g),
                                   "sources_seed": BATCH_SOURCES_SEED,
                                   "certified_by": "johnson_closed_form",
                                   "queries": batch}}


def er_golden():
    """The 256 Erdos-Renyi instances of the batched workload, each from its
    own source (a small sample of values per instance: the digests carry the
    exactness)."""
    queries = []
    for g in synth.er_batch(256):
        rec = solve_record(g, g.src, johnson(g, [g.src])[0], samples=16)
        rec.update({"n": g.n, "m": g.m, "graph_sha256": graph_digest(g)})
        queries.append(rec)
    return {"er256": {"count": len(queries), "certified_by": "johnson_closed_form",
                      "queries": queries}}


def grid_golden():
    g = synth.config_graph("grid64")
    rec = solve_record(g, g.src, dijkstra(g, g.src), samples=256)
    rec.update({"n": g.n, "m": g.m, "graph_sha256": graph_digest(g),
                "certified_by": "dijkstra"})
    return {"grid64": rec}


def main():
    which = sys.argv[1:] or ["grid", "rmat", "road", "er"]
    for name in which:
        print(f"{name} ...", flush=True)
        res = {"grid": grid_golden, "rmat": rmat_golden, "road": road_golden,
               "er": er_golden}[name]()
        path = os.path.join(HERE, {"grid": "grid64.json", "rmat": "rmat20.json",
                                   "road": "road2048.json", "er": "er256.json"}[name])
        with open(path, "w") as f:
            json.dump(res, f)
        print(f"wrote {path}", flush=True)


if __name__ == "__main__":
    main()
