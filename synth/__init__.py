"""Seeded synthetic inputs for the queue-driven Bellman-Ford path.

This module only builds inputs: graphs in CSR form, edge weights, sources and
queue payloads. It holds none of the method's arithmetic (no relaxation, no
queue protocol, no distances), so both the CPU oracle and the HIP path can be
fed from it without sharing any code with each other.

Every generator is deterministic from its seed (numpy's PCG64 through a
SeedSequence, with one spawned sub-stream per purpose: structure, base
weights, potentials, sources), so the same call produces the same bytes on any
machine with this numpy.

Graph shapes stand in for the paper's SuiteSparse inputs (Section IV, Table 1),
which are not available: road-like meshes, power-law (RMAT) and uniform random
(Erdos-Renyi) graphs.

CSR convention used everywhere: ``offsets`` int64[n+1], ``cols`` int32[m],
``w`` int32[m]; edges of vertex u are ``cols[offsets[u]:offsets[u+1]]``, kept
in generation order within a row (stable sort by source). Self-loops and
parallel edges are allowed.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 0x5EED0000


@dataclass
class Graph:
    n: int
    offsets: np.ndarray  # int64[n+1]
    cols: np.ndarray     # int32[m]
    w: np.ndarray        # int32[m]
    src: int = 0
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.cols.shape[0])

    def nbytes(self) -> int:
        return self.offsets.nbytes + self.cols.nbytes + self.w.nbytes


def _streams(seed: int, k: int):
    ss = np.random.SeedSequence(seed)
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(k)]


def csr_from_edges(n: int, src: np.ndarray, dst: np.ndarray, w: np.ndarray,
                   name: str = "", source: int = 0, meta: dict | None = None) -> Graph:
    """Stable-sort an edge list by source into CSR (row order = list order)."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    w = np.asarray(w)
    if src.size:
        if src.min() < 0 or src.max() >= n or dst.min() < 0 or dst.max() >= n:
            raise ValueError("edge endpoint out of range")
    if w.size and (w.min() < np.iinfo(np.int32).min or w.max() > np.iinfo(np.int32).max):
        raise ValueError("weight outside int32")
    order = np.argsort(src, kind="stable")
    counts = np.bincount(src, minlength=n).astype(np.int64)
    offsets = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    return Graph(n=n, offsets=offsets, cols=dst[order].astype(np.int32),
                 w=w[order].astype(np.int32), src=int(source), name=name,
                 meta=dict(meta or {}))


def edges_of(g: Graph):
    """(src, dst, w) arrays of a CSR graph, in CSR order."""
    deg = np.diff(g.offsets)
    src = np.repeat(np.arange(g.n, dtype=np.int64), deg)
    return src, g.cols.astype(np.int64), g.w.astype(np.int64)


# ----------------------------------------------------------------------------
# weights
# ----------------------------------------------------------------------------

def potential_shift(src, dst, rng_w0, rng_p, n, w0_lo=1, w0_hi=1000, p_lo=0, p_hi=1000):
    """Weights w = w0 + p(u) - p(v) with w0 ~ U{w0_lo..w0_hi} and p ~ U{p_lo..p_hi}.

    Some edges get negative weights, yet every cycle weighs sum(w0) >= 1, so
    there is no negative cycle (the potentials cancel around any cycle).
    Returns (w, w0, p), all int64.
    """
    w0 = rng_w0.integers(w0_lo, w0_hi + 1, size=src.shape[0], dtype=np.int64)
    p = rng_p.integers(p_lo, p_hi + 1, size=n, dtype=np.int64)
    w = w0 + p[src] - p[dst]
    return w, w0, p


# ----------------------------------------------------------------------------
# graph families
# ----------------------------------------------------------------------------

def grid_edges(rows: int, cols: int):
    """4-neighbour mesh, both directions; vertex id = r*cols + c.

    Edge order: for every vertex, right, left, down, up (the ones in bounds);
    the CSR sort keeps that order within each row.
    """
    r, c = np.divmod(np.arange(rows * cols, dtype=np.int64), cols)
    vid = r * cols + c
    parts_s, parts_d = [], []
    for dr, dc in ((0, 1), (0, -1), (1, 0), (-1, 0)):
        ok = (r + dr >= 0) & (r + dr < rows) & (c + dc >= 0) & (c + dc < cols)
        parts_s.append(vid[ok])
        parts_d.append(vid[ok] + dr * cols + dc)
    return np.concatenate(parts_s), np.concatenate(parts_d)


def grid64(seed: int = SEED_BASE + 0, side: int = 64) -> Graph:
    """64x64 4-neighbour grid, w ~ U{1..100} independently per direction, src 0."""
    (rw,) = _streams(seed, 1)
    s, d = grid_edges(side, side)
    w = rw.integers(1, 101, size=s.shape[0], dtype=np.int64)
    return csr_from_edges(side * side, s, d, w, name=f"grid{side}x{side}", source=0,
                          meta={"seed": seed, "family": "grid"})


def rmat_edges(scale: int, edge_factor: int, a: float, b: float, c: float, rng):
    """RMAT edges (no noise), self-loops and duplicates kept, then a seeded
    vertex relabelling (the Graph500 convention)."""
    n = 1 << scale
    m = edge_factor * n
    src = np.zeros(m, dtype=np.int64)
    dst = np.zeros(m, dtype=np.int64)
    ab, abc = a + b, a + b + c
    for bit in range(scale):
        q = rng.random(m)
        row = q >= ab                      # quadrants c, d
        col = (q >= a) & (q < ab) | (q >= abc)  # quadrants b, d
        src |= row.astype(np.int64) << bit
        dst |= col.astype(np.int64) << bit
    perm = rng.permutation(n).astype(np.int64)
    return n, perm[src], perm[dst]


def max_degree_source(offsets: np.ndarray) -> int:
    deg = np.diff(offsets)
    return int(np.argmax(deg))  # first (lowest id) on ties


def rmat(scale: int = 20, edge_factor: int = 16, a=0.57, b=0.19, c=0.19,
         seed: int = SEED_BASE + 1) -> Graph:
    """RMAT graph with potential-shifted weights; source = max out-degree vertex."""
    rs, rw, rp = _streams(seed, 3)
    n, s, d = rmat_edges(scale, edge_factor, a, b, c, rs)
    w, _, p = potential_shift(s, d, rw, rp, n)
    g = csr_from_edges(n, s, d, w, name=f"rmat{scale}", meta={
        "seed": seed, "family": "rmat", "scale": scale, "edge_factor": edge_factor})
    g.src = max_degree_source(g.offsets)
    g.meta["potential"] = p
    return g


def road(side: int = 2048, shortcut_frac: float = 0.01, plant_cycle: bool = False,
         seed: int = SEED_BASE + 2) -> Graph:
    """Road-like large-diameter mesh: side x side 4-neighbour grid plus
    round(shortcut_frac * grid edges) directed diagonal shortcuts, each from a
    uniform random vertex to a uniform random in-bounds diagonal neighbour;
    potential-shifted weights; source 0 (the corner).

    With ``plant_cycle`` the three vertices a=(h,h), b=(h,h+1), c=(h+1,h+1),
    h = side//2, get the edges a->b, b->c (already in the mesh) and an added
    c->a, all three with w0 = -1: a cycle of weight -3. Any other cycle through
    them still weighs >= 0, so it is the only negative simple cycle.
    """
    rs, rw, rp = _streams(seed, 3)
    gs, gd = grid_edges(side, side)
    n = side * side
    k = int(round(shortcut_frac * gs.shape[0]))
    v = rs.integers(0, n, size=k, dtype=np.int64)
    r, cc = np.divmod(v, side)
    # pick uniformly among the in-bounds diagonal neighbours
    diag = np.array([(-1, -1), (-1, 1), (1, -1), (1, 1)], dtype=np.int64)
    okm = np.stack([(r + dr >= 0) & (r + dr < side) & (cc + dc >= 0) & (cc + dc < side)
                    for dr, dc in diag], axis=1)
    cnt = okm.sum(axis=1)
    pick = (rs.random(k) * cnt).astype(np.int64)
    csum = np.cumsum(okm, axis=1)
    which = np.argmax(csum > pick[:, None], axis=1)
    sd = (r + diag[which, 0]) * side + (cc + diag[which, 1])
    s = np.concatenate([gs, v])
    d = np.concatenate([gd, sd])
    meta = {"seed": seed, "family": "road", "side": side, "shortcuts": k,
            "planted_cycle": bool(plant_cycle)}
    w, w0, p = potential_shift(s, d, rw, rp, n)
    if plant_cycle:
        h = side // 2
        a_, b_, c_ = h * side + h, h * side + h + 1, (h + 1) * side + h + 1
        # replace w0 of the existing mesh edges a->b and b->c
        for (x, y) in ((a_, b_), (b_, c_)):
            idx = np.nonzero((s[: gs.shape[0]] == x) & (d[: gs.shape[0]] == y))[0]
            assert idx.size == 1
            w0[idx[0]] = -1
        s = np.concatenate([s, [c_]])
        d = np.concatenate([d, [a_]])
        w0 = np.concatenate([w0, [-1]])
        w = w0 + p[s] - p[d]
        meta["cycle"] = (a_, b_, c_)
    g = csr_from_edges(n, s, d, w, name=f"road{side}" + ("_negcycle" if plant_cycle else ""),
                       source=0, meta=meta)
    g.meta["potential"] = p
    return g


def erdos_renyi(n: int, avg_degree: int = 8, seed: int = SEED_BASE + 3,
                source: int | None = None) -> Graph:
    """G(n, m = avg_degree*n): uniform endpoints, no self-loops, duplicates
    allowed; potential-shifted weights; source uniform unless given."""
    rs, rw, rp, rsrc = _streams(seed, 4)
    m = avg_degree * n
    s = rs.integers(0, n, size=m, dtype=np.int64)
    d = rs.integers(0, n - 1, size=m, dtype=np.int64)
    d = d + (d >= s)
    w, _, p = potential_shift(s, d, rw, rp, n)
    src = int(rsrc.integers(0, n)) if source is None else int(source)
    g = csr_from_edges(n, s, d, w, name=f"er{n}", source=src,
                       meta={"seed": seed, "family": "er", "avg_degree": avg_degree})
    g.meta["potential"] = p
    return g


def er_batch_sizes(count: int = 256, lo: float = 1e3, hi: float = 2e5,
                   seed: int = SEED_BASE + 3) -> np.ndarray:
    """Instance sizes log-uniform in [lo, hi] (batched workload)."""
    (r,) = _streams(seed ^ 0xB47C, 1)
    return np.rint(np.exp(r.uniform(np.log(lo), np.log(hi), size=count))).astype(np.int64)


def er_batch(count: int = 256, lo: float = 1e3, hi: float = 2e5,
             seed: int = SEED_BASE + 3):
    """The batched workload: ``count`` ER instances of log-uniform size, each
    with its own seed and random source."""
    sizes = er_batch_sizes(count, lo, hi, seed)
    return [erdos_renyi(int(nv), 8, seed=seed * 1000 + i) for i, nv in enumerate(sizes)]


def random_sources(g: Graph, k: int, seed: int) -> np.ndarray:
    """k distinct sources drawn uniformly from vertices with out-degree > 0."""
    (r,) = _streams(seed, 1)
    cand = np.nonzero(np.diff(g.offsets) > 0)[0]
    return np.sort(r.choice(cand, size=min(k, cand.size), replace=False)).astype(np.int64)


def random_small(n: int, m: int, wlo: int, whi: int, seed: int, self_loops=True) -> Graph:
    """Small random multigraph for parity and pin tests."""
    rs, rw = _streams(seed, 2)
    s = rs.integers(0, n, size=m, dtype=np.int64)
    d = rs.integers(0, n, size=m, dtype=np.int64)
    if not self_loops and n > 1:
        d = rs.integers(0, n - 1, size=m, dtype=np.int64)
        d = d + (d >= s)
    w = rw.integers(wlo, whi + 1, size=m, dtype=np.int64)
    return csr_from_edges(n, s, d, w, name=f"rand{n}_{m}", source=0, meta={"seed": seed})


def potential_random(n: int, m: int, seed: int, w0_hi: int = 1000, p_hi: int = 1000) -> Graph:
    """Small random multigraph with potential-shifted weights (no negative cycle)."""
    rs, rw, rp = _streams(seed, 3)
    s = rs.integers(0, n, size=m, dtype=np.int64)
    d = rs.integers(0, n, size=m, dtype=np.int64)
    w, _, p = potential_shift(s, d, rw, rp, n, 1, w0_hi, 0, p_hi)
    g = csr_from_edges(n, s, d, w, name=f"prand{n}_{m}", source=0, meta={"seed": seed})
    g.meta["potential"] = p
    return g


def queue_payload(n_items: int, producers: int) -> np.ndarray:
    """Payload for queue tests: item i from producer (i % producers) with
    sequence number (i // producers), packed as (producer << 20) | seq when it
    fits, so every item is distinct and names its producer and order."""
    i = np.arange(n_items, dtype=np.int64)
    return (((i % producers) << 20) | (i // producers)).astype(np.int32)


# named configurations -------------------------------------------------------

def config_graph(name: str) -> Graph:
    if name == "grid64":
        return grid64()
    if name == "rmat20":
        return rmat(20)
    if name == "road2048":
        return road(2048, plant_cycle=False)
    if name == "road2048_negcycle":
        return road(2048, plant_cycle=True)
    if name == "er200k":
        return erdos_renyi(200_000, 8, seed=SEED_BASE + 4)
    raise KeyError(name)
