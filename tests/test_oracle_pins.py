"""Pins of the CPU oracle against what the mathematics fixes independently of it.

Each test checks the oracle against something other than itself: brute-force
enumeration of simple paths and cycles, a library Dijkstra (scipy), the
closed form for potential-shifted weights (Johnson reweighting), BFS levels,
prefix sums on a path, dynamic programming on a DAG, planted negative cycles,
and collections.deque for the sequential FIFO.
"""
import collections

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.csgraph as csg

import oracle
import synth

INF = oracle.INF


# ---------------------------------------------------------------------------
# independent reference computations (none of them calls the oracle)
# ---------------------------------------------------------------------------

def _min_parallel(g):
    """{(u, v): min weight} over parallel edges."""
    s, d, w = synth.edges_of(g)
    best = {}
    for a, b, c in zip(s.tolist(), d.tolist(), w.tolist()):
        if (a, b) not in best or c < best[(a, b)]:
            best[(a, b)] = c
    return best


def brute_force(g, src):
    """Exhaustive simple-path enumeration (tiny graphs only).

    Returns (dist, neg, penult): dist[v] = min weight over simple paths
    src->v; neg = some simple cycle of negative weight contains a vertex
    reachable from src; penult[v] = set of second-to-last vertices over the
    minimum-weight simple paths to v.
    """
    n = g.n
    best = _min_parallel(g)
    adj = collections.defaultdict(list)
    for (a, b), c in best.items():
        adj[a].append((b, c))
    dist = [INF] * n
    penult = [set() for _ in range(n)]
    dist[src] = 0

    def dfs(u, seen, acc):
        for v, c in adj[u]:
            if v in seen:
                continue
            t = acc + c
            if t < dist[v]:
                dist[v] = t
                penult[v] = {u}
            elif t == dist[v]:
                penult[v].add(u)
            dfs(v, seen | {v}, t)

    dfs(src, {src}, 0)
    reach = {v for v in range(n) if dist[v] != INF}
    neg = False
    # every simple cycle is enumerated once, from its smallest vertex s0; a
    # cycle has a reachable vertex iff all its vertices (s0 too) are reachable
    for s0 in sorted(reach):

        def cyc(u, seen, acc):
            nonlocal neg
            for v, c in adj[u]:
                if v == s0:
                    if acc + c < 0:
                        neg = True
                elif v > s0 and v not in seen:
                    cyc(v, seen | {v}, acc + c)

        cyc(s0, {s0}, 0)
    return np.array(dist, dtype=np.int64), neg, penult


def brute_neg_inf(g, src):
    """Minus-infinity vertices by enumeration (tiny graphs only): the
    vertices reachable from a simple cycle of negative weight whose vertices
    src reaches. Returns a bool array."""
    n = g.n
    best = _min_parallel(g)
    adj = collections.defaultdict(list)
    for (a, b), c in best.items():
        adj[a].append((b, c))

    def reach_from(starts):
        seen = set(starts)
        todo = list(starts)
        while todo:
            u = todo.pop()
            for v, _ in adj[u]:
                if v not in seen:
                    seen.add(v)
                    todo.append(v)
        return seen

    reach = reach_from([src])
    on_neg = set()
    for s0 in sorted(reach):

        def cyc(u, path, acc):
            for v, c in adj[u]:
                if v == s0:
                    if acc + c < 0:
                        on_neg.update(path)
                elif v > s0 and v not in path:
                    cyc(v, path + [v], acc + c)

        cyc(s0, [s0], 0)
    out = np.zeros(n, dtype=bool)
    for v in reach_from(sorted(on_neg)):
        out[v] = True
    return out


def scipy_dijkstra(g, w=None, src=None):
    """Library Dijkstra on min-deduplicated edges (all weights must be >= 1)."""
    s, d, ww = synth.edges_of(g)
    if w is not None:
        ww = np.asarray(w, dtype=np.int64)
    assert ww.min() >= 1
    order = np.lexsort((ww, d, s))
    s, d, ww = s[order], d[order], ww[order]
    keep = np.ones(s.size, dtype=bool)
    keep[1:] = (s[1:] != s[:-1]) | (d[1:] != d[:-1])
    mat = sp.csr_matrix((ww[keep].astype(np.float64), (s[keep], d[keep])), shape=(g.n, g.n))
    r = csg.dijkstra(mat, directed=True, indices=g.src if src is None else src)
    out = np.full(g.n, INF, dtype=np.int64)
    fin = np.isfinite(r)
    out[fin] = r[fin].astype(np.int64)
    return out


def johnson_expected(g, src=None):
    """Potential-shifted weights w = w0 + p(u) - p(v): every path P from s to
    v has w(P) = w0(P) + p(s) - p(v), so d_w(v) = d_w0(v) + p(s) - p(v)."""
    s_, d_, w = synth.edges_of(g)
    p = g.meta["potential"].astype(np.int64)
    w0 = w - p[s_] + p[d_]
    src = g.src if src is None else src
    d0 = scipy_dijkstra(g, w0, src)
    out = np.full(g.n, INF, dtype=np.int64)
    fin = d0 != INF
    out[fin] = d0[fin] + p[src] - p[np.nonzero(fin)[0]]
    return out


def check_certificate(g, src, dist, pred):
    """Feasibility + tight acyclic src-rooted predecessor tree => exact
    shortest distances (needs no reference answer); INF iff unreachable."""
    s, d, w = synth.edges_of(g)
    assert dist[src] == 0 and pred[src] == -1
    fin = dist[s] != INF
    assert np.all(dist[d[fin]] <= dist[s[fin]] + w[fin]), "infeasible edge"
    reach = csg.breadth_first_order(
        sp.csr_matrix((np.ones(g.m), (s, d)), shape=(g.n, g.n)), src, directed=True,
        return_predecessors=False)
    reached = np.zeros(g.n, dtype=bool)
    reached[reach] = True
    assert np.array_equal(reached, dist != INF), "INF does not match unreachability"
    vs = np.nonzero(reached)[0]
    vs = vs[vs != src]
    assert np.all(pred[vs] >= 0)
    best = _min_parallel(g) if g.m < 200_000 else None
    if best is not None:
        for v in vs.tolist():
            u = int(pred[v])
            assert (u, v) in best and dist[u] != INF
            # some parallel edge u->v is tight (the min one is the tightest)
            assert dist[u] + best[(u, v)] <= dist[v]
    # acyclic and rooted: following pred from any reached vertex ends at src
    node = vs.copy()
    steps = 0
    while node.size:
        node = pred[node]
        steps += 1
        assert steps <= g.n, "pred graph has a cycle"
        node = node[node != src]


# ---------------------------------------------------------------------------
# tests
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(400))
def test_brute_force_tiny(seed):
    """Simple-path / simple-cycle enumeration on tiny multigraphs with
    negative weights and self-loops: distances and the flag."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 8))
    m = int(rng.integers(0, 3 * n + 1))
    g = synth.random_small(n, m, -5, 10, seed=1000 + seed)
    src = int(rng.integers(0, n))
    d_bf, neg_bf, _ = brute_force(g, src)
    d2, neg2, _ = oracle.bf_rounds(g, src)
    d3, neg3, _, _ = oracle.bf_fifo(g, src)
    assert neg2 == neg_bf
    assert neg3 == neg_bf
    if not neg_bf:
        assert np.array_equal(d2, d_bf)
        assert np.array_equal(d3, d_bf)


@pytest.mark.parametrize("seed", range(150))
def test_pred_is_smallest_penultimate(seed):
    """On graphs with no zero- or negative-weight cycles, the smallest tight
    in-neighbour equals the smallest second-to-last vertex over all
    minimum-weight simple paths (enumerated)."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 8))
    m = int(rng.integers(0, 3 * n + 1))
    if seed % 2:
        g = synth.potential_random(n, m, seed=5000 + seed, w0_hi=6, p_hi=6)
    else:
        g = synth.random_small(n, m, 1, 6, seed=5000 + seed)
    src = int(rng.integers(0, n))
    d_bf, neg_bf, penult = brute_force(g, src)
    assert not neg_bf
    d, p, neg = oracle.sssp(g, src)
    assert not neg and np.array_equal(d, d_bf)
    for v in range(n):
        if v == src or d_bf[v] == INF:
            assert p[v] == -1
        else:
            assert p[v] == min(penult[v])


@pytest.mark.parametrize("edges", [
    ([0, 0, 1, 2], [1, 2, 3, 3], [1, 1, 1, 1]),
    ([0, 0, 0, 0, 2, 3, 4, 1], [2, 3, 4, 1, 5, 5, 5, 5], [2, 1, 1, 1, 1, 2, 2, 2]),
])
def test_pred_ties_consecutive_ids(edges):
    """Several tight in-neighbours with consecutive ids: the smallest wins."""
    s, t, w = edges
    n = max(max(s), max(t)) + 1
    g = synth.csr_from_edges(n, s, t, w)
    d_bf, _, penult = brute_force(g, 0)
    d, p, neg = oracle.sssp(g, 0)
    assert np.array_equal(d, d_bf)
    assert p[n - 1] == min(penult[n - 1])


def test_dijkstra_grid64():
    g = synth.grid64()
    assert g.n == 4096 and g.m == 16128
    d, p, neg = oracle.sssp(g)
    assert not neg
    assert np.array_equal(d, scipy_dijkstra(g))
    check_certificate(g, g.src, d, p)
    d3, neg3, _, _ = oracle.bf_fifo(g)
    assert not neg3 and np.array_equal(d3, d)


@pytest.mark.parametrize("seed", range(6))
def test_dijkstra_random_positive(seed):
    g = synth.random_small(300, 1500, 1, 50, seed=77 + seed)
    d, p, neg = oracle.sssp(g)
    assert not neg
    assert np.array_equal(d, scipy_dijkstra(g))
    check_certificate(g, 0, d, p)


@pytest.mark.parametrize("maker", [
    lambda: synth.rmat(12, 16, seed=11),
    lambda: synth.road(48, plant_cycle=False, seed=12),
    lambda: synth.erdos_renyi(3000, 8, seed=13),
    lambda: synth.potential_random(500, 4000, seed=14),
])
def test_johnson_closed_form(maker):
    """Potential-shifted graphs (negative edges, no negative cycle): the
    closed form from a library Dijkstra on w0 must equal both oracles."""
    g = maker()
    exp = johnson_expected(g)
    d2, neg2, _ = oracle.bf_rounds(g)
    d3, neg3, _, _ = oracle.bf_fifo(g)
    assert not neg2 and not neg3
    assert np.array_equal(d2, exp)
    assert np.array_equal(d3, exp)
    check_certificate(g, g.src, d2, oracle.pred(g, d2))


def test_unit_weights_bfs_levels():
    g = synth.random_small(2000, 9000, 1, 1, seed=5)
    d, p, neg = oracle.sssp(g)
    s, t, _ = synth.edges_of(g)
    mat = sp.csr_matrix((np.ones(g.m), (s, t)), shape=(g.n, g.n))
    lv = csg.shortest_path(mat, directed=True, unweighted=True, indices=0)
    exp = np.where(np.isfinite(lv), lv, -1).astype(np.int64)
    exp[exp < 0] = INF
    assert np.array_equal(d, exp)


@pytest.mark.parametrize("reverse", [False, True])
def test_path_prefix_sums(reverse):
    """A path graph needs n-1 rounds; distances are prefix sums (with
    negative weights too). Reversed ids make every round advance by one edge
    only, which also exercises the last round before the cycle test."""
    n = 200
    rng = np.random.default_rng(3)
    w = rng.integers(-50, 50, size=n - 1)
    ids = np.arange(n)[::-1] if reverse else np.arange(n)
    g = synth.csr_from_edges(n, ids[:-1], ids[1:], w, source=int(ids[0]))
    d, neg, rounds = oracle.bf_rounds(g)
    assert not neg
    exp = np.zeros(n, dtype=np.int64)
    exp[ids[1:]] = np.cumsum(w)
    assert np.array_equal(d, exp)
    if reverse:
        assert rounds == n  # n-1 improving rounds + one quiet round
    d3, neg3, _, _ = oracle.bf_fifo(g)
    assert not neg3 and np.array_equal(d3, exp)


@pytest.mark.parametrize("seed", range(5))
def test_dag_topological_dp(seed):
    """Random DAG (edges go from lower to higher topological rank) with
    negative weights: dynamic programming in topological order."""
    rng = np.random.default_rng(seed)
    n, m = 400, 3000
    rank = rng.permutation(n)          # vertex -> rank
    a = rng.integers(0, n, size=m)
    b = rng.integers(0, n, size=m)
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    ok = lo != hi
    lo, hi = lo[ok], hi[ok]
    inv = np.argsort(rank)             # rank -> vertex
    s, t = inv[lo], inv[hi]
    w = rng.integers(-100, 100, size=s.size)
    src = int(inv[0])
    g = synth.csr_from_edges(n, s, t, w, source=src)
    exp = np.full(n, INF, dtype=np.int64)
    exp[src] = 0
    order = np.argsort(lo, kind="stable")
    for i in order:
        if exp[s[i]] != INF:
            exp[t[i]] = min(exp[t[i]], exp[s[i]] + w[i])
    d, p, neg = oracle.sssp(g)
    assert not neg and np.array_equal(d, exp)


@pytest.mark.parametrize("cyc_len", [1, 2, 3, 7, 40])
@pytest.mark.parametrize("reachable", [True, False])
def test_planted_negative_cycle(cyc_len, reachable):
    """A potential-shifted graph has no negative cycle; plant one of total
    weight -1 among fresh vertices, joined to the graph (reachable) or in a
    separate component (not reachable from src)."""
    base = synth.potential_random(300, 2000, seed=cyc_len * 10 + reachable)
    s, t, w = synth.edges_of(base)
    n0 = base.n
    cyc = np.arange(n0, n0 + cyc_len)
    cw = np.full(cyc_len, 5, dtype=np.int64)
    cw[-1] = -(5 * (cyc_len - 1)) - 1          # cycle total = -1
    cs, ct = cyc, np.roll(cyc, -1)
    extra_s = [cs]
    extra_t = [ct]
    extra_w = [cw]
    if reachable:
        extra_s.append(np.array([0]))
        extra_t.append(np.array([n0]))
        extra_w.append(np.array([3]))
    else:
        # the cycle reaches the main graph, but nothing reaches the cycle
        extra_s.append(np.array([n0]))
        extra_t.append(np.array([5]))
        extra_w.append(np.array([3]))
    g = synth.csr_from_edges(n0 + cyc_len, np.concatenate([s] + extra_s),
                             np.concatenate([t] + extra_t), np.concatenate([w] + extra_w),
                             source=0)
    d2, neg2, _ = oracle.bf_rounds(g)
    d3, neg3, _, _ = oracle.bf_fifo(g)
    assert neg2 == reachable
    assert neg3 == reachable
    if not reachable:
        assert np.array_equal(d2, d3)
        assert np.all(d2[cyc] == INF)


def test_negative_self_loop():
    g = synth.csr_from_edges(3, [0, 1, 1], [1, 1, 2], [4, -1, 2], source=0)
    assert oracle.bf_rounds(g)[1] and oracle.bf_fifo(g)[1]
    g2 = synth.csr_from_edges(3, [0, 2, 1], [1, 2, 2], [4, -1, 2], source=1)
    # vertex 2 has the negative loop and is reachable from 1
    assert oracle.bf_rounds(g2)[1] and oracle.bf_fifo(g2)[1]
    g3 = synth.csr_from_edges(3, [0, 2], [1, 2], [4, -1], source=0)
    assert not oracle.bf_rounds(g3)[1] and not oracle.bf_fifo(g3)[1]


def test_road_planted_cycle_small():
    """The road generator's planted 3-cycle (weight -3) is found; without it
    the closed form holds."""
    ga = synth.road(40, plant_cycle=False, seed=99)
    gb = synth.road(40, plant_cycle=True, seed=99)
    assert not oracle.bf_rounds(ga)[1]
    assert np.array_equal(oracle.bf_rounds(ga)[0], johnson_expected(ga))
    assert oracle.bf_rounds(gb)[1]
    assert oracle.bf_fifo(gb)[1]
    a, b, c = gb.meta["cycle"]
    s, t, w = synth.edges_of(gb)
    tot = sum(int(w[(s == x) & (t == y)].min()) for x, y in ((a, b), (b, c), (c, a)))
    assert tot == -3


def test_unreachable_and_isolated():
    g = synth.csr_from_edges(5, [0, 1, 3], [1, 2, 4], [1, 1, -7], source=0)
    d, p, neg = oracle.sssp(g)
    assert not neg
    assert d.tolist() == [0, 1, 2, INF, INF]
    assert p.tolist() == [-1, 0, 1, -1, -1]
    g1 = synth.csr_from_edges(1, [], [], [], source=0)
    d, p, neg = oracle.sssp(g1)
    assert d.tolist() == [0] and p.tolist() == [-1] and not neg


def test_multi_edges_take_min_and_zero_cycle():
    g = synth.csr_from_edges(3, [0, 0, 0, 1, 2], [1, 1, 2, 2, 1], [9, 2, 5, 3, -3],
                             source=0)
    d, p, neg = oracle.sssp(g)
    assert not neg
    assert d.tolist() == [0, 2, 5]
    # 1 <-> 2 is a zero-weight cycle: 2 is a tight in-neighbour of 1 only if
    # d[2] - 3 == d[1] (5 - 3 = 2): both 0 and 2 are tight; smallest is 0
    assert p.tolist() == [-1, 0, 0]


@pytest.mark.parametrize("seed", range(20))
def test_fifo_matches_deque(seed):
    rng = np.random.default_rng(seed)
    cap = int(rng.integers(1, 9))
    k = 300
    ops = np.where(rng.random(k) < 0.55, rng.integers(0, 10**6, size=k), -1)
    res, out, size = oracle.fifo_run(cap, ops)
    q = collections.deque()
    for i, op in enumerate(ops.tolist()):
        if op >= 0:
            ok = len(q) < cap
            if ok:
                q.append(op)
            assert res[i] == ok
        else:
            if q:
                assert res[i] == 1 and out[i] == q.popleft()
            else:
                assert res[i] == 0
    assert size == len(q)


@pytest.mark.slow
def test_rmat_medium_rounds_vs_fifo():
    g = synth.rmat(15, 16, seed=21)
    d2, neg2, rounds = oracle.bf_rounds(g)
    d3, neg3, pops, relax = oracle.bf_fifo(g)
    assert not neg2 and not neg3
    assert np.array_equal(d2, d3)
    assert np.array_equal(d2, johnson_expected(g))
    assert pops >= np.count_nonzero(d2 != INF) - 1


# ---------------------------------------------------------------------------
# minus-infinity marking
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(400))
def test_neg_inf_brute_tiny(seed):
    """The marked set is the set reachable from reachable negative simple
    cycles; every other reached vertex keeps its exact (simple-path) distance
    and a tight predecessor."""
    rng = np.random.default_rng(20000 + seed)
    n = int(rng.integers(1, 8))
    m = int(rng.integers(0, 3 * n + 1))
    g = synth.random_small(n, m, -5, 10, seed=21000 + seed)
    src = int(rng.integers(0, n))
    d, p, neg = oracle.neg_inf(g, src)
    mk = brute_neg_inf(g, src)
    assert np.array_equal(d == oracle.NEG_INF, mk)
    assert neg == bool(mk.any())
    assert neg == brute_force(g, src)[1]
    # vertices no negative cycle reaches: distances of the simple paths that
    # avoid the marked vertices (a path through one would make them marked)
    keep = np.nonzero(~mk)[0]
    sub_s, sub_t, sub_w = synth.edges_of(g)
    ok = ~mk[sub_s] & ~mk[sub_t]
    if not mk[src]:
        sub = synth.csr_from_edges(n, sub_s[ok], sub_t[ok], sub_w[ok], source=src)
        d_bf, _, _ = brute_force(sub, src)
        assert np.array_equal(d[keep], d_bf[keep])
    best = _min_parallel(g)
    for v in range(n):
        if mk[v] or d[v] == INF or v == src:
            assert p[v] == -1
        else:
            u = int(p[v])
            assert (u, v) in best and not mk[u] and d[u] + best[(u, v)] == d[v]


def test_neg_inf_no_cycle_is_plain():
    for seed in range(5):
        g = synth.potential_random(800, 5000, seed=22000 + seed)
        d, p, neg = oracle.neg_inf(g)
        d2, p2, neg2 = oracle.sssp(g, method="fifo")
        assert not neg and not neg2
        assert np.array_equal(d, d2) and np.array_equal(p, p2)


def test_neg_inf_long_path_then_cycle():
    """A reversed-id path of 50 vertices needs all n-1 rounds before its end
    is exact; a negative cycle hangs off the middle and reaches a tail."""
    n = 60
    ids = np.arange(50)[::-1]
    s = list(ids[:-1])
    t = list(ids[1:])
    w = list(np.random.default_rng(5).integers(-20, 20, size=49))
    # cycle 50 -> 51 -> 52 -> 50 of weight -1, entered from path vertex ids[25]
    s += [int(ids[25]), 50, 51, 52, 52, 53]
    t += [50, 51, 52, 50, 53, 54]
    w += [3, 1, 1, -3, 4, 4]
    g = synth.csr_from_edges(n, s, t, w, source=int(ids[0]))
    d, p, neg = oracle.neg_inf(g)
    assert neg
    exp = np.zeros(50, dtype=np.int64)
    exp[ids[1:]] = np.cumsum(w[:49])
    assert np.array_equal(d[:50], exp)
    assert np.all(d[50:55] == oracle.NEG_INF)
    assert np.all(d[55:] == INF)
    assert np.all(p[50:] == -1)


# ---------------------------------------------------------------------------
# the multi-core timing baseline gives the oracle's results
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(60))
def test_jacobi_baseline_matches_rounds(seed):
    rng = np.random.default_rng(30000 + seed)
    n = int(rng.integers(1, 80))
    g = synth.random_small(n, int(rng.integers(0, 5 * n + 1)), -6, 30, seed=31000 + seed)
    src = int(rng.integers(0, n))
    d, neg, rounds, threads = oracle.bf_jacobi(g, oracle.transpose(g), src)
    d_ref, neg_ref, _ = oracle.bf_rounds(g, src)
    assert neg == neg_ref and threads >= 1
    if not neg:
        assert np.array_equal(d, d_ref)


def test_jacobi_baseline_medium():
    g = synth.rmat(14, 16, seed=5)
    d, neg, rounds, threads = oracle.bf_jacobi(g, oracle.transpose(g))
    d_ref, neg_ref, _ = oracle.bf_rounds(g)
    assert not neg and not neg_ref and np.array_equal(d, d_ref)
