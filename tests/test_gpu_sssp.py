"""GPU parity of the queue-driven Bellman-Ford (sssp_bf through the C ABI)
against the CPU oracle: distances, predecessors and the negative-cycle flag
must be bit-identical, on small graphs covering the edge cases, at sizes that
span many batches, chunks and ragged tails, and on the full-size workloads
in the launch shape the benchmark uses."""
import json
import os

import numpy as np
import pytest

import goldens
import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pkg = pytest.importorskip("paper_2608_21826_amd")

HERE = os.path.dirname(os.path.abspath(__file__))


def _dev(g):
    d = torch.device("cuda:0")
    return (torch.from_numpy(g.offsets).to(d), torch.from_numpy(g.cols).to(d),
            torch.from_numpy(g.w).to(d))


@pytest.fixture(scope="module")
def ctx():
    c = pkg.SsspContext(1 << 16, 1 << 20)
    yield c
    c.close()


def run(ctx, g, src=None, launch=None, validate=True):
    src = g.src if src is None else src
    print(f"[sssp] {g.name} n={g.n} m={g.m} src={src} launch={launch}", flush=True)
    off, col, w = _dev(g)
    dist, pred, neg = ctx.solve(off, col, w, src, launch=launch, validate=validate)
    torch.cuda.synchronize()
    return dist.cpu().numpy(), pred.cpu().numpy(), neg


def check(ctx, g, src=None, launch=None, method="rounds"):
    src = g.src if src is None else src
    d, p, neg = run(ctx, g, src, launch)
    d_ref, p_ref, neg_ref = oracle.sssp(g, src, method=method)
    assert neg == neg_ref
    if not neg_ref:
        bad = np.nonzero(d != d_ref)[0]
        assert bad.size == 0, f"dist differs at {bad[:5]}: {d[bad[:5]]} vs {d_ref[bad[:5]]}"
        bad = np.nonzero(p != p_ref)[0]
        assert bad.size == 0, f"pred differs at {bad[:5]}: {p[bad[:5]]} vs {p_ref[bad[:5]]}"
    return d, p, neg


def test_grid64(ctx):
    g = synth.grid64()
    check(ctx, g)
    st = ctx.stats()
    assert st["relaxations"] >= g.m and st["dequeued"] >= g.n


@pytest.mark.parametrize("seed", range(40))
def test_random_small_negative(ctx, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 60))
    m = int(rng.integers(0, 5 * n + 1))
    g = synth.random_small(n, m, -6, 30, seed=900 + seed)
    check(ctx, g, src=int(rng.integers(0, n)))


@pytest.mark.parametrize("seed", range(12))
def test_potential_shifted_medium(ctx, seed):
    g = synth.potential_random(3000 + 500 * seed, 20000 + 3000 * seed, seed=300 + seed)
    check(ctx, g, method="fifo")


@pytest.mark.parametrize("b", [1, 2, 4])
@pytest.mark.parametrize("wgs", [1, 3, 0])
def test_launch_shapes(ctx, b, wgs):
    g = synth.potential_random(20000, 160000, seed=77)
    check(ctx, g, launch={"ticket_batch": b, "wg_count": wgs}, method="fifo")


@pytest.mark.parametrize("wgs", [1, 5, 0])
@pytest.mark.parametrize("b", [1, 4])
def test_bwd_policy(ctx, wgs, b):
    """The BWD broker policy changes only how dequeues take from the count;
    the results are the same."""
    g = synth.potential_random(20000, 160000, seed=78)
    check(ctx, g, launch={"ticket_batch": b, "wg_count": wgs, "flags": pkg.BQ_F_BWD},
          method="fifo")


@pytest.mark.parametrize("seg", [1, 2, 3, 8])
@pytest.mark.parametrize("wgs", [2, 9, 0])
def test_queue_segments(ctx, seg, wgs):
    """The queue split into segments (home by workgroup, stealing from the
    fullest other segment) gives the same results, also with segments that
    no workgroup calls home."""
    g = synth.potential_random(20000, 160000, seed=79)
    check(ctx, g, launch={"segments": seg, "wg_count": wgs, "ticket_batch": 2}, method="fifo")


@pytest.mark.parametrize("seed", range(8))
def test_queue_segments_small_negative(ctx, seed):
    rng = np.random.default_rng(4200 + seed)
    n = int(rng.integers(1, 80))
    g = synth.random_small(n, int(rng.integers(0, 5 * n + 1)), -6, 30, seed=4300 + seed)
    check(ctx, g, src=int(rng.integers(0, n)), launch={"segments": 8, "wg_count": 16})


def test_queue_segments_rejects_too_many(ctx):
    g = synth.grid64()
    off, col, w = _dev(g)
    with pytest.raises(pkg.BQError) as e:
        ctx.solve(off, col, w, 0, launch={"segments": 9})
    assert e.value.status == pkg.BQ_EINVAL


@pytest.mark.parametrize("seed", range(6))
def test_bwd_policy_small_negative(ctx, seed):
    rng = np.random.default_rng(4000 + seed)
    n = int(rng.integers(1, 60))
    g = synth.random_small(n, int(rng.integers(0, 5 * n + 1)), -6, 30, seed=4100 + seed)
    check(ctx, g, src=int(rng.integers(0, n)), launch={"flags": pkg.BQ_F_BWD})


def test_single_vertex_and_no_edges(ctx):
    g = synth.csr_from_edges(1, [], [], [])
    d, p, neg = run(ctx, g)
    assert d.tolist() == [0] and p.tolist() == [-1] and not neg
    g = synth.csr_from_edges(5, [], [], [], source=3)
    d, p, neg = run(ctx, g)
    assert d.tolist() == [oracle.INF] * 3 + [0, oracle.INF] and not neg


def test_self_loops_multi_edges_zero_cycles(ctx):
    g = synth.csr_from_edges(4, [0, 0, 0, 1, 2, 1, 3, 3], [1, 1, 2, 2, 1, 1, 3, 0],
                             [9, 2, 5, 3, -3, 0, 4, 1], source=0)
    check(ctx, g)


def test_hub_rows_are_split(ctx):
    """Rows longer than the chunk size are scanned as several queue items;
    a star with 30k leaves plus a second hub reached through it."""
    rng = np.random.default_rng(5)
    n = 40000
    s = [np.zeros(30000, dtype=np.int64), np.full(9000, 17, dtype=np.int64),
         rng.integers(0, n, size=20000)]
    t = [np.arange(1, 30001), rng.integers(0, n, size=9000), rng.integers(0, n, size=20000)]
    s, t = np.concatenate(s), np.concatenate(t)
    w = rng.integers(-5, 60, size=s.size)
    p = rng.integers(0, 50, size=n)
    w = np.abs(w) + p[s] - p[t] + 1
    g = synth.csr_from_edges(n, s, t, w, source=0)
    check(ctx, g, method="fifo")
    assert ctx.stats()["fanout"] > 0


@pytest.mark.parametrize("cyc_len", [1, 2, 3, 9, 200])
@pytest.mark.parametrize("reachable", [True, False])
def test_planted_negative_cycles(ctx, cyc_len, reachable):
    base = synth.potential_random(5000, 40000, seed=cyc_len + 31 * reachable)
    s, t, w = synth.edges_of(base)
    n0 = base.n
    cyc = np.arange(n0, n0 + cyc_len)
    cw = np.full(cyc_len, 7, dtype=np.int64)
    cw[-1] = -(7 * (cyc_len - 1)) - 2
    extra = (np.array([0, n0]), np.array([n0, 0]), np.array([5, 5]))
    if not reachable:
        extra = (np.array([n0]), np.array([0]), np.array([5]))
    g = synth.csr_from_edges(n0 + cyc_len, np.concatenate([s, cyc, extra[0]]),
                             np.concatenate([t, np.roll(cyc, -1), extra[1]]),
                             np.concatenate([w, cw, extra[2]]), source=0)
    d, p, neg = run(ctx, g)
    assert neg == reachable
    if not reachable:
        d_ref, p_ref, _ = oracle.sssp(g, method="fifo")
        assert np.array_equal(d, d_ref) and np.array_equal(p, p_ref)


# ---------------------------------------------------------------------------
# minus-infinity marking (BQ_F_NEGINF)
# ---------------------------------------------------------------------------

def check_neg_inf(ctx, g, src=None, launch=None):
    src = g.src if src is None else src
    print(f"[sssp] neg_inf {g.name} n={g.n} m={g.m} src={src} launch={launch}", flush=True)
    off, col, w = _dev(g)
    dist, pred, neg = ctx.solve(off, col, w, src, launch=launch, validate=True, neg_inf=True)
    d, p = dist.cpu().numpy(), pred.cpu().numpy()
    d_ref, p_ref, neg_ref = oracle.neg_inf(g, src)
    assert neg == neg_ref
    bad = np.nonzero(d != d_ref)[0]
    assert bad.size == 0, f"dist differs at {bad[:5]}: {d[bad[:5]]} vs {d_ref[bad[:5]]}"
    bad = np.nonzero(p != p_ref)[0]
    assert bad.size == 0, f"pred differs at {bad[:5]}: {p[bad[:5]]} vs {p_ref[bad[:5]]}"
    return neg


@pytest.mark.parametrize("seed", range(30))
def test_neg_inf_random_small(ctx, seed):
    rng = np.random.default_rng(8700 + seed)
    n = int(rng.integers(1, 60))
    g = synth.random_small(n, int(rng.integers(0, 4 * n + 1)), -6, 30, seed=8800 + seed)
    launch = {"segments": 8, "wg_count": 16} if seed % 2 else None
    check_neg_inf(ctx, g, src=int(rng.integers(0, n)), launch=launch)


def _cycle_with_tail(cyc_len, seed):
    base = synth.potential_random(1200, 9000, seed=seed)
    s, t, w = synth.edges_of(base)
    n0 = base.n
    cyc = np.arange(n0, n0 + cyc_len)
    cw = np.full(cyc_len, 4, dtype=np.int64)
    cw[-1] = -(4 * (cyc_len - 1)) - 1
    tail = np.arange(n0 + cyc_len, n0 + cyc_len + 50)
    ts = np.concatenate([[cyc[0]], tail[:-1]])
    return synth.csr_from_edges(
        n0 + cyc_len + 50,
        np.concatenate([s, [17], cyc, ts]),
        np.concatenate([t, [cyc[0]], np.roll(cyc, -1), tail]),
        np.concatenate([w, [5], cw, np.full(50, 2)]), source=0)


@pytest.mark.parametrize("cyc_len", [1, 2, 7, 300])
def test_neg_inf_cycle_with_tail(ctx, cyc_len):
    g = _cycle_with_tail(cyc_len, 8900 + cyc_len)
    assert check_neg_inf(ctx, g)
    assert check_neg_inf(ctx, g, launch={"segments": 1, "ticket_batch": 4})


def test_neg_inf_two_cycles_and_no_cycle(ctx):
    """Two separate negative cycles, each with its own downstream set."""
    g1 = _cycle_with_tail(3, 8950)
    s, t, w = synth.edges_of(g1)
    n = g1.n
    extra = (np.array([40, n, n + 1, n + 2]), np.array([n, n + 1, n + 2, n]),
             np.array([1, -2, -2, 3]))
    g = synth.csr_from_edges(n + 3, np.concatenate([s, extra[0]]),
                             np.concatenate([t, extra[1]]), np.concatenate([w, extra[2]]),
                             source=0)
    assert check_neg_inf(ctx, g)
    assert check_neg_inf(ctx, synth.road(48, plant_cycle=True, seed=8960))
    assert not check_neg_inf(ctx, synth.road(48, plant_cycle=False, seed=8960))
    assert not check_neg_inf(ctx, synth.potential_random(5000, 40000, seed=8961))


def test_solve_after_negative_cycle_reuses_context(ctx):
    g = synth.road(40, plant_cycle=True, seed=99)
    assert run(ctx, g)[2]
    check(ctx, synth.road(40, plant_cycle=False, seed=99), method="fifo")
    check(ctx, synth.grid64())


def test_range_error(ctx):
    g = synth.csr_from_edges(3, [0, 1], [1, 2], [2**31 - 1, -2**31 + 5], source=0)
    off, col, w = _dev(g)
    n_big = synth.csr_from_edges(40000, [0, 1], [1, 2], [2**31 - 1, 7], source=0)
    o2, c2, w2 = _dev(n_big)
    with pytest.raises(pkg.BQError) as e:
        ctx.solve(o2, c2, w2, 0)
    assert e.value.status == pkg.BQ_ERANGE
    # the context still works afterwards
    check(ctx, g)


def test_malformed_csr_rejected(ctx):
    g = synth.csr_from_edges(4, [0, 1, 2], [1, 2, 3], [1, 1, 1])
    off, col, w = _dev(g)
    bad = col.clone()
    bad[1] = 99
    with pytest.raises(pkg.BQError) as e:
        ctx.solve(off, bad, w, 0, validate=True)
    assert e.value.status == pkg.BQ_EINVAL
    with pytest.raises(pkg.BQError):
        ctx.solve(off, col, w, 7)
    check(ctx, g)


def test_repeated_solves_are_identical(ctx):
    g = synth.rmat(14, 16, seed=3)
    first = run(ctx, g)
    for _ in range(3):
        again = run(ctx, g)
        assert np.array_equal(first[0], again[0]) and np.array_equal(first[1], again[1])
    d_ref, p_ref, _ = oracle.sssp(g, method="fifo")
    assert np.array_equal(first[0], d_ref) and np.array_equal(first[1], p_ref)


# ---------------------------------------------------------------------------
# full-size workloads, default launch (as timed by bench.py)
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def big_ctx():
    c = pkg.SsspContext(1 << 22, 17_000_000)
    yield c
    c.close()


def test_rmat20_full(big_ctx):
    g = synth.config_graph("rmat20")
    d, p, neg = run(big_ctx, g, validate=False)
    d_ref, neg_ref, _, _ = oracle.bf_fifo(g)
    assert not neg and not neg_ref
    assert np.array_equal(d, d_ref)
    assert np.array_equal(p, oracle.pred(g, d_ref))
    print("[sssp] rmat20 stats", big_ctx.stats(), flush=True)


# Launch shapes of the autotuner's family (workgroup count, queue segments,
# row chunk, ticket batch, broker policy); the bench runs one of them.
RMAT_SHAPES = [
    None,
    {"wg_count": 192, "segments": 2},
    {"wg_count": 256, "segments": 4},
    {"wg_count": 256, "segments": 4, "ticket_batch": 2},
    {"wg_count": 256, "ticket_batch": 4},
    {"wg_count": 128, "segments": 2, "row_chunk": 64},
    {"wg_count": 216, "segments": 2, "row_chunk": 256},
    {"wg_count": 384, "segments": 8, "ticket_batch": 2},
    {"wg_count": 96, "segments": 1, "ticket_batch": 4},
    {"wg_count": 192, "segments": 2, "flags": pkg.BQ_F_BWD},
]


@pytest.fixture(scope="module")
def rmat20():
    g = synth.config_graph("rmat20")
    rec = goldens.load("rmat20")
    assert goldens.graph_digest(g) == rec["graph_sha256"], "generator output changed"
    return g, _dev(g), rec


@pytest.mark.parametrize("launch", RMAT_SHAPES, ids=lambda x: json.dumps(x))
def test_rmat20_golden_shapes(big_ctx, rmat20, launch):
    """RMAT-20 at full size in every shape the autotuner may pick: the
    stored result (oracle, certified by the Johnson closed form), byte for
    byte."""
    g, (off, col, w), rec = rmat20
    print(f"[sssp] rmat20 golden launch={launch}", flush=True)
    dist, pred, neg = big_ctx.solve(off, col, w, g.src, launch=launch)
    assert not neg
    goldens.check(rec, dist.cpu().numpy(), pred.cpu().numpy(), f"rmat20 {launch}")


def test_rmat20_autotuned_shape(big_ctx, rmat20):
    """The shape the autotuner picks on this machine, as the benchmark times it."""
    g, (off, col, w), rec = rmat20
    launch, ms = big_ctx.autotune(off, col, w, g.src, reps=3)
    print(f"[sssp] rmat20 autotuned {launch} {ms:.3f} ms", flush=True)
    for _ in range(3):
        dist, pred, neg = big_ctx.solve(off, col, w, g.src, launch=launch)
        assert not neg
        goldens.check(rec, dist.cpu().numpy(), pred.cpu().numpy(), f"rmat20 {launch}")


def test_road2048_full(big_ctx):
    rec = goldens.load("road2048")
    g = synth.config_graph("road2048")
    assert goldens.graph_digest(g) == rec["graph_sha256"], "generator output changed"
    d, p, neg = run(big_ctx, g, validate=False)
    print("[sssp] road2048 stats", big_ctx.stats(), flush=True)
    assert not neg
    goldens.check(rec, d, p, "road2048")


def test_road2048_planted_negative_cycle(big_ctx):
    g = synth.config_graph("road2048_negcycle")
    assert goldens.load("road2048_negcycle")["neg_cycle"]
    d, p, neg = run(big_ctx, g, validate=False)
    print("[sssp] road2048_negcycle stats", big_ctx.stats(), flush=True)
    assert neg


def test_road2048_negative_cycle_marks_everything(big_ctx):
    """The mesh has edges both ways, so the planted cycle reaches every
    vertex: with marking, every distance is minus infinity (a property that
    holds at any size; the oracle's n rounds are out of reach here)."""
    g = synth.config_graph("road2048_negcycle")
    off, col, w = _dev(g)
    dist, pred, neg = big_ctx.solve(off, col, w, g.src, neg_inf=True)
    print("[sssp] road2048_negcycle marking stats", big_ctx.stats(), flush=True)
    assert neg
    assert bool((dist == np.iinfo(np.int64).min).all()) and bool((pred == -1).all())


# ---------------------------------------------------------------------------
# watchdog: a wait limit far below the solve time
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("launch", [{}, {"segments": 1, "ticket_batch": 4},
                                    {"flags": pkg.BQ_F_BWD, "wg_count": 64}])
def test_watchdog_fires_then_context_recovers(ctx, launch):
    """timeout_us = 1: the solve (milliseconds on this 256 x 256 mesh) runs
    past its deadline of ten wait limits, so every wave leaves through the
    kernel's own bounded checks and the call returns BQ_ETIMEOUT. The context
    rebuilds its queue on the next call, which must be exact."""
    g = synth.road(256, plant_cycle=False, seed=8970)
    off, col, w = _dev(g)
    print(f"[sssp] watchdog launch={launch}", flush=True)
    with pytest.raises(pkg.BQError) as ei:
        ctx.solve(off, col, w, g.src, launch=dict(launch, timeout_us=1))
    assert ei.value.status == pkg.BQ_ETIMEOUT
    check(ctx, g, launch=launch or None, method="fifo")
    # a second expiry right after a clean solve, then a clean solve again
    with pytest.raises(pkg.BQError) as ei:
        ctx.solve(off, col, w, g.src, launch={"timeout_us": 1})
    assert ei.value.status == pkg.BQ_ETIMEOUT
    check(ctx, g, method="fifo")


# ---------------------------------------------------------------------------
# near / far buckets (bucket_width > 0): a different order of work, the same
# results
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("bw", [1, 4, 64])
@pytest.mark.parametrize("seed", range(8))
def test_buckets_random_negative(ctx, bw, seed):
    rng = np.random.default_rng(5000 + seed)
    n = int(rng.integers(1, 80))
    m = int(rng.integers(0, 6 * n + 1))
    g = synth.random_small(n, m, -6, 30, seed=5100 + seed)
    check(ctx, g, src=int(rng.integers(0, n)), launch={"bucket_width": bw})


@pytest.mark.parametrize("bw", [1, 8])
@pytest.mark.parametrize("launch", [{}, {"segments": 1}, {"ticket_batch": 4, "wg_count": 32},
                                    {"flags": pkg.BQ_F_BWD, "segments": 8, "wg_count": 64}],
                         ids=lambda x: json.dumps(x))
def test_buckets_meshes_and_hubs(ctx, bw, launch):
    L = dict(launch, bucket_width=bw)
    for g in (synth.road(128, plant_cycle=False, seed=5200), synth.rmat(14, 16, seed=5201),
              synth.potential_random(20000, 160000, seed=5202)):
        check(ctx, g, launch=L, method="fifo")


@pytest.mark.parametrize("cyc_len", [1, 3, 50])
def test_buckets_negative_cycles_and_marking(ctx, cyc_len):
    g = synth.road(48, plant_cycle=True, seed=5300 + cyc_len)
    d, p, neg = run(ctx, g, launch={"bucket_width": 4})
    assert neg
    assert check_neg_inf(ctx, g, launch={"bucket_width": 4})
    rng = np.random.default_rng(cyc_len)
    n = 400
    src = rng.integers(0, n, 1600)
    dst = rng.integers(0, n, 1600)
    w = rng.integers(1, 50, 1600)
    cyc = np.arange(100, 100 + cyc_len)
    s2 = np.concatenate([src, cyc, [0]])
    d2 = np.concatenate([dst, np.roll(cyc, -1), [100]])
    w2 = np.concatenate([w, np.full(cyc_len, -1), [5]])
    g2 = synth.csr_from_edges(n, s2, d2, w2, name="cyc", source=0, meta={})
    check(ctx, g2, launch={"bucket_width": 1})
    assert check_neg_inf(ctx, g2, launch={"bucket_width": 1})


def test_road2048_buckets_golden(big_ctx):
    rec = goldens.load("road2048")
    g = synth.config_graph("road2048")
    off, col, w = _dev(g)
    for L in ({"bucket_width": 4}, {"bucket_width": 16, "wg_count": 1024, "segments": 8}):
        dist, pred, neg = big_ctx.solve(off, col, w, g.src, launch=L)
        print(f"[sssp] road2048 buckets {L} stats {big_ctx.stats()}", flush=True)
        assert not neg
        goldens.check(rec, dist.cpu().numpy(), pred.cpu().numpy(), f"road2048 {L}")
    g = synth.config_graph("road2048_negcycle")
    off, col, w = _dev(g)
    assert big_ctx.solve(off, col, w, g.src, launch={"bucket_width": 4})[2]


# Both scan widths: graphs under 6 edges per vertex on average run the
# short-row kernel (4 edges per lane per step), the others the default one
# (8). The same families on both sides of that line, with hubs split into
# chunks, negative weights and every ticket batch.
@pytest.mark.parametrize("deg", [2, 5, 6, 12])
@pytest.mark.parametrize("launch", [None, {"ticket_batch": 2, "segments": 2},
                                    {"ticket_batch": 4, "wg_count": 16}, {"bucket_width": 4}])
def test_both_scan_widths(ctx, deg, launch):
    n = 3000
    g = synth.potential_random(n, deg * n, seed=500 + deg)
    check(ctx, g, launch=launch)
    h = synth.rmat(12, edge_factor=max(1, deg), seed=600 + deg)
    check(ctx, h, launch=launch)
