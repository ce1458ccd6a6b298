"""GPU parity of the round form over an edge queue (sssp_bf_rounds through
the C ABI) against the CPU oracle's rounds: distances, predecessors and the
negative-cycle flag must be bit-identical. The number of rounds the GPU needs
depends on the order in which concurrent waves relax edges, so it is checked
against its bounds, not compared."""
import json
import os

import numpy as np
import pytest

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
    c = pkg.RoundsContext(1 << 16, 1 << 20)
    yield c
    c.close()


def run(ctx, g, src=None, launch=None, validate=True):
    src = g.src if src is None else src
    print(f"[rounds] {g.name} n={g.n} m={g.m} src={src} launch={launch}", flush=True)
    off, col, w = _dev(g)
    dist, pred, neg = ctx.solve(off, col, w, src, launch=launch, validate=validate)
    torch.cuda.synchronize()
    return dist.cpu().numpy(), pred.cpu().numpy(), neg


def check(ctx, g, src=None, launch=None, method="rounds"):
    src = g.src if src is None else src
    d, p, neg = run(ctx, g, src, launch)
    d_ref, p_ref, neg_ref = oracle.sssp(g, src, method=method)
    assert neg == neg_ref
    st = ctx.stats()
    assert 1 <= st["rounds"] <= g.n
    assert st["relaxations"] == st["rounds"] * g.m
    if not neg_ref:
        bad = np.nonzero(d != d_ref)[0]
        assert bad.size == 0, f"dist differs at {bad[:5]}: {d[bad[:5]]} vs {d_ref[bad[:5]]}"
        bad = np.nonzero(p != p_ref)[0]
        assert bad.size == 0, f"pred differs at {bad[:5]}: {p[bad[:5]]} vs {p_ref[bad[:5]]}"
        # every reached vertex but the source was lowered at least once
        assert st["changes"] >= int((d_ref != oracle.INF).sum()) - 1
    else:
        assert st["rounds"] == g.n
    return d, p, neg


def test_grid64(ctx):
    check(ctx, synth.grid64())


@pytest.mark.parametrize("seed", range(40))
def test_random_small_negative(ctx, seed):
    rng = np.random.default_rng(7000 + seed)
    n = int(rng.integers(1, 60))
    m = int(rng.integers(0, 5 * n + 1))
    g = synth.random_small(n, m, -6, 30, seed=7100 + seed)
    check(ctx, g, src=int(rng.integers(0, n)))


@pytest.mark.parametrize("seed", range(6))
def test_potential_shifted_medium(ctx, seed):
    g = synth.potential_random(3000 + 700 * seed, 20000 + 5000 * seed, seed=7200 + seed)
    check(ctx, g, method="fifo")


@pytest.mark.parametrize("launch", [
    {"wg_size": 64, "wg_count": 1}, {"wg_size": 128, "wg_count": 3}, {"wg_size": 512},
    {"wg_size": 1024, "ticket_batch": 1}, {"ticket_batch": 64}, {"ticket_batch": 3, "wg_count": 7},
    {"flags": pkg.BQ_F_BWD}, {"flags": pkg.BQ_F_BWD, "ticket_batch": 1, "wg_count": 2},
])
def test_launch_shapes(ctx, launch):
    g = synth.potential_random(20000, 160000, seed=7300)
    check(ctx, g, launch=launch, method="fifo")


def test_single_vertex_and_no_edges(ctx):
    g = synth.csr_from_edges(1, [], [], [])
    d, p, neg = run(ctx, g)
    assert d.tolist() == [0] and p.tolist() == [-1] and not neg
    assert ctx.stats()["rounds"] == 1
    g = synth.csr_from_edges(5, [], [], [], source=3)
    d, p, neg = run(ctx, g)
    assert d.tolist() == [oracle.INF] * 3 + [0, oracle.INF] and not neg


def test_negative_self_loop_on_one_vertex(ctx):
    g = synth.csr_from_edges(1, [0], [0], [-1])
    assert run(ctx, g)[2]
    assert ctx.stats()["rounds"] == 1


def test_self_loops_multi_edges_zero_cycles(ctx):
    g = synth.csr_from_edges(4, [0, 0, 0, 1, 2, 1, 3, 3], [1, 1, 2, 2, 1, 1, 3, 0],
                             [9, 2, 5, 3, -3, 0, 4, 1], source=0)
    check(ctx, g)


@pytest.mark.parametrize("cyc_len", [1, 3, 40])
@pytest.mark.parametrize("reachable", [True, False])
def test_planted_negative_cycles(ctx, cyc_len, reachable):
    base = synth.potential_random(1500, 12000, seed=7400 + cyc_len + 31 * reachable)
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
    check(ctx, g)


def test_road_planted_cycle_then_reuse(ctx):
    g = synth.road(64, plant_cycle=True, seed=7500)
    check(ctx, g)
    check(ctx, synth.road(64, plant_cycle=False, seed=7500), method="fifo")


def test_range_error(ctx):
    rng = np.random.default_rng(3)
    n = 50000
    s = rng.integers(0, n, size=50000)
    t = rng.integers(0, n, size=50000)
    w = rng.integers(1, 10, size=50000)
    w[17] = 2**31 - 1
    g = synth.csr_from_edges(n, s, t, w, source=0)
    off, col, wt = _dev(g)
    with pytest.raises(pkg.BQError) as e:
        ctx.solve(off, col, wt, 0)
    assert e.value.status == pkg.BQ_ERANGE
    check(ctx, synth.grid64())


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
    for bad_launch in ({"wg_size": 96}, {"ticket_batch": 65}):
        with pytest.raises(pkg.BQError):
            ctx.solve(off, col, w, 0, launch=bad_launch)
    check(ctx, g)


@pytest.mark.parametrize("launch", [{}, {"flags": pkg.BQ_F_BWD, "ticket_batch": 4}])
def test_watchdog_fires_then_context_recovers(ctx, launch):
    """timeout_us = 1: the rounds of this 256 x 256 mesh (hundreds of them,
    milliseconds in all) run past the host's deadline of ten wait limits, and
    waves that wait longer than the limit give up inside the kernel, so the
    call returns BQ_ETIMEOUT after every issued round has ended through its
    own bounded waits. The next call on the same context must be exact."""
    g = synth.road(256, plant_cycle=False, seed=8971)
    off, col, w = _dev(g)
    print(f"[rounds] watchdog launch={launch}", flush=True)
    with pytest.raises(pkg.BQError) as ei:
        ctx.solve(off, col, w, g.src, launch=dict(launch, timeout_us=1))
    assert ei.value.status == pkg.BQ_ETIMEOUT
    check(ctx, g, launch=launch or None)


def test_repeated_solves_are_identical(ctx):
    g = synth.rmat(14, 16, seed=3)
    first = run(ctx, g)
    for _ in range(3):
        again = run(ctx, g)
        assert np.array_equal(first[0], again[0]) and np.array_equal(first[1], again[1])
    d_ref, p_ref, _ = oracle.sssp(g, method="rounds")
    assert np.array_equal(first[0], d_ref) and np.array_equal(first[1], p_ref)


def test_agrees_with_queue_solver(ctx):
    """The two GPU forms (vertex queue, edge-queue rounds) on the same input."""
    g = synth.potential_random(30000, 240000, seed=7600)
    off, col, w = _dev(g)
    d1, p1, n1 = ctx.solve(off, col, w, g.src)
    qctx = pkg.SsspContext(g.n, g.m)
    d2, p2, n2 = qctx.solve(off, col, w, g.src)
    qctx.close()
    assert not n1 and not n2
    assert torch.equal(d1, d2) and torch.equal(p1, p2)


# ---------------------------------------------------------------------------
# minus-infinity marking (BQ_F_NEGINF)
# ---------------------------------------------------------------------------

def check_neg_inf(ctx, g, src=None, launch=None):
    src = g.src if src is None else src
    print(f"[rounds] neg_inf {g.name} n={g.n} m={g.m} src={src}", flush=True)
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
    rng = np.random.default_rng(7700 + seed)
    n = int(rng.integers(1, 60))
    g = synth.random_small(n, int(rng.integers(0, 4 * n + 1)), -6, 30, seed=7800 + seed)
    check_neg_inf(ctx, g, src=int(rng.integers(0, n)))


@pytest.mark.parametrize("cyc_len", [1, 2, 7])
def test_neg_inf_cycle_with_tail(ctx, cyc_len):
    """A negative cycle hanging off a potential-shifted graph, with a tree
    of vertices below it (all minus infinity) and the rest exact."""
    base = synth.potential_random(1200, 9000, seed=7900 + cyc_len)
    s, t, w = synth.edges_of(base)
    n0 = base.n
    cyc = np.arange(n0, n0 + cyc_len)
    cw = np.full(cyc_len, 4, dtype=np.int64)
    cw[-1] = -(4 * (cyc_len - 1)) - 1
    tail = np.arange(n0 + cyc_len, n0 + cyc_len + 50)
    ts = np.concatenate([[cyc[0]], tail[:-1]])
    extra_s = np.concatenate([[17], cyc, ts])
    extra_t = np.concatenate([[cyc[0]], np.roll(cyc, -1), tail])
    extra_w = np.concatenate([[5], cw, np.full(50, 2)])
    g = synth.csr_from_edges(n0 + cyc_len + 50, np.concatenate([s, extra_s]),
                             np.concatenate([t, extra_t]), np.concatenate([w, extra_w]),
                             source=0)
    assert check_neg_inf(ctx, g)
    # the cycle and the tail below it are minus infinity, the rest exact
    assert int((oracle.neg_inf(g)[0] == oracle.NEG_INF).sum()) == cyc_len + 50


def test_neg_inf_road_and_no_cycle(ctx):
    assert check_neg_inf(ctx, synth.road(48, plant_cycle=True, seed=7950))
    assert not check_neg_inf(ctx, synth.road(48, plant_cycle=False, seed=7950))
    assert not check_neg_inf(ctx, synth.potential_random(5000, 40000, seed=7951))


# ---------------------------------------------------------------------------
# full-size workloads
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def big_ctx():
    c = pkg.RoundsContext(1 << 22, 17_000_000)
    yield c
    c.close()


def test_rmat20_full(big_ctx):
    g = synth.config_graph("rmat20")
    d, p, neg = run(big_ctx, g, validate=False)
    print("[rounds] rmat20 stats", big_ctx.stats(), flush=True)
    d_ref, neg_ref, _ = oracle.bf_rounds(g)
    assert not neg and not neg_ref
    assert np.array_equal(d, d_ref)
    assert np.array_equal(p, oracle.pred(g, d_ref))


def test_road2048_full(big_ctx):
    import hashlib
    rec = json.load(open(os.path.join(HERE, "golden", "road2048.json")))["road2048"]
    g = synth.config_graph("road2048")
    d, p, neg = run(big_ctx, g, validate=False)
    print("[rounds] road2048 stats", big_ctx.stats(), flush=True)
    assert not neg
    idx = np.array(rec["sample_idx"])
    assert np.array_equal(d[idx], np.array(rec["sample_dist"]))
    assert hashlib.sha256(np.ascontiguousarray(d).tobytes()).hexdigest() == rec["dist_sha256"]
    assert hashlib.sha256(np.ascontiguousarray(p).tobytes()).hexdigest() == rec["pred_sha256"]
