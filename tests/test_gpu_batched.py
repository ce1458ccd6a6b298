"""GPU parity of the batched form (sssp_bf_batched through the C ABI): every
query in a batch must get exactly the oracle's answer (and so the answer
sssp_bf gives it alone), whatever else shares the launch."""
import numpy as np
import pytest

import goldens
import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pkg = pytest.importorskip("paper_2608_21826_amd")

DEV = torch.device("cuda:0")


def upload(g):
    return (torch.from_numpy(g.offsets).to(DEV), torch.from_numpy(g.cols).to(DEV),
            torch.from_numpy(g.w).to(DEV))


def make_queries(graphs_srcs):
    qs, keep = [], []
    for g, src, t in graphs_srcs:
        off, col, w = t
        dist = torch.empty(g.n, dtype=torch.int64, device=DEV)
        pred = torch.empty(g.n, dtype=torch.int32, device=DEV)
        qs.append((off, col, w, src, dist, pred))
        keep.append((g, src))
    return qs, keep


def check_all(qs, keep, neg, method="fifo"):
    torch.cuda.synchronize()
    for (off, col, w, src, dist, pred), (g, s), flag in zip(qs, keep, neg):
        d_ref, p_ref, neg_ref = oracle.sssp(g, s, method=method)
        assert flag == neg_ref, f"{g.name} src={s}: flag {flag} vs {neg_ref}"
        if not neg_ref:
            d = dist.cpu().numpy()
            p = pred.cpu().numpy()
            assert np.array_equal(d, d_ref), f"{g.name} src={s}: dist differs"
            assert np.array_equal(p, p_ref), f"{g.name} src={s}: pred differs"


@pytest.fixture(scope="module")
def batch():
    b = pkg.SsspBatch(64, 4_000_000, 40_000_000)
    yield b
    b.close()


def mixed_graphs(seed, k):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(k):
        kind = i % 4
        if kind == 0:
            g = synth.potential_random(int(rng.integers(1, 3000)), int(rng.integers(0, 20000)),
                                       seed=seed * 100 + i)
        elif kind == 1:
            n = int(rng.integers(1, 60))
            g = synth.random_small(n, int(rng.integers(0, 5 * n + 1)), 0, 20, seed=seed * 100 + i)
        elif kind == 2:
            g = synth.erdos_renyi(int(rng.integers(1000, 30000)), 8, seed=seed * 100 + i)
        else:
            g = synth.rmat(int(rng.integers(8, 13)), 16, seed=seed * 100 + i)
        src = int(rng.integers(0, g.n))
        out.append((g, src, upload(g)))
    return out


@pytest.mark.parametrize("seed", range(4))
def test_mixed_batch_matches_oracle(batch, seed):
    print(f"[batched] mixed seed={seed}", flush=True)
    qs, keep = make_queries(mixed_graphs(seed, 24))
    neg = batch.solve(qs)
    check_all(qs, keep, neg)
    st = batch.stats()
    assert st["relaxations"] > 0


@pytest.mark.parametrize("launch", [
    {"wg_count": 1}, {"wg_count": 3}, {"wg_count": 7, "ticket_batch": 2},
    {"row_chunk": 256}, {"queue_scale": 1}, {"row_chunk": 64, "wg_count": 16},
    {"flags": 8, "wg_count": 5}, {"flags": 8, "ticket_batch": 4},
    {"wg_count": 9}, {"wg_count": 12, "ticket_batch": 2},
])
def test_launch_shapes(batch, launch):
    print(f"[batched] launch {launch}", flush=True)
    qs, keep = make_queries(mixed_graphs(11, 12))
    neg = batch.solve(qs, launch=launch)
    check_all(qs, keep, neg)


def test_negative_cycle_in_the_mix(batch):
    """One query with a planted cycle; it alone is flagged and the others are
    exact. The next batch (same context) is clean."""
    items = mixed_graphs(5, 9)
    gneg = synth.road(40, plant_cycle=True, seed=99)
    items.insert(4, (gneg, 0, upload(gneg)))
    qs, keep = make_queries(items)
    neg = batch.solve(qs)
    assert neg[4] and sum(neg) == 1
    check_all(qs, keep, neg)
    qs2, keep2 = make_queries(mixed_graphs(6, 10))
    check_all(qs2, keep2, batch.solve(qs2))


def test_negative_cycle_marking_in_the_mix(batch):
    """With BQ_F_NEGINF the query with a cycle gets minus infinity where the
    cycle reaches and exact values elsewhere; the others are exact."""
    items = mixed_graphs(7, 9)
    base = synth.potential_random(1200, 9000, seed=61)
    s, t, w = synth.edges_of(base)
    n0 = base.n
    gneg = synth.csr_from_edges(n0 + 3, np.concatenate([s, [17, n0, n0 + 1, n0 + 2]]),
                                np.concatenate([t, [n0, n0 + 1, n0 + 2, n0]]),
                                np.concatenate([w, [5, 2, 2, -5]]), source=0)
    items.insert(3, (gneg, 0, upload(gneg)))
    qs, keep = make_queries(items)
    neg = batch.solve(qs, launch={"flags": pkg.BQ_F_NEGINF})
    assert neg[3] and sum(neg) == 1
    torch.cuda.synchronize()
    d_ref, p_ref, _ = oracle.neg_inf(gneg, 0)
    assert np.array_equal(qs[3][4].cpu().numpy(), d_ref)
    assert np.array_equal(qs[3][5].cpu().numpy(), p_ref)
    check_all(qs[:3] + qs[4:], keep[:3] + keep[4:], neg[:3] + neg[4:])


def test_large_queries_get_segments(batch):
    """Queries large enough to feed 16+ workgroups get up to 8 queue segments
    when the slot arena has room; results stay exact, alone and mixed with
    small queries, with and without a planted negative cycle (marking mode)."""
    big = synth.rmat(18, 16, seed=41)
    road = synth.road(600, plant_cycle=False, seed=42)
    items = [(big, big.src, upload(big))]
    qs, keep = make_queries(items)
    check_all(qs, keep, batch.solve(qs))
    items += [(road, 0, upload(road))] + mixed_graphs(43, 6)
    qs, keep = make_queries(items)
    check_all(qs, keep, batch.solve(qs, launch={"ticket_batch": 2}), method="fifo")
    roadneg = synth.road(300, plant_cycle=True, seed=44)
    qs, keep = make_queries([(roadneg, 0, upload(roadneg)), (big, big.src, upload(big))])
    neg = batch.solve(qs, launch={"flags": pkg.BQ_F_NEGINF})
    assert neg == [True, False]
    torch.cuda.synchronize()
    assert bool((qs[0][4] == np.iinfo(np.int64).min).all())
    check_all(qs[1:], keep[1:], neg[1:], method="fifo")


def test_shared_graph_many_sources(batch):
    g = synth.rmat(14, 16, seed=4)
    t = upload(g)
    srcs = synth.random_sources(g, 32, seed=8)
    qs, keep = make_queries([(g, int(s), t) for s in srcs])
    neg = batch.solve(qs)
    check_all(qs, keep, neg)


def test_graph_replay(batch):
    """The launch sequence as a hipGraph, replayed with eager device work and
    synchronizations in between; every replay must equal the eager result."""
    qs, keep = make_queries(mixed_graphs(21, 16))
    neg0 = batch.solve(qs)
    ref = [(q[4].clone(), q[5].clone()) for q in qs]
    for rep in range(4):
        for q in qs:
            q[4].fill_(-7)
            q[5].fill_(-7)
        junk = torch.randn(1 << 16, device=DEV).sum()
        torch.cuda.synchronize()
        neg = batch.solve(qs, graph=True)
        assert neg == neg0
        for (d0, p0), q in zip(ref, qs):
            assert torch.equal(d0, q[4]) and torch.equal(p0, q[5])
        del junk
    check_all(qs, keep, neg0)


def test_alone_equals_in_mix(batch):
    items = mixed_graphs(31, 10)
    qs, keep = make_queries(items)
    batch.solve(qs)
    ctx = pkg.SsspContext(200_000, 2_000_000)
    for (off, col, w, src, dist, pred), (g, s) in zip(qs, keep):
        d1, p1, n1 = ctx.solve(off, col, w, s)
        assert torch.equal(d1, dist) and torch.equal(p1, pred)
    ctx.close()


# ---------------------------------------------------------------------------
# the measured batched workloads
# ---------------------------------------------------------------------------

def test_er256_full():
    """256 Erdos-Renyi queries, sizes log-uniform 1k..200k, degree 8: every
    answer against the stored oracle results (certified by the Johnson closed
    form), byte for byte."""
    graphs = synth.er_batch(256)
    rec = goldens.load("er256")["queries"]
    assert len(rec) == len(graphs)
    for g, r in zip(graphs, rec):
        assert goldens.graph_digest(g) == r["graph_sha256"] and g.src == r["src"], g.name
    tn = sum(g.n for g in graphs)
    tm = sum(g.m for g in graphs)
    print(f"[batched] er256 total n={tn} m={tm}", flush=True)
    b = pkg.SsspBatch(256, tn, tm)
    qs, keep = make_queries([(g, g.src, upload(g)) for g in graphs])
    neg = b.solve(qs, graph=True)
    print(f"[batched] er256 stats {b.stats()}", flush=True)
    torch.cuda.synchronize()
    assert not any(neg)
    for (off, col, w, src, dist, pred), (g, s), r in zip(qs, keep, rec):
        goldens.check(r, dist.cpu().numpy(), pred.cpu().numpy(), f"{g.name} src={s}")
    b.close()


def check_rmat20_x64(qs, neg):
    """All 64 queries against the stored per-source results (oracle,
    certified by the Johnson closed form)."""
    rec = goldens.load("rmat20_x64_sources")
    assert len(rec["queries"]) == len(qs) == len(neg)
    torch.cuda.synchronize()
    for (off, col, w, src, dist, pred), r, flag in zip(qs, rec["queries"], neg):
        assert src == r["src"] and not flag
        goldens.check(r, dist.cpu().numpy(), pred.cpu().numpy(), f"rmat20 src={src}")


@pytest.fixture(scope="module")
def rmat20_x64():
    g = synth.rmat(20)
    rec = goldens.load("rmat20_x64_sources")
    assert goldens.graph_digest(g) == rec["graph_sha256"], "generator output changed"
    t = upload(g)
    srcs = synth.random_sources(g, 64, seed=rec["sources_seed"])
    b = pkg.SsspBatch(64, 64 * g.n, 64 * g.m)
    qs, keep = make_queries([(g, int(s), t) for s in srcs])
    yield g, b, qs
    b.close()


def test_rmat20_64_sources(rmat20_x64):
    g, b, qs = rmat20_x64
    neg = b.solve(qs, graph=True)
    print(f"[batched] rmat20x64 stats {b.stats()}", flush=True)
    check_rmat20_x64(qs, neg)
    # the oracle itself on two of them
    sample = [0, 37]
    check_all([qs[i] for i in sample], [(g, qs[i][3]) for i in sample], [neg[i] for i in sample])


@pytest.mark.parametrize("launch", [{"wg_count": 256, "ticket_batch": 1},
                                    {"wg_count": 512, "ticket_batch": 2, "row_chunk": 256},
                                    {"wg_count": 1024, "ticket_batch": 1, "queue_scale": 1}],
                         ids=str)
def test_rmat20_64_sources_shapes(rmat20_x64, launch):
    """The batched launch shapes the autotuner picks from, all 64 answers
    exact in each; the hipGraph is replayed twice."""
    g, b, qs = rmat20_x64
    for _ in range(2):
        for q in qs:
            q[4].fill_(-7)
        neg = b.solve(qs, launch=launch, graph=True)
        check_rmat20_x64(qs, neg)


def test_rmat20_64_sources_autotuned(rmat20_x64):
    g, b, qs = rmat20_x64
    launch, ms = b.autotune(qs)
    print(f"[batched] rmat20x64 autotuned {launch} {ms:.3f} ms", flush=True)
    check_rmat20_x64(qs, b.solve(qs, launch=launch, graph=True))


def test_batched_watchdog_then_recovery(batch):
    """timeout_us = 1 on a batch of road meshes: every query runs past its
    deadline, the kernels leave through their own bounded checks and the
    call returns BQ_ETIMEOUT; the next call on the same workspace is exact."""
    items = []
    for i in range(6):
        g = synth.road(96 + 16 * i, plant_cycle=False, seed=8980 + i)
        items.append((g, 0, upload(g)))
    qs, keep = make_queries(items)
    with pytest.raises(pkg.BQError) as ei:
        batch.solve(qs, launch={"timeout_us": 1})
    assert ei.value.status == pkg.BQ_ETIMEOUT
    check_all(qs, keep, batch.solve(qs))
    with pytest.raises(pkg.BQError) as ei:
        batch.solve(qs, launch={"timeout_us": 1}, graph=True)
    assert ei.value.status == pkg.BQ_ETIMEOUT
    check_all(qs, keep, batch.solve(qs, graph=True))


@pytest.mark.parametrize("wgs", [8, 24, 64])
def test_many_small_queries_on_few_workgroups(batch, wgs):
    """More queries than workgroups: each XCD's claim list holds several
    queries, later ones are claimed as earlier ones finish, and workgroups
    whose list is used up help elsewhere; every answer stays exact."""
    print(f"[batched] 64 small queries, wg_count={wgs}", flush=True)
    items = []
    for i in range(64):
        g = (synth.erdos_renyi(500 + 97 * i, 8, seed=700 + i) if i % 2 == 0
             else synth.potential_random(200 + 31 * i, 6 * (200 + 31 * i), seed=700 + i))
        items.append((g, int(i * 7919 % g.n), upload(g)))
    qs, keep = make_queries(items)
    check_all(qs, keep, batch.solve(qs, launch={"wg_count": wgs}))


@pytest.mark.parametrize("flags", [0, pkg.BQ_F_NOREMAP], ids=["remapped", "vertex_order"])
def test_shared_graphs_mixed_with_own(batch, flags):
    """Queries that share a graph (several per graph: RMAT with hubs and
    split rows, a mesh, a graph with a planted negative cycle) next to
    queries on graphs of their own. Shared graphs get the degree-class key
    layout unless BQ_F_NOREMAP; every answer, flag and predecessor must be
    the oracle's either way."""
    rm = synth.rmat(14, 16, seed=31)
    mesh = synth.road(40, plant_cycle=False, seed=32)
    cyc = synth.road(24, plant_cycle=True, seed=33)
    pr = synth.potential_random(4000, 30000, seed=34)
    t_rm, t_mesh, t_cyc, t_pr = upload(rm), upload(mesh), upload(cyc), upload(pr)
    items = [(rm, int(s), t_rm) for s in synth.random_sources(rm, 5, seed=35)]
    items += [(mesh, int(s), t_mesh) for s in (0, 17, 1599)]
    items += [(cyc, int(s), t_cyc) for s in (0, 300)]
    items += [(pr, 11, t_pr), (pr, 2222, t_pr)]
    items += [(synth.erdos_renyi(3000 + 500 * i, 8, seed=36 + i), 1 + i, None) for i in range(4)]
    items = [(g, s, t if t is not None else upload(g)) for g, s, t in items]
    qs, keep = make_queries(items)
    print(f"[batched] shared graphs, flags={flags}", flush=True)
    for graph in (False, True):
        for q in qs:
            q[4].fill_(-3)
        check_all(qs, keep, batch.solve(qs, launch={"flags": flags}, graph=graph))


@pytest.mark.parametrize("flags", [0, pkg.BQ_F_NOREMAP], ids=["remapped", "vertex_order"])
def test_shared_graph_minus_infinity(batch, flags):
    """Marking mode on a shared graph with a reachable negative cycle: the
    minus-infinity vertices and the exact labels of the rest match the
    oracle for every query (the cycle search walks parents through the key
    layout)."""
    g = synth.road(32, plant_cycle=True, seed=41)
    t = upload(g)
    srcs = [0, 5, 517, 1023]
    qs, keep = make_queries([(g, s, t) for s in srcs])
    neg = batch.solve(qs, launch={"flags": flags | pkg.BQ_F_NEGINF})
    torch.cuda.synchronize()
    for (off, col, w, src, dist, pred), flag in zip(qs, neg):
        d_ref, p_ref, neg_ref = oracle.neg_inf(g, src)
        assert flag == neg_ref
        assert np.array_equal(dist.cpu().numpy(), d_ref)
        assert np.array_equal(pred.cpu().numpy(), p_ref)


@pytest.mark.parametrize("bw", [1, 4])
def test_batched_buckets(batch, bw):
    """Near / far buckets in the batched form: meshes, hubs, shared graphs,
    a reachable negative cycle and graphs of their own in one launch; every
    answer must be the oracle's."""
    mesh = synth.road(64, plant_cycle=False, seed=61)
    rm = synth.rmat(13, 16, seed=62)
    cyc = synth.road(20, plant_cycle=True, seed=63)
    t_mesh, t_rm = upload(mesh), upload(rm)
    items = [(mesh, int(s), t_mesh) for s in (0, 100, 4095)]
    items += [(rm, int(s), t_rm) for s in synth.random_sources(rm, 3, seed=64)]
    items += [(cyc, 0, upload(cyc)), (synth.road(90, seed=65), 7, None),
              (synth.potential_random(6000, 50000, seed=66), 5, None)]
    items = [(g, s, t if t is not None else upload(g)) for g, s, t in items]
    qs, keep = make_queries(items)
    for graph in (False, True):
        check_all(qs, keep, batch.solve(qs, launch={"bucket_width": bw}, graph=graph))
    # a lone large mesh with every queue segment
    big = synth.road(600, plant_cycle=False, seed=67)
    qs, keep = make_queries([(big, 0, upload(big))])
    check_all(qs, keep, batch.solve(qs, launch={"bucket_width": bw, "wg_count": 64}))
