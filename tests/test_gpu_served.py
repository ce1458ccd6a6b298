"""GPU checks of the served form (bq_server_run through the C ABI): with
requests arriving while others run, every response equals the oracle (the
same answer the query gets alone); launches overlap on several lanes;
admission by memory holds requests back without losing any."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pkg = pytest.importorskip("paper_2608_21826_amd")

DEV = torch.device("cuda:0")


def dev_csr(g):
    return (torch.from_numpy(g.offsets).to(DEV), torch.from_numpy(g.cols).to(DEV),
            torch.from_numpy(g.w).to(DEV))


def host_csr(g):
    return (torch.from_numpy(g.offsets).pin_memory(), torch.from_numpy(g.cols).pin_memory(),
            torch.from_numpy(g.w).pin_memory())


def build_trace(resident, uploads, count, mean_gap_us, seed, outputs=True):
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs, truth = [], []
    for i in range(count):
        t += rng.exponential(mean_gap_us)
        if rng.random() < 0.25 and uploads:
            g = uploads[int(rng.integers(0, len(uploads)))]
            src = int(rng.integers(0, g.n))
            r = {"arrival_us": t, "src": src, "upload": host_csr(g)}
        else:
            gid = int(rng.integers(0, len(resident)))
            g = resident[gid]
            src = int(rng.integers(0, g.n))
            r = {"arrival_us": t, "src": src, "graph": gid}
        if outputs:
            r["dist"] = torch.empty(g.n, dtype=torch.int64, device=DEV)
            r["pred"] = torch.empty(g.n, dtype=torch.int32, device=DEV)
        reqs.append(r)
        truth.append((g, src))
    return reqs, truth


def make_server(resident, lanes=3, arena=1 << 28, max_batch=16):
    mn = max(g.n for g in resident) * max_batch
    mm = max(g.m for g in resident) * max_batch
    srv = pkg.Server(lanes, max_batch, mn, mm, arena)
    for g in resident:
        srv.add_graph(*dev_csr(g))
    return srv


@pytest.fixture(scope="module")
def graphs():
    resident = [synth.grid64(), synth.rmat(14, 16, seed=3), synth.erdos_renyi(20000, 8, seed=4)]
    uploads = [synth.erdos_renyi(5000, 8, seed=5), synth.erdos_renyi(40000, 8, seed=6)]
    return resident, uploads


def check(reqs, truth, resp):
    torch.cuda.synchronize()
    for r, (g, src), x in zip(reqs, truth, resp):
        assert x["status"] == 0
        d_ref, p_ref, neg = oracle.sssp(g, src, method="fifo")
        assert bool(x["neg_cycle"]) == neg
        assert np.array_equal(r["dist"].cpu().numpy(), d_ref)
        assert np.array_equal(r["pred"].cpu().numpy(), p_ref)
        deg = np.diff(g.offsets)
        assert x["reached_edges"] == int(deg[d_ref != oracle.INF].sum())
        assert x["latency_us"] >= x["wait_us"] >= 0


@pytest.mark.parametrize("seed,gap", [(1, 50.0), (2, 300.0)])
def test_mix_matches_oracle(graphs, seed, gap):
    resident, uploads = graphs
    print(f"[served] seed={seed} gap={gap}", flush=True)
    srv = make_server(resident)
    reqs, truth = build_trace(resident, uploads, 60, gap, seed)
    resp, st = srv.run(reqs)
    print(f"[served] stats {st}", flush=True)
    check(reqs, truth, resp)
    assert st["launches"] < len(reqs)      # requests were batched together
    assert st["max_lanes_busy"] >= 2       # launches overlapped on the device
    srv.close()


def test_alone_equals_in_mix(graphs):
    resident, uploads = graphs
    srv = make_server(resident, lanes=1, max_batch=1)
    reqs, truth = build_trace(resident, uploads, 12, 10.0, 9)
    resp, st = srv.run(reqs)
    assert st["launches"] == 12
    check(reqs, truth, resp)
    srv.close()


def test_admission_by_memory(graphs):
    """An arena that holds about one uploaded graph at a time: uploads queue
    up behind each other, nothing is lost, the peak stays within it."""
    resident, uploads = graphs
    big = uploads[1]
    arena = int((big.n + 1) * 8 + big.m * 8 + 4096)
    srv = make_server(resident, lanes=3, arena=arena)
    reqs, truth = [], []
    for i in range(8):
        g = uploads[i % 2]
        src = int(i * 37 % g.n)
        reqs.append({"arrival_us": 10.0 * i, "src": src, "upload": host_csr(g),
                     "dist": torch.empty(g.n, dtype=torch.int64, device=DEV),
                     "pred": torch.empty(g.n, dtype=torch.int32, device=DEV)})
        truth.append((g, src))
    resp, st = srv.run(reqs)
    check(reqs, truth, resp)
    assert st["arena_peak_bytes"] <= arena
    srv.close()


def test_rejections(graphs):
    resident, uploads = graphs
    srv = make_server(resident, lanes=2)
    reqs = [{"arrival_us": 0.0, "src": 0, "graph": 99},
            {"arrival_us": 1.0, "src": 10**6, "graph": 0},
            {"arrival_us": 2.0, "src": 0, "graph": 1,
             "dist": torch.empty(resident[1].n, dtype=torch.int64, device=DEV),
             "pred": torch.empty(resident[1].n, dtype=torch.int32, device=DEV)}]
    resp, st = srv.run(reqs)
    assert resp[0]["status"] == pkg.BQ_EINVAL
    assert resp[1]["status"] == pkg.BQ_EINVAL
    assert resp[2]["status"] == 0
    check(reqs[2:], [(resident[1], 0)], resp[2:])
    srv.close()


def test_engine_outputs_without_caller_buffers(graphs):
    resident, uploads = graphs
    srv = make_server(resident, lanes=2)
    reqs, truth = build_trace(resident, uploads, 30, 40.0, 13, outputs=False)
    resp, st = srv.run(reqs)
    for x, (g, src) in zip(resp, truth):
        assert x["status"] == 0
        d_ref, _, _ = oracle.sssp(g, src, method="fifo")
        deg = np.diff(g.offsets)
        assert x["reached_edges"] == int(deg[d_ref != oracle.INF].sum())
    srv.close()


def test_large_requests_go_alone(graphs):
    """Requests with work for 64+ workgroups are launched one per launch (so
    they run with all queue segments); small ones are still batched, passing
    over the large ones; every answer is exact."""
    resident, uploads = graphs
    big = synth.rmat(19, 16, seed=12)  # (n + m/16) / 16384 = 64
    srv = make_server(resident + [big], lanes=2, max_batch=16)
    rng = np.random.default_rng(13)
    reqs, truth = [], []
    for i in range(14):
        gid = 3 if i % 3 == 0 else int(rng.integers(0, 3))
        g = (resident + [big])[gid]
        src = int(rng.integers(0, g.n))
        reqs.append({"arrival_us": 0.0, "src": src, "graph": gid,
                     "dist": torch.empty(g.n, dtype=torch.int64, device=DEV),
                     "pred": torch.empty(g.n, dtype=torch.int32, device=DEV)})
        truth.append((g, src))
    resp, st = srv.run(reqs)
    print(f"[served] size classes {st}", flush=True)
    check(reqs, truth, resp)
    n_big = sum(1 for r in reqs if r["graph"] == 3)
    # every large request had a launch of its own; the 9 small ones shared
    assert n_big + 1 <= st["launches"] < len(reqs)
    srv.close()


def test_reserved_small_lane(graphs):
    """With the last lane reserved, large requests queued in front of small
    ones run only on the other lane, small ones also start on the reserved
    lane, and every answer is still exact."""
    resident, uploads = graphs
    big = synth.rmat(19, 16, seed=12)  # (n + m/16) / 16384 = 64
    srv = make_server(resident + [big], lanes=2, max_batch=16)
    # k must leave at least one lane for large requests
    assert pkg.lib().bq_server_set_small_lanes(srv.handle, 2) == pkg.BQ_EINVAL
    assert pkg.lib().bq_server_set_small_lanes(srv.handle, -1) == pkg.BQ_EINVAL
    assert pkg.lib().bq_server_set_small_lanes(srv.handle, 1) == 0
    rng = np.random.default_rng(14)
    reqs, truth = [], []
    for i in range(12):
        gid = 3 if i < 3 else int(rng.integers(0, 3))
        g = (resident + [big])[gid]
        src = int(rng.integers(0, g.n))
        reqs.append({"arrival_us": 0.0, "src": src, "graph": gid,
                     "dist": torch.empty(g.n, dtype=torch.int64, device=DEV),
                     "pred": torch.empty(g.n, dtype=torch.int32, device=DEV)})
        truth.append((g, src))
    resp, st = srv.run(reqs)
    print(f"[served] reserved lane {st} lanes {[x['lane'] for x in resp]}", flush=True)
    check(reqs, truth, resp)
    assert all(x["lane"] == 0 for x, r in zip(resp, reqs) if r["graph"] == 3)
    assert any(x["lane"] == 1 for x, r in zip(resp, reqs) if r["graph"] != 3)
    assert all(x["lane"] in (0, 1) for x in resp)
    srv.close()


def test_lane_is_reported(graphs):
    """Every request that ran names the lane of its launch; a rejected one
    names none."""
    resident, uploads = graphs
    srv = make_server(resident, lanes=3)
    reqs, truth = build_trace(resident, uploads, 20, 40.0, 15)
    reqs.append({"arrival_us": reqs[-1]["arrival_us"] + 1.0, "src": 0, "graph": 99})
    resp, st = srv.run(reqs)
    check(reqs[:-1], truth, resp[:-1])
    assert all(0 <= x["lane"] < 3 for x in resp[:-1])
    assert resp[-1]["status"] == pkg.BQ_EINVAL and resp[-1]["lane"] == -1
    srv.close()


def test_full_size_mix_matches_goldens():
    """The benchmark's resident graphs at full size (RMAT-20, road2048 and
    an ER graph of 200k vertices) with Poisson arrivals and one-off ER
    uploads mixed in: RMAT-20 queries at the stored sources (its default
    source and eight of the 64 batched sources) and road2048 queries at its
    source must equal the stored results byte for byte in the mix, and the
    others the oracle."""
    import goldens
    rmat, road, er = (synth.config_graph(x) for x in ("rmat20", "road2048", "er200k"))
    r_rec, x_rec, d_rec = (goldens.load(x) for x in ("rmat20", "rmat20_x64_sources", "road2048"))
    assert goldens.graph_digest(rmat) == r_rec["graph_sha256"]
    assert goldens.graph_digest(road) == d_rec["graph_sha256"]
    uploads = [synth.erdos_renyi(nv, 8, seed=synth.SEED_BASE + 60 + i)
               for i, nv in enumerate((10_000, 60_000, 250_000))]
    resident = [rmat, road, er]
    srv = pkg.Server(4, 32, 8 * road.n, 8 * road.m, 2 << 30)
    for g in resident:
        srv.add_graph(*dev_csr(g))
    # road2048 requests (large, launched alone) with near / far buckets
    srv.set_graph_launch(1, {"bucket_width": 4, "wg_count": 64})
    with pytest.raises(pkg.BQError):
        srv.set_graph_launch(7, {"bucket_width": 1})
    plan = ([("g", 0, r_rec)] + [("g", 0, q) for q in x_rec["queries"][:8]] +
            [("g", 1, d_rec), ("g", 1, d_rec)] +
            [("g", 2, int(s)) for s in synth.random_sources(er, 4, seed=77)] +
            [("u", i, int(i * 7919 % uploads[i].n)) for i in range(3)])
    rng = np.random.default_rng(21)
    order = rng.permutation(len(plan))
    t = 0.0
    reqs, truth = [], []
    for k in order:
        kind, gi, what = plan[k]
        g = resident[gi] if kind == "g" else uploads[gi]
        src = what["src"] if isinstance(what, dict) else what
        t += rng.exponential(3000.0)
        r = {"arrival_us": t, "src": src,
             "dist": torch.empty(g.n, dtype=torch.int64, device=DEV),
             "pred": torch.empty(g.n, dtype=torch.int32, device=DEV)}
        if kind == "g":
            r["graph"] = gi
        else:
            r["upload"] = host_csr(g)
        reqs.append(r)
        truth.append((g, src, what))
    print(f"[served] full-size mix of {len(reqs)} requests", flush=True)
    resp, st = srv.run(reqs)
    print(f"[served] full-size mix {st}", flush=True)
    torch.cuda.synchronize()
    for r, (g, src, what), x in zip(reqs, truth, resp):
        assert x["status"] == 0 and not x["neg_cycle"]
        d, p = r["dist"].cpu().numpy(), r["pred"].cpu().numpy()
        if isinstance(what, dict):
            goldens.check(what, d, p, f"{g.name} src={src} in the mix")
            assert x["reached_edges"] == what["m_reached"]
        else:
            d_ref, p_ref, _ = oracle.sssp(g, src, method="fifo")
            assert np.array_equal(d, d_ref) and np.array_equal(p, p_ref)
    assert st["max_lanes_busy"] >= 2
    srv.close()
