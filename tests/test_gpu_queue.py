"""GPU checks of the Broker Queue through the C ABI.

- One wave = a sequential client: an interleaved sequence of bulk enqueues
  and dequeues must reproduce the sequential FIFO oracle exactly (values,
  order, Full/Empty counts), also with tiny capacities (many ticket rounds).
- Many waves: counts are fixed by the FIFO specification (min(n, free)),
  and the multiset is conserved.
- The Section IV "Global Mixed" run: position rule, conservation,
  per-producer FIFO and quiescent counters, from full position logs.
"""
import numpy as np
import pytest

import oracle
from oracle import history

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pkg = pytest.importorskip("paper_2608_21826_amd")

ONE_WAVE = {"wg_size": 64, "wg_count": 1}


@pytest.mark.parametrize("cap", [64, 128, 1024])
@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("b,flags", [(1, 0), (1, pkg.BQ_F_BWD), (4, 0)])
def test_one_wave_matches_sequential_fifo(cap, seed, b, flags):
    """One wave is a sequential client: Broker Queue and BWD alike reduce to
    the sequential FIFO, also with 64*b operations per ticket."""
    if 64 * b > cap:
        pytest.skip("chunk larger than the queue")
    print(f"[queue] one-wave cap={cap} seed={seed} b={b} flags={flags}", flush=True)
    ONE = dict(ONE_WAVE, ticket_batch=b, flags=flags)
    rng = np.random.default_rng(seed)
    q = pkg.Queue(cap)
    ops = []          # oracle op list
    got_ok, got_out = [], []
    nxt = 0
    for step in range(40):
        if rng.random() < 0.55:
            k = int(rng.integers(0, 3 * cap // 2))
            vals = np.arange(nxt, nxt + k, dtype=np.int32)
            nxt += k
            ok = q.enqueue(torch.from_numpy(vals).cuda(), launch=ONE) if k else 0
            ops.extend(vals.tolist())
            got_ok.append(("e", k, ok))
        else:
            k = int(rng.integers(0, 3 * cap // 2))
            out = q.dequeue(k, launch=ONE).cpu().numpy() if k else np.zeros(0, np.int32)
            ops.extend([-1] * k)
            got_ok.append(("d", k, out))
    res, out, size = oracle.fifo_run(cap, np.array(ops, dtype=np.int64))
    i = 0
    for kind, k, val in got_ok:
        r = res[i:i + k]
        if kind == "e":
            assert val == int(r.sum())
            # a one-wave bulk enqueue succeeds for a prefix of the array
            assert np.all(r[:val] == 1) and np.all(r[val:] == 0)
        else:
            exp = out[i:i + k][r == 1]
            assert np.array_equal(val, exp)
        i += k
    h, t, c = q.counters()
    assert t - h == size == c
    q.close()


def test_zero_size_calls_change_nothing():
    """n = 0 enqueues and dequeues (NULL data pointers) report 0 successes and
    leave the counters alone, on an empty and on a non-empty queue; a dequeue
    from the drained queue is Empty for every position and moves no head."""
    print("[queue] zero-size calls", flush=True)
    L = pkg.lib()
    q = pkg.Queue(64)
    ok = torch.full((1,), 7, dtype=torch.int64, device="cuda")

    def zero_calls():
        for f in (L.bq_enqueue, L.bq_dequeue):
            ok.fill_(7)
            st = f(q.handle, None, 0, pkg._ptr(ok), None, pkg._stream())
            assert st == pkg.BQ_OK and int(ok.item()) == 0

    zero_calls()
    assert q.counters() == (0, 0, 0)
    vals = torch.arange(100, 110, dtype=torch.int32, device="cuda")
    assert q.enqueue(vals, launch=ONE_WAVE) == 10
    zero_calls()
    assert q.counters() == (0, 10, 10)
    out = q.dequeue(20, launch=ONE_WAVE)
    assert torch.equal(out.cpu(), vals.cpu())
    assert q.counters() == (10, 10, 0)
    assert q.dequeue(5).numel() == 0
    assert q.counters() == (10, 10, 0)
    q.close()


@pytest.mark.parametrize("cap", [64, 4096, 1 << 16])
@pytest.mark.parametrize("bwd", [False, True])
def test_many_waves_counts_and_conservation(cap, bwd):
    """Broker Queue: success counts follow the FIFO specification exactly.
    BWD (single-shot check, not linearizable) may refuse while room is
    transiently reserved by others, so it can only fall short. Either way
    every value that comes out went in once, and all come out by the end."""
    import collections
    print(f"[queue] many-waves cap={cap} bwd={bwd}", flush=True)
    L = {"flags": pkg.BQ_F_BWD} if bwd else None
    q = pkg.Queue(cap)
    rng = np.random.default_rng(cap)
    size = 0
    offered = collections.Counter()
    taken = collections.Counter()
    n_in = 0
    nxt = 0
    for rep in range(6):
        n = int(rng.integers(1, 3 * cap))
        vals = np.arange(nxt, nxt + n, dtype=np.int32)
        nxt += n
        ok = q.enqueue(torch.from_numpy(vals).cuda(), launch=L)
        if bwd:
            assert ok <= min(n, cap - size)
        else:
            assert ok == min(n, cap - size)
        offered.update(vals.tolist())
        size += ok
        n_in += ok
        h, t, c = q.counters()
        assert t - h == c == size
        k = int(rng.integers(1, 2 * cap))
        out = q.dequeue(k, launch=L).cpu().numpy()
        if bwd:
            assert out.size <= min(k, size)
        else:
            assert out.size == min(k, size)
        size -= out.size
        taken.update(out.tolist())
    for _ in range(4):  # BWD may stop early; a few sweeps drain it
        out = q.dequeue(4 * cap, launch=L).cpu().numpy()
        taken.update(out.tolist())
    h, t, c = q.counters()
    assert c == 0 and t == h
    assert sum(taken.values()) == n_in
    assert all(v == 1 for v in taken.values())
    assert all(offered[k] >= 1 for k in taken)
    q.close()


def test_many_waves_exact_multiset():
    q = pkg.Queue(1 << 14)
    vals = np.random.default_rng(1).permutation(10000).astype(np.int32)
    assert q.enqueue(torch.from_numpy(vals).cuda()) == 10000
    out = q.dequeue(20000).cpu().numpy()
    history.check_conservation(vals, out, np.zeros(0))
    q.close()


def _mixed(cap, n_ops, launch=None):
    b = (launch or {}).get("ticket_batch", 1)
    print(f"[queue] mixed cap={cap} n_ops={n_ops} launch={launch}", flush=True)
    q = pkg.Queue(cap)
    st, el, dl = q.bench_mixed(n_ops, launch=launch, log=True)
    torch.cuda.synchronize()
    half = n_ops // 2
    assert st["enq_ok"] == half and st["deq_ok"] == half
    el, dl = el.cpu().numpy(), dl.cpu().numpy()
    history.check_positions(el, dl, half)
    history.check_conservation(np.arange(half), dl, np.zeros(0))
    # value i: chunk c = i // K of enqueuer wave c % W, lane (i % K) % 64,
    # that lane's item (c // W) * b + (i % K) // 64. Recode as (producer, seq).
    # Partitioned: the same within segment s = i // P (P = half / S), with
    # W / S enqueuer waves per segment; a producer stays in its segment.
    S = max(1, (launch or {}).get("segments", 1))
    P = half // S
    W = st["enq_waves"] // S
    K = 64 * b
    i = el.astype(np.int64)
    seg = i // P
    r = i - seg * P
    c = r // K
    prod = (seg * W + c % W) * 64 + (r % K) % 64
    seq = (c // W) * b + (r % K) // 64
    history.check_producer_fifo((prod << 20) | seq, 20)
    # each segment's log slice holds only that segment's values
    assert np.array_equal(seg, np.arange(half) // P)
    h, t, c = q.counters()
    history.check_quiescent(h, t, c, cap // S)
    q.close()
    return st


@pytest.mark.parametrize("cap", [64, 256, 4096, 1 << 20])
def test_mixed_small(cap):
    _mixed(cap, 1 << 20)


@pytest.mark.parametrize("wgs,wgsize", [(2, 64), (8, 256), (64, 512)])
@pytest.mark.parametrize("b", [1, 4, 16])
def test_mixed_shapes(wgs, wgsize, b):
    _mixed(1024, 1 << 18, {"wg_count": wgs, "wg_size": wgsize, "ticket_batch": b})


@pytest.mark.parametrize("b", [1, 8])
def test_mixed_bwd(b):
    """The BWD policy under the mixed scenario: every operation still
    completes (Full/Empty are retried) and the history checks hold."""
    _mixed(4096, 1 << 20, {"ticket_batch": b, "flags": pkg.BQ_F_BWD})


@pytest.mark.parametrize("segments", [2, 8])
@pytest.mark.parametrize("b", [1, 4])
def test_mixed_partitioned(segments, b):
    """The partitioned queue (one Broker Queue per XCD): each segment passes
    the position rule, conservation and per-producer order on its own."""
    _mixed(1 << 14, 1 << 20, {"ticket_batch": b, "segments": segments})


def test_mixed_partitioned_tiny_segments():
    """8 segments of 128 slots with b = 2: every segment only one chunk deep."""
    _mixed(1 << 10, 1 << 18, {"ticket_batch": 2, "segments": 8, "wg_count": 16})


def test_partitioned_rejects_bad_segment_counts():
    q = pkg.Queue(1 << 10)
    for L in ({"segments": 3}, {"segments": 16}, {"segments": 8, "ticket_batch": 4}):
        with pytest.raises(pkg.BQError):
            q.bench_mixed(1 << 12, launch=L)
    with pytest.raises(pkg.BQError):
        q.bench_mixed(6 * 8 + 2, launch={"segments": 8})  # n_ops/2 not a multiple of 8
    q.close()


@pytest.mark.parametrize("segments", [1, 8])
@pytest.mark.parametrize("bwd", [False, True])
def test_enqdeq_partitioned(segments, bwd):
    """Every segment holds exactly its share of the enqueues, so no enqueue
    can be refused under either policy (the broker reservation of a phase
    that only enqueues never finds the count short), and the dequeue phase
    takes every item back."""
    q = pkg.Queue(1 << 16)
    L = {"ticket_batch": 4, "segments": segments, "flags": pkg.BQ_F_BWD if bwd else 0}
    e, d = q.bench_enqdeq(1 << 17, launch=L)
    assert e["enq_ok"] == 1 << 16 and e["enq_full"] == 0
    assert d["deq_ok"] == 1 << 16 and d["deq_empty"] == 0
    q.close()


@pytest.mark.parametrize("cap,n_ops", [(1 << 16, 1 << 16), (1 << 16, 1 << 17), (1 << 12, 1 << 16)])
@pytest.mark.parametrize("bwd", [False, True])
def test_enqdeq(cap, n_ops, bwd):
    """Section IV EnqDeq: all enqueues, then all dequeues, one attempt each.
    Where the queue holds every enqueue, the count is exact under both
    policies; past capacity BWD may refuse a little more than the room it
    had (it never looks at the count twice), the Broker Queue exactly the
    excess. Either way the dequeues take back what went in and the
    counters agree at rest."""
    q = pkg.Queue(cap)
    L = {"ticket_batch": 4, "flags": pkg.BQ_F_BWD if bwd else 0}
    e, d = q.bench_enqdeq(n_ops, launch=L)
    half = n_ops // 2
    if half <= cap or not bwd:
        assert e["enq_ok"] == min(half, cap)
        assert (e["enq_full"] > 0) == (half > cap)
    else:
        assert 0 < e["enq_ok"] <= cap
    assert d["deq_ok"] == e["enq_ok"]
    h, t, c = q.counters()
    assert c == 0 and t == h == e["enq_ok"]
    q.close()


@pytest.mark.parametrize("b", [1, 4])
def test_bwd_bulk_exact_where_refusal_is_impossible(b):
    """BWD through bq_enqueue / bq_dequeue with many waves: the enqueue fits,
    so all of it succeeds; every value comes out exactly once (the dequeue
    output is the log), and the queue is empty at rest."""
    cap = 1 << 15
    L = {"flags": pkg.BQ_F_BWD, "ticket_batch": b}
    q = pkg.Queue(cap)
    vals = np.random.default_rng(b).permutation(cap).astype(np.int32)
    assert q.enqueue(torch.from_numpy(vals).cuda(), launch=L) == cap
    out = q.dequeue(cap, launch=L).cpu().numpy()
    assert out.size == cap
    history.check_conservation(vals, out, np.zeros(0))
    h, t, c = q.counters()
    assert c == 0 and t == h == cap
    q.close()


def test_queue_watchdog_then_recovery():
    """A 1 us watchdog on a tiny, crowded queue: waits for room or items
    outlast it, so the run stops through the kernel's own bounded checks and
    returns BQ_ETIMEOUT (the queue is reset by the call). If this box ever
    finishes the run inside the limit, the run must be whole. Either way
    the same queue then passes the full history checks."""
    cap = 64
    q = pkg.Queue(cap)
    try:
        st = q.bench_mixed(1 << 22, launch={"ticket_batch": 1, "timeout_us": 1})[0]
        print(f"[queue] watchdog did not fire: {st}", flush=True)
        assert st["enq_ok"] == st["deq_ok"] == 1 << 21
    except pkg.BQError as ex:
        assert ex.status == pkg.BQ_ETIMEOUT
    h, t, c = q.counters()
    assert c == 0 and t == h
    q.close()
    _mixed(cap, 1 << 18)


@pytest.mark.parametrize("b", [2, 8])
def test_mixed_batch_tiny_capacity(b):
    """K = 64*b items per ticket with a queue only a few chunks deep."""
    _mixed(64 * b * 2, 1 << 18, {"ticket_batch": b})


def test_mixed_full_size():
    """The measured configuration: 2^20 slots, 2^26 operations."""
    st = _mixed(1 << 20, 1 << 26)
    print(f"[queue] full mixed {st}", flush=True)
