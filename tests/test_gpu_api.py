"""GPU checks of C ABI calls that the other tests reach only through a wrapper
or not at all:

- the two halves of the batched call, sssp_bf_batched_start and
  sssp_batch_finish: a second start while a launch runs and a finish with
  nothing started are refused as the header states, a finish without
  waiting answers BQ_EBUSY or the result, and the result (distances,
  predecessors, flags, reached edges per query) equals the oracle's;
- the solver's timeline (BQ_F_TRACE, sssp_last_trace) leaves the answer
  exact and counts dequeued vertex items in increasing order;
- bq_reset on a queue that holds items: it is empty again and then behaves
  as a new one-wave FIFO.
"""
import ctypes
import time

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pkg = pytest.importorskip("paper_2608_21826_amd")

DEV = torch.device("cuda:0")


def upload(g):
    return tuple(torch.from_numpy(a).to(DEV) for a in (g.offsets, g.cols, g.w))


def reached_edges(g, d):
    return int(np.diff(g.offsets)[d != oracle.INF].sum())


def test_batched_start_finish():
    graphs = [synth.rmat(15, seed=synth.SEED_BASE + 71)] + \
             [synth.potential_random(int(n), int(4 * n), seed=70 + i)
              for i, n in enumerate((300, 2000, 9000))]
    print(f"[api] start/finish over {[g.n for g in graphs]}", flush=True)
    qs = []
    for g in graphs:
        off, col, w = upload(g)
        qs.append((off, col, w, int(g.src), torch.empty(g.n, dtype=torch.int64, device=DEV),
                   torch.empty(g.n, dtype=torch.int32, device=DEV)))
    b = pkg.SsspBatch(len(qs), sum(g.n for g in graphs), sum(g.m for g in graphs))
    L = pkg.lib()
    arr = b._table(qs)
    neg = (ctypes.c_int32 * len(qs))()
    reach = (ctypes.c_int64 * len(qs))()
    assert L.sssp_batch_finish(b.handle, neg, reach, 1) == pkg.BQ_EINVAL  # nothing started
    s = pkg._stream()
    assert L.sssp_bf_batched_start(b.handle, len(qs), arr, None, s) == pkg.BQ_OK
    assert L.sssp_bf_batched_start(b.handle, len(qs), arr, None, s) == pkg.BQ_EBUSY
    t0 = time.time()
    while True:
        st = L.sssp_batch_finish(b.handle, neg, reach, 0)
        if st != pkg.BQ_EBUSY:
            break
        assert time.time() - t0 < 60, "the batched launch did not finish"
        time.sleep(0.001)
    assert st == pkg.BQ_OK
    torch.cuda.synchronize()
    for (off, col, w, src, dist, pred), g, flag, r in zip(qs, graphs, neg, reach):
        d_ref, p_ref, neg_ref = oracle.sssp(g, src, method="fifo")
        assert bool(flag) == neg_ref == False  # noqa: E712
        assert np.array_equal(dist.cpu().numpy(), d_ref), g.name
        assert np.array_equal(pred.cpu().numpy(), p_ref), g.name
        assert r == reached_edges(g, d_ref), g.name
    # the workspace takes the next launch, here through the blocking call
    assert b.solve(qs) == [False] * len(qs)
    b.close()


@pytest.mark.parametrize("launch", [None, {"bucket_width": 4}, {"segments": 2, "ticket_batch": 2}])
def test_trace_keeps_the_answer(launch):
    g = synth.rmat(14, seed=synth.SEED_BASE + 72)
    print(f"[api] trace {launch} on {g.name}", flush=True)
    off, col, w = upload(g)
    ctx = pkg.SsspContext(g.n, g.m)
    d, p, neg = ctx.solve(off, col, w, g.src, launch=launch, trace=True)
    tr = ctx.trace()
    st = ctx.stats()
    d_ref, p_ref, neg_ref = oracle.sssp(g, g.src, method="fifo")
    assert not neg and not neg_ref
    assert np.array_equal(d.cpu().numpy(), d_ref) and np.array_equal(p.cpu().numpy(), p_ref)
    assert tr.shape[0] > 0 and tr.shape[1] == 4
    deq = tr[:, 1].astype(np.int64)
    assert np.all(np.diff(deq) > 0)
    assert deq[-1] <= st["dequeued"]
    ctx.close()


def test_reset_empties_a_live_queue():
    print("[api] bq_reset", flush=True)
    one = {"wg_size": 64, "wg_count": 1}
    q = pkg.Queue(256)
    vals = torch.arange(1000, 1200, dtype=torch.int32, device=DEV)
    assert q.enqueue(vals, launch=one) == 200
    assert q.dequeue(30, launch=one).numel() == 30
    assert q.counters() == (30, 200, 170)
    q.reset()
    assert q.counters() == (0, 0, 0)
    assert q.dequeue(10, launch=one).numel() == 0
    v2 = torch.arange(7, 7 + 256, dtype=torch.int32, device=DEV)
    assert q.enqueue(v2, launch=one) == 256
    assert q.enqueue(v2[:5], launch=one) == 0  # full
    assert torch.equal(q.dequeue(256, launch=one).cpu(), v2.cpu())
    assert q.counters() == (256, 256, 0)
    q.close()
