"""The queue's CPU baselines (oracle/queue_cpu.c): the host Broker Queue
model on several threads must pass the same history checks as the GPU queue
(position rule, conservation, per-producer order), and the sequential ring
must move every item."""
import numpy as np
import pytest

import oracle
from oracle import history


@pytest.mark.parametrize("cap,threads", [(1, 2), (2, 4), (64, 8), (1 << 12, 6), (1 << 16, 8)])
def test_bq_model_histories(cap, threads):
    n_ops = 1 << 15
    half = n_ops // 2
    t, fails, el, dl = oracle.bq_mixed(cap, n_ops, threads, log=True)
    history.check_positions(el, dl, half)
    history.check_conservation(np.arange(half), dl, np.zeros(0))
    # enqueuer k of `threads // 2` owns the contiguous values [lo_k, hi_k)
    per = threads // 2
    bounds = np.array([half * k // per for k in range(per + 1)])
    prod = np.searchsorted(bounds, el, side="right") - 1
    seq = el - bounds[prod]
    history.check_producer_fifo((prod.astype(np.int64) << 20) | seq, 20)
    assert fails >= 0


def test_ring_mixed_runs():
    assert oracle.ring_mixed(1 << 10, 1 << 16) >= 0.0
