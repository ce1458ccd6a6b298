"""Checks of concurrent queue histories (test infrastructure).

A concurrent run of the queue does not have one right answer: the order in
which lanes win their tickets is up to the hardware. What the paper fixes is
that the queue is a linearizable FIFO (Section II.B's definitions, the Broker
Queue of Section III.A): every history must be explainable by the sequential
FIFO in ``oracle.fifo_run``. These checks test the consequences of that which
a log of positions can show:

- position rule (Alg. 1, PUT_DATA / READ_DATA): the item read by the dequeuer
  that drew head position P is the item written by the enqueuer that drew
  tail position P;
- conservation: what was dequeued plus what is still inside equals, as a
  multiset, what was enqueued;
- per-producer FIFO: items of one producer leave in the order that producer
  put them in;
- quiescent count: at rest 0 <= tail - head <= capacity and count equals it.

Pinned by tests/test_history_pins.py: histories of a sequential bounded
FIFO pass every check; one planted defect each (a swapped position, a lost
item, a duplicated item, a per-producer reorder, disagreeing counters) is
rejected; and planted mistakes in these checks are caught by those pins.
"""
from __future__ import annotations

import numpy as np


def check_positions(enq_log: np.ndarray, deq_log: np.ndarray, n_deq: int) -> None:
    """enq_log[P] / deq_log[P]: value written / read at queue position P."""
    a = np.asarray(enq_log[:n_deq])
    b = np.asarray(deq_log[:n_deq])
    bad = np.nonzero(a != b)[0]
    if bad.size:
        p = int(bad[0])
        raise AssertionError(f"position {p}: enqueued {a[p]} but dequeued {b[p]} "
                             f"({bad.size} mismatches)")


def check_conservation(enqueued: np.ndarray, dequeued: np.ndarray,
                       remaining: np.ndarray) -> None:
    x = np.sort(np.asarray(enqueued, dtype=np.int64))
    y = np.sort(np.concatenate([np.asarray(dequeued, dtype=np.int64),
                                np.asarray(remaining, dtype=np.int64)]))
    if x.shape != y.shape or not np.array_equal(x, y):
        raise AssertionError(f"multiset not conserved: {x.size} in, {y.size} out/left")


def check_producer_fifo(values_by_position: np.ndarray, producer_shift: int = 20) -> None:
    """Values are (producer << shift) | seq; along increasing positions, the
    seq numbers of each producer must increase."""
    v = np.asarray(values_by_position, dtype=np.int64)
    prod = v >> producer_shift
    seq = v & ((1 << producer_shift) - 1)
    order = np.lexsort((np.arange(v.size), prod))  # by producer, then position
    p_sorted, s_sorted = prod[order], seq[order]
    same = p_sorted[1:] == p_sorted[:-1]
    bad = np.nonzero(same & (s_sorted[1:] <= s_sorted[:-1]))[0]
    if bad.size:
        i = int(bad[0])
        raise AssertionError(f"producer {p_sorted[i]}: seq {s_sorted[i + 1]} left after "
                             f"{s_sorted[i]}")


def check_quiescent(head: int, tail: int, count: int, capacity: int) -> None:
    size = tail - head
    if not (0 <= size <= capacity):
        raise AssertionError(f"tail - head = {size} outside [0, {capacity}]")
    if count != size:
        raise AssertionError(f"count {count} != tail - head {size}")
