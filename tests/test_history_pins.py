"""Pins of the queue-history checks (oracle/history.py).

The GPU queue tests accept a concurrent run when its position logs pass
check_positions, check_conservation, check_producer_fifo and
check_quiescent. Those checks are the consequences of linearizability to a
bounded FIFO (Section II.B) that a log of positions can show, with the
position rule coming from Alg. 1's tickets (PUT_DATA writes and READ_DATA
reads slot P mod N in round P / N). These tests show that each check

- accepts every history a sequential bounded FIFO produces (built here with
  collections.deque, not with the oracle), and
- rejects a history with one planted defect of the kind a broken queue
  would show: a dequeuer that read the wrong position, a lost item, an item
  delivered twice, two items of one producer leaving out of order, and
  counters that disagree at rest.

A final group plants plausible mistakes in the checks themselves (a swapped
sort key, an off-by-one slice, a non-strict comparison, ...) and shows that
the same pins reject every such mutant.
"""
import collections
import os
import types

import numpy as np
import pytest

from oracle import history

SHIFT = 20


def sequential_history(rng, producers=5, per_producer=40, cap=16, consumers=3):
    """Run a bounded FIFO (collections.deque) under a random schedule of
    producers that enqueue their items in sequence order and consumers that
    dequeue. Full / Empty attempts are retried later, as in the mixed
    scenario. Returns the enqueue and dequeue position logs (value at
    position P), the dequeue log stopping when every item has left."""
    fifo = collections.deque()
    nxt = [0] * producers
    enq_log, deq_log = [], []
    total = producers * per_producer
    while len(deq_log) < total:
        if rng.random() < 0.5:
            p = int(rng.integers(0, producers))
            if nxt[p] < per_producer and len(fifo) < cap:
                v = (p << SHIFT) | nxt[p]
                nxt[p] += 1
                fifo.append(v)
                enq_log.append(v)
        else:
            _ = int(rng.integers(0, consumers))
            if fifo:
                deq_log.append(fifo.popleft())
    return np.array(enq_log, np.int64), np.array(deq_log, np.int64)


def partial_history(rng, extra=7):
    """A history that stops with `extra` items still inside the queue."""
    el, dl = sequential_history(rng)
    keep = dl.size - extra
    return el, dl[:keep], el[keep:]


def check_all(el, dl, left, head, tail, count, cap, h=history):
    n = dl.size
    h.check_positions(el, dl, n)
    h.check_conservation(el, dl, left)
    h.check_producer_fifo(el, SHIFT)
    h.check_producer_fifo(dl, SHIFT)
    h.check_quiescent(head, tail, count, cap)


# ---------------------------------------------------------------------------
# valid histories pass
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(20))
def test_sequential_histories_pass(seed):
    rng = np.random.default_rng(seed)
    el, dl, left = partial_history(rng, extra=int(rng.integers(0, 10)))
    check_all(el, dl, left, dl.size, el.size, el.size - dl.size, 16)


def test_empty_history_passes():
    e = np.zeros(0, np.int64)
    check_all(e, e, e, 0, 0, 0, 64)


# ---------------------------------------------------------------------------
# one planted defect each, and the check that must reject it
# ---------------------------------------------------------------------------

def rejects(fn, *args):
    with pytest.raises(AssertionError):
        fn(*args)


@pytest.mark.parametrize("seed", range(10))
def test_swapped_positions_rejected(seed):
    """Two dequeuers that read each other's positions: same multiset, but the
    position rule fails."""
    rng = np.random.default_rng(100 + seed)
    el, dl = sequential_history(rng)
    i, j = sorted(rng.choice(dl.size, size=2, replace=False).tolist())
    bad = dl.copy()
    bad[i], bad[j] = dl[j], dl[i]
    history.check_conservation(el, bad, np.zeros(0))  # the multiset still holds
    rejects(history.check_positions, el, bad, dl.size)


def test_position_mismatch_in_last_slot_rejected():
    el, dl = sequential_history(np.random.default_rng(1))
    bad = dl.copy()
    bad[-1] = bad[-1] + 1
    rejects(history.check_positions, el, bad, dl.size)


@pytest.mark.parametrize("seed", range(10))
def test_lost_item_rejected(seed):
    """An item that went in and never came out (nor is inside)."""
    rng = np.random.default_rng(200 + seed)
    el, dl, left = partial_history(rng, extra=3)
    k = int(rng.integers(0, dl.size))
    rejects(history.check_conservation, el, np.delete(dl, k), left)
    rejects(history.check_conservation, el, dl, left[1:])


@pytest.mark.parametrize("seed", range(10))
def test_duplicated_item_rejected(seed):
    """An item delivered twice, in place of another one (same count)."""
    rng = np.random.default_rng(300 + seed)
    el, dl = sequential_history(rng)
    i, j = rng.choice(dl.size, size=2, replace=False).tolist()
    bad = dl.copy()
    bad[i] = dl[j]
    rejects(history.check_conservation, el, bad, np.zeros(0))
    # one extra copy on top of a complete delivery
    rejects(history.check_conservation, el, np.append(dl, dl[j]), np.zeros(0))


@pytest.mark.parametrize("seed", range(10))
def test_producer_reorder_rejected(seed):
    """Two items of one producer, far apart with other producers' items
    between them, leave in the wrong order. Positions stay consistent
    (both logs swapped), so only the per-producer order can see it."""
    rng = np.random.default_rng(400 + seed)
    el, dl = sequential_history(rng)
    prod = el >> SHIFT
    p = int(rng.integers(0, prod.max() + 1))
    pos = np.nonzero(prod == p)[0]
    # two positions of producer p with another producer's item between them
    for a in range(pos.size):
        for b in range(pos.size - 1, a, -1):
            if np.any(prod[pos[a]:pos[b]] != p):
                i, j = int(pos[a]), int(pos[b])
                break
        else:
            continue
        break
    bad = el.copy()
    bad[i], bad[j] = el[j], el[i]
    history.check_positions(bad, bad, bad.size)
    history.check_conservation(el, bad, np.zeros(0))
    rejects(history.check_producer_fifo, bad, SHIFT)


def test_adjacent_producer_reorder_rejected():
    v = np.array([(1 << SHIFT) | 1, (1 << SHIFT) | 0, (2 << SHIFT) | 0], np.int64)
    rejects(history.check_producer_fifo, v, SHIFT)


def test_repeated_sequence_number_rejected():
    """The same (producer, seq) twice: not strictly increasing."""
    v = np.array([(3 << SHIFT) | 5, (0 << SHIFT) | 1, (3 << SHIFT) | 5], np.int64)
    rejects(history.check_producer_fifo, v, SHIFT)


def test_interleaved_producers_in_order_pass():
    """Producers interleave arbitrarily; each on its own is increasing."""
    v = np.array([(2 << SHIFT) | 0, (0 << SHIFT) | 0, (2 << SHIFT) | 1, (1 << SHIFT) | 0,
                  (0 << SHIFT) | 4, (2 << SHIFT) | 9], np.int64)
    history.check_producer_fifo(v, SHIFT)


@pytest.mark.parametrize("head,tail,count,cap", [
    (10, 15, 4, 16),      # count != tail - head
    (10, 15, 6, 16),
    (10, 27, 17, 16),     # more than capacity inside
    (15, 10, -5, 16),     # head passed tail
    (0, 0, 1, 16),
])
def test_bad_counters_rejected(head, tail, count, cap):
    rejects(history.check_quiescent, head, tail, count, cap)


@pytest.mark.parametrize("head,tail,count,cap", [(0, 0, 0, 1), (7, 23, 16, 16), (5, 5, 0, 64)])
def test_good_counters_pass(head, tail, count, cap):
    history.check_quiescent(head, tail, count, cap)


# ---------------------------------------------------------------------------
# planted mistakes in the checks themselves
# ---------------------------------------------------------------------------

SRC = open(os.path.join(os.path.dirname(history.__file__), "history.py")).read()

MUTANTS = {
    # sort by position first: producers are no longer grouped, so a
    # producer's items are compared with whatever item comes next
    "lexsort_keys_swapped": ("np.lexsort((np.arange(v.size), prod))",
                             "np.lexsort((prod, np.arange(v.size)))"),
    # sort by producer only (unstable order inside a producer)
    "lexsort_no_position": ("np.lexsort((np.arange(v.size), prod))",
                            "np.argsort(prod, kind='quicksort')[::-1]"),
    "fifo_non_strict": ("(s_sorted[1:] <= s_sorted[:-1])", "(s_sorted[1:] < s_sorted[:-1])"),
    "fifo_wrong_shift": ("prod = v >> producer_shift", "prod = v >> (producer_shift + 1)"),
    "positions_off_by_one": ("a = np.asarray(enq_log[:n_deq])\n    b = np.asarray(deq_log[:n_deq])",
                             "a = np.asarray(enq_log[:n_deq - 1])\n"
                             "    b = np.asarray(deq_log[:n_deq - 1])"),
    "positions_sorted": ("bad = np.nonzero(a != b)[0]",
                         "bad = np.nonzero(np.sort(a) != np.sort(b))[0]"),
    "conservation_unique": ("y = np.sort(np.concatenate(", "y = np.unique(np.concatenate("),
    "conservation_no_remaining": ("np.asarray(remaining, dtype=np.int64)]))",
                                  "np.asarray(remaining, dtype=np.int64)[:0]]))"),
    "quiescent_no_count": ("    if count != size:", "    if False:"),
    "quiescent_open_bound": ("if not (0 <= size <= capacity):",
                             "if not (0 <= size <= capacity + 1):"),
}


def _mutant(name):
    old, new = MUTANTS[name]
    assert SRC.count(old) == 1, f"mutation site of {name} not found once"
    mod = types.ModuleType(f"history_{name}")
    exec(compile(SRC.replace(old, new), f"history_{name}.py", "exec"), mod.__dict__)
    return mod


def _pins_pass(h) -> bool:
    """The pins above, run against module h; False as soon as one fails."""
    try:
        for seed in range(6):
            rng = np.random.default_rng(seed)
            el, dl, left = partial_history(rng, extra=int(rng.integers(0, 10)))
            check_all(el, dl, left, dl.size, el.size, el.size - dl.size, 16, h=h)
        cases = []
        for seed in range(6):
            rng = np.random.default_rng(500 + seed)
            el, dl, left = partial_history(rng, extra=3)
            i, j = sorted(rng.choice(dl.size, size=2, replace=False).tolist())
            sw = dl.copy()
            sw[i], sw[j] = dl[j], dl[i]
            cases.append(lambda el=el, sw=sw: h.check_positions(el, sw, sw.size))
            cases.append(lambda el=el, dl=dl, left=left: h.check_conservation(el, dl, left[1:]))
            du = dl.copy()
            du[i] = dl[j]
            cases.append(lambda el=el, du=du, left=left: h.check_conservation(el, du, left))
            cases.append(lambda el=el, dl=dl, left=left, j=j:
                         h.check_conservation(el, np.append(dl, dl[j]), left))
            last = dl.copy()
            last[-1] += 1
            cases.append(lambda el=el, last=last: h.check_positions(el, last, last.size))
            prod = el >> SHIFT
            for p in range(prod.max() + 1):
                pos = np.nonzero(prod == p)[0]
                if pos.size >= 2 and np.any(prod[pos[0]:pos[-1]] != p):
                    bad = el.copy()
                    bad[pos[0]], bad[pos[-1]] = el[pos[-1]], el[pos[0]]
                    cases.append(lambda bad=bad: h.check_producer_fifo(bad, SHIFT))
                    break
        cases.append(lambda: h.check_producer_fifo(
            np.array([(3 << SHIFT) | 5, (0 << SHIFT) | 1, (3 << SHIFT) | 5], np.int64), SHIFT))
        cases.append(lambda: h.check_producer_fifo(
            np.array([(1 << SHIFT) | 1, (1 << SHIFT) | 0], np.int64), SHIFT))
        for args in ((10, 15, 4, 16), (10, 27, 17, 16), (15, 10, -5, 16), (0, 17, 17, 16)):
            cases.append(lambda args=args: h.check_quiescent(*args))
        for case in cases:
            try:
                case()
            except AssertionError:
                continue
            return False
        h.check_producer_fifo(np.array([(2 << SHIFT) | 0, (0 << SHIFT) | 0, (2 << SHIFT) | 1,
                                        (1 << SHIFT) | 0], np.int64), SHIFT)
        h.check_quiescent(7, 23, 16, 16)
    except AssertionError:
        return False
    return True


def test_pins_pass_on_the_real_checks():
    assert _pins_pass(history)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    assert not _pins_pass(_mutant(name)), f"mutant {name} survived the pins"
