"""Planted mistakes in the oracle must be caught by its pins.

Each case copies oracle.c, plants one plausible mistake (a wrong comparison,
sign, index or bound), builds the copy into a temporary library on the CPU
and checks that the pins of test_oracle_pins reject it. This shows the pins
are strong enough to catch that class of error in the real oracle.

Mutants that cannot change any output are left out: e.g. a wrong tie test in
the predecessor loop (rows are visited in increasing id, so the first tight
in-neighbour found is already the smallest), or a dropped hop increment in
the FIFO form (its parent-graph check finds the same cycles).
"""
import collections
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
import synth

sys.path.insert(0, os.path.dirname(__file__))
from test_oracle_pins import brute_force, brute_neg_inf  # noqa: E402

SRC = open(os.path.join(os.path.dirname(oracle.__file__), "oracle.c")).read()

MUTANTS = {
    "rounds_le": ("if (nd < d[v]) {\n                        d[v] = nd;\n                        changes++;",
                  "if (nd <= d[v]) {\n                        d[v] = nd;\n                        changes++;"),
    "rounds_no_inf_guard": ("if (dist1 != ORACLE_INF) {", "if (1) {"),
    "rounds_sign": ("int64_t nd = dist1 + (int64_t)w[e];", "int64_t nd = dist1 - (int64_t)w[e];"),
    "rounds_last_round": ("if (i == (int64_t)n - 1 && changes > 0)",
                          "if (i == (int64_t)n - 2 && changes > 0)"),
    "rounds_no_early_exit_reset": ("        int64_t changes = 0;\n        rounds++;",
                                   "        static int64_t changes = 0;\n        rounds++;"),
    "pred_transposed": ("if (d[u] + (int64_t)w[e] == d[v] &&", "if (d[v] + (int64_t)w[e] == d[u] &&"),
    "fifo_no_requeue": ("if (!inq[v]) {", "if (!inq[v] && d[v] == ORACLE_INF) {"),
    "fifo_le": ("            if (nd < d[v]) {\n                d[v] = nd;\n                hops[v]",
                "            if (nd <= d[v]) {\n                d[v] = nd;\n                hops[v]"),
    "pred_largest": ("(pred[v] < 0 || u < pred[v])", "(pred[v] < 0 || u > pred[v])"),
    "queue_lifo": ("out[i] = ring[head];\n                head = (head + 1) % cap;",
                   "out[i] = ring[(head + size - 1) % cap];"),
    "queue_capacity": ("if (size == cap) {", "if (size == cap + 1) {"),
    "neginf_no_spread": ("                if (!mark[col[e]]) {\n                    mark[col[e]] = 1;",
                         "                if (0) {\n                    mark[col[e]] = 1;"),
    "neginf_le": ("if (d[u] + (int64_t)w[e] < d[col[e]])\n                mark[col[e]] = 1;",
                  "if (d[u] + (int64_t)w[e] <= d[col[e]])\n                mark[col[e]] = 1;"),
    "neginf_short_rounds": ("for (int64_t i = 0; i + 1 < n; i++) {",
                            "for (int64_t i = 0; i + 2 < n; i++) {"),
}


def _build(tmp_path, name, text):
    src = tmp_path / f"{name}.c"
    src.write_text(text)
    out = tmp_path / f"lib{name}.so"
    subprocess.run(["gcc", "-O1", "-std=c11", "-shared", "-fPIC", "-o", str(out), str(src)],
                   check=True)
    return oracle.load(str(out))


def _pins_pass(lib) -> bool:
    """Run a compact set of pins; False as soon as one fails."""
    try:
        # brute force on tiny graphs (distances and flag) incl. pred
        for seed in range(120):
            rng = np.random.default_rng(seed)
            n = int(rng.integers(1, 8))
            m = int(rng.integers(0, 3 * n + 1))
            g = synth.random_small(n, m, -5, 10, seed=1000 + seed)
            src = int(rng.integers(0, n))
            d_bf, neg_bf, _ = brute_force(g, src)
            d2, neg2, _ = oracle.bf_rounds(g, src, lib)
            d3, neg3, _, _ = oracle.bf_fifo(g, src, lib)
            if neg2 != neg_bf or neg3 != neg_bf:
                return False
            if not neg_bf and not (np.array_equal(d2, d_bf) and np.array_equal(d3, d_bf)):
                return False
        for seed in range(60):
            rng = np.random.default_rng(seed)
            n = int(rng.integers(2, 8))
            m = int(rng.integers(0, 3 * n + 1))
            g = synth.random_small(n, m, 1, 6, seed=5000 + seed)
            src = int(rng.integers(0, n))
            d_bf, _, penult = brute_force(g, src)
            d, p, neg = oracle.sssp(g, src, lib=lib)
            for v in range(n):
                exp = -1 if (v == src or d_bf[v] == oracle.INF) else min(penult[v])
                if p[v] != exp:
                    return False
        # ties between consecutive ids (a diamond and a wider fan)
        for g in (synth.csr_from_edges(4, [0, 0, 1, 2], [1, 2, 3, 3], [1, 1, 1, 1]),
                  synth.csr_from_edges(6, [0, 0, 0, 0, 2, 3, 4, 1], [2, 3, 4, 1, 5, 5, 5, 5],
                                       [2, 1, 1, 1, 1, 2, 2, 2])):
            d_bf, _, penult = brute_force(g, 0)
            d, p, neg = oracle.sssp(g, 0, lib=lib)
            if p[-1] != min(penult[-1]):
                return False
        # path graph needing n-1 rounds
        n = 60
        w = np.random.default_rng(3).integers(-50, 50, size=n - 1)
        ids = np.arange(n)[::-1]
        g = synth.csr_from_edges(n, ids[:-1], ids[1:], w, source=int(ids[0]))
        d, neg, _ = oracle.bf_rounds(g, None, lib)
        exp = np.zeros(n, dtype=np.int64)
        exp[ids[1:]] = np.cumsum(w)
        if neg or not np.array_equal(d, exp):
            return False
        # sequential FIFO vs deque
        for seed in range(10):
            rng = np.random.default_rng(seed)
            cap = int(rng.integers(1, 9))
            ops = np.where(rng.random(200) < 0.55, rng.integers(0, 10**6, size=200), -1)
            res, out, size = oracle.fifo_run(cap, ops, lib)
            q = collections.deque()
            for i, op in enumerate(ops.tolist()):
                if op >= 0:
                    ok = len(q) < cap
                    if ok:
                        q.append(op)
                    if res[i] != ok:
                        return False
                elif q:
                    if res[i] != 1 or out[i] != q.popleft():
                        return False
                elif res[i] != 0:
                    return False
        # a planted reachable zero-weight 2-cycle next to a -1 one
        g = synth.csr_from_edges(4, [0, 1, 2, 0, 3], [1, 2, 1, 3, 3], [1, 2, -2, 1, 0],
                                 source=0)
        if oracle.bf_fifo(g, None, lib)[1] or oracle.bf_rounds(g, None, lib)[1]:
            return False
        g = synth.csr_from_edges(3, [0, 1, 2], [1, 2, 1], [1, 2, -3], source=0)
        if not oracle.bf_fifo(g, None, lib)[1] or not oracle.bf_rounds(g, None, lib)[1]:
            return False
        # minus-infinity marking: tiny graphs and a path needing n-1 rounds
        for seed in range(120):
            rng = np.random.default_rng(20000 + seed)
            n = int(rng.integers(1, 8))
            m = int(rng.integers(0, 3 * n + 1))
            g = synth.random_small(n, m, -5, 10, seed=21000 + seed)
            src = int(rng.integers(0, n))
            d, p, neg = oracle.neg_inf(g, src, lib)
            if not np.array_equal(d == oracle.NEG_INF, brute_neg_inf(g, src)):
                return False
        n = 40
        ids = np.arange(n)[::-1]
        w = np.random.default_rng(4).integers(-20, 20, size=n - 1)
        g = synth.csr_from_edges(n, ids[:-1], ids[1:], w, source=int(ids[0]))
        d, p, neg = oracle.neg_inf(g, None, lib)
        if neg or np.any(d == oracle.NEG_INF):
            return False
    except (AssertionError, IndexError, ValueError, OverflowError):
        return False
    return True


def test_pins_accept_real_oracle(tmp_path):
    lib = _build(tmp_path, "real", SRC)
    assert _pins_pass(lib)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_reject_mutant(tmp_path, name):
    old, new = MUTANTS[name]
    assert SRC.count(old) == 1, f"mutation anchor for {name} not unique/found"
    lib = _build(tmp_path, name, SRC.replace(old, new))
    assert not _pins_pass(lib), f"pins did not catch mutant {name}"
