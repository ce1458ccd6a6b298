"""Stored expected results of the full-size configurations (test helper).

The JSON files under tests/golden/ are written by tests/golden/make_golden.py,
which calls only the CPU oracle and certifies every result with an
independent algorithm before it writes (the Johnson closed form on the
potential-shifted graphs, a library Dijkstra on the grid, the planted
cycle's weight and reachability for the flag). A GPU result is compared
with them through SHA-256 digests of its bytes.
"""
import hashlib
import json
import os

import numpy as np

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
FILES = {"grid64": "grid64.json", "rmat20": "rmat20.json", "rmat20_x64_sources": "rmat20.json",
         "road2048": "road2048.json", "road2048_negcycle": "road2048.json",
         "er256": "er256.json"}


def load(name: str) -> dict:
    with open(os.path.join(HERE, FILES[name])) as f:
        return json.load(f)[name]


def digest(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def graph_digest(g) -> str:
    h = hashlib.sha256()
    for a in (g.offsets, g.cols, g.w):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def check(rec: dict, dist: np.ndarray, pred: np.ndarray, what: str = "") -> None:
    """dist / pred (host arrays) must be the stored result, byte for byte.
    The stored samples are compared first, so a mismatch names positions."""
    idx = np.asarray(rec["sample_idx"], dtype=np.int64)
    d_s, p_s = np.asarray(rec["sample_dist"]), np.asarray(rec["sample_pred"])
    bad = np.nonzero(dist[idx] != d_s)[0]
    assert bad.size == 0, (f"{what}: dist differs at {idx[bad[:5]].tolist()}: "
                           f"{dist[idx[bad[:5]]].tolist()} vs {d_s[bad[:5]].tolist()}")
    bad = np.nonzero(pred[idx] != p_s)[0]
    assert bad.size == 0, (f"{what}: pred differs at {idx[bad[:5]].tolist()}: "
                           f"{pred[idx[bad[:5]]].tolist()} vs {p_s[bad[:5]].tolist()}")
    assert digest(dist) == rec["dist_sha256"], f"{what}: dist digest differs"
    assert digest(pred) == rec["pred_sha256"], f"{what}: pred digest differs"
