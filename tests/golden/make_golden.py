"""Write the stored expected results for the full-size road configurations.

Calls only the CPU oracle (sequential FIFO Bellman-Ford + smallest-id tight
predecessor) on graphs from the seeded generators, and stores SHA-256
digests of the inputs and outputs plus a sample of values, so the GPU tests
can check bit-exactness without re-running the ~1 minute CPU solve.

Run from the repository root:  python tests/golden/make_golden.py
"""
import hashlib
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402


def sha(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def graph_digest(g) -> str:
    h = hashlib.sha256()
    for a in (g.offsets, g.cols, g.w):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def main():
    out = {}
    for name in ("road2048", "road2048_negcycle"):
        g = synth.config_graph(name)
        d, neg, pops, relax = oracle.bf_fifo(g)
        rec = {"n": g.n, "m": g.m, "src": g.src, "graph_sha256": graph_digest(g),
               "neg_cycle": bool(neg), "oracle": "bf_fifo", "pops": pops,
               "relaxations": relax}
        if not neg:
            p = oracle.pred(g, d)
            rng = np.random.default_rng(12345)
            idx = np.sort(rng.choice(g.n, size=2000, replace=False))
            rec.update({"dist_sha256": sha(d), "pred_sha256": sha(p),
                        "reached": int(np.count_nonzero(d != oracle.INF)),
                        "sample_idx": idx.tolist(), "sample_dist": d[idx].tolist(),
                        "sample_pred": p[idx].tolist()})
        out[name] = rec
        print(name, {k: v for k, v in rec.items() if not k.startswith("sample")}, flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "road2048.json")
    with open(path, "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
