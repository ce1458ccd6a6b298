"""bench.py's command line on the CPU: it refuses more than one GPU with a
message (the multi-GPU form of the path is not built) before touching a
device, and its counter-summary reader ignores summaries taken on other
sources or missing files. The served leg's shortest-path certificate
accepts the oracle's answers and rejects planted mistakes."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import synth  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU only" in (r.stdout + r.stderr)


def test_counter_summary_reader(tmp_path):
    from paper_2608_21826_amd.profsum import kernel_source_hash
    p = tmp_path / "s.txt"
    p.write_text("# header = ignored\n"
                 "kernel = k_solve<128>\n"
                 "hbm_bytes_per_launch = 1234\n"
                 f"kernel_source_hash = {kernel_source_hash()}\n"
                 "kernel = k_bench_mixed\n"
                 "hbm_bytes_per_launch = 99\n"
                 "kernel_source_hash = 0000000000000000\n")
    assert bench.read_counter_summary(str(p), "k_solve<128>", "hbm_bytes_per_launch") == 1234.0
    # another instantiation, a stale hash, a missing key or file: no value
    assert bench.read_counter_summary(str(p), "k_solve<64>", "hbm_bytes_per_launch") is None
    assert bench.read_counter_summary(str(p), "k_bench_mixed", "hbm_bytes_per_launch") is None
    assert bench.read_counter_summary(str(p), "k_solve<128>", "l2_hit_rate") is None
    assert bench.read_counter_summary(str(tmp_path / "none.txt"), "k_solve<128>", "x") is None


def _oracle_case(seed):
    import oracle
    g = synth.potential_random(400, 800, seed=seed)
    d, p, neg = oracle.sssp(g, g.src, method="fifo")
    assert not neg
    return g, d, p


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_certificate_accepts_oracle_and_rejects_planted_mistakes(seed):
    """bench.certify_sssp (the served leg's check) accepts the oracle's answer
    and rejects each planted mistake: a label one too high, one too low, an
    unreached vertex given a label, a wrong source label, a wrong pred."""
    torch = pytest.importorskip("torch")
    import oracle
    g, d, p = _oracle_case(seed)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a))
    off, col, w = t(g.offsets), t(g.cols), t(g.w)
    assert bench.certify_sssp(torch, off, col, w, g.src, t(d), t(p))
    reached = np.nonzero((d != oracle.INF) & (np.arange(g.n) != g.src))[0]
    unreached = np.nonzero(d == oracle.INF)[0]
    rng = np.random.default_rng(seed)
    v = int(rng.choice(reached))
    for delta in (1, -1):
        d2 = d.copy()
        d2[v] += delta
        assert not bench.certify_sssp(torch, off, col, w, g.src, t(d2), t(p)), delta
    if unreached.size:
        d2 = d.copy()
        d2[int(unreached[0])] = 0
        assert not bench.certify_sssp(torch, off, col, w, g.src, t(d2), t(p))
    d2 = d.copy()
    d2[g.src] = -1
    assert not bench.certify_sssp(torch, off, col, w, g.src, t(d2), t(p))
    p2 = p.copy()
    p2[v] = (p2[v] + 1) % g.n
    assert not bench.certify_sssp(torch, off, col, w, g.src, t(d), t(p2))
