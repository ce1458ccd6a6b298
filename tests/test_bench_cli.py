"""bench.py's command line on the CPU: it refuses more than one GPU with a
message (the multi-GPU form of the path is not built) before touching a
device, and its counter-summary reader ignores summaries taken on other
sources or missing files."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU only" in (r.stdout + r.stderr)


def test_counter_summary_reader(tmp_path):
    import bench
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
