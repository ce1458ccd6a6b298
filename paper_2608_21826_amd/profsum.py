"""Summaries of rocprofv3 result databases (kernel trace and counter runs).

    python -m paper_2608_21826_amd.profsum trace <results.db> [--last N kernel-substring]
    python -m paper_2608_21826_amd.profsum pmc <fetch.db> <write.db> <kernel-substring> [--last N]
    python -m paper_2608_21826_amd.profsum counters <db> <kernel-substring> <counter>... [--last N]

`trace` prints per-kernel call counts and average / min / max durations.
`counters` prints a kernel's counter values per dispatch and their means, and
the L2 hit rate when TCC_HIT_sum and TCC_MISS_sum are among them.
`pmc` prints FETCH_SIZE and WRITE_SIZE per dispatch (KiB, as the counters
read), scales each by what the same counter reads for the calibration copy
kernel (k_probe_copy: 1 GiB read and 1 GiB written), and prints HBM bytes per
launch of the kernel named by the substring, plus the hash of the solver
sources the run was taken on.
`--last N` keeps only the last N dispatches (in dispatch order) of the named
kernel, for runs where the timed launches follow others of the same kernel
(a launch search, smaller cases).
"""
from __future__ import annotations

import collections
import hashlib
import os
import re
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CALIB_BYTES = 1 << 30


KERNEL_SOURCES = ("bq_device.hpp", "sssp_device.hpp", "sssp_kernels.hpp")
SOURCES_OF = {  # kernel-name substring -> the sources its code comes from
    "k_bsolve": ("bq_device.hpp", "sssp_device.hpp", "sssp_batched.hip"),
    "k_bench_mixed": ("bq_device.hpp", "bq_queue.hip"),
}


def _code_of(text: str) -> str:
    """The code of a C++ source without its comments and with its blank
    space collapsed: editing a comment does not change what a summary
    describes."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_hash(kernel: str = "k_solve") -> str:
    """Hash of the code of the sources a kernel is built from (the
    single-query solver's by default); a counter summary taken on other code
    no longer describes it."""
    files = next((v for k, v in SOURCES_OF.items() if k in kernel), KERNEL_SOURCES)
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(HERE, "csrc", f)) as fh:
            h.update(_code_of(fh.read()).encode())
    return h.hexdigest()[:16]


def _short(name: str) -> str:
    name = name.replace("(anonymous namespace)::", "")
    return name.split("(")[0] if "(" in name else name


def trace(db: str, last: int = 0, kernel: str = "") -> str:
    c = sqlite3.connect(db)
    rows = list(c.execute("select name, duration from kernels order by dispatch_id"))
    agg = collections.defaultdict(list)
    for n, d in rows:
        agg[_short(n)].append(d)
    if last:
        agg = {n: ds[-last:] for n, ds in agg.items() if kernel in n}
    lines = [f"{'kernel':48s} {'calls':>6s} {'avg_us':>12s} {'min_us':>12s} {'max_us':>12s}"]
    for n, ds in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
        lines.append(f"{n[:48]:48s} {len(ds):6d} {sum(ds) / len(ds) / 1e3:12.3f} "
                     f"{min(ds) / 1e3:12.3f} {max(ds) / 1e3:12.3f}")
    return "\n".join(lines)


def _counter(db: str, cname: str, last: int = 0):
    c = sqlite3.connect(db)
    agg = collections.defaultdict(list)
    for k, n, v in c.execute("select kernel_name, counter_name, value from counters_collection "
                             "order by dispatch_id"):
        if n == cname:
            agg[_short(k)].append(float(v))
    if last:
        agg = {k: (vs if "k_probe_copy" in k else vs[-last:]) for k, vs in agg.items()}
    return agg


def pmc(fetch_db: str, write_db: str, kernel: str, last: int = 0) -> str:
    f = _counter(fetch_db, "FETCH_SIZE", last)
    w = _counter(write_db, "WRITE_SIZE", last)
    cf = [v for k, v in f.items() if "k_probe_copy" in k][0][0]
    cw = [v for k, v in w.items() if "k_probe_copy" in k][0][0]
    fscale = CALIB_BYTES / (cf * 1024.0)
    wscale = CALIB_BYTES / (cw * 1024.0)
    kf = [v for k, v in f.items() if kernel in k][0]
    kw = [v for k, v in w.items() if kernel in k][0]
    fb = sum(kf) / len(kf) * 1024.0 * fscale
    wb = sum(kw) / len(kw) * 1024.0 * wscale
    out = [
        f"kernel = {kernel}",
        f"fetch_kib_per_dispatch = {[round(x) for x in kf]}",
        f"write_kib_per_dispatch = {[round(x) for x in kw]}",
        f"calib_copy_fetch_kib = {cf:.0f}",
        f"calib_copy_write_kib = {cw:.0f}",
        f"fetch_scale = {fscale:.4f}",
        f"write_scale = {wscale:.4f}",
        f"hbm_fetch_bytes_per_launch = {fb:.0f}",
        f"hbm_write_bytes_per_launch = {wb:.0f}",
        f"hbm_bytes_per_launch = {fb + wb:.0f}",
        f"kernel_source_hash = {kernel_source_hash(kernel)}",
    ]
    return "\n".join(out)


def counters(db: str, kernel: str, names, last: int = 0) -> str:
    """Per-dispatch values and means of counters of one kernel; with
    TCC_HIT_sum and TCC_MISS_sum also the L2 hit rate."""
    out = [f"kernel = {kernel}"]
    means = {}
    for cname in names:
        vals = [v for k, v in _counter(db, cname, last).items() if kernel in k][0]
        means[cname] = sum(vals) / len(vals)
        out.append(f"{cname}_per_dispatch = {[round(x) for x in vals]}")
        out.append(f"{cname}_mean = {means[cname]:.0f}")
    if "TCC_HIT_sum" in means and "TCC_MISS_sum" in means:
        h, m = means["TCC_HIT_sum"], means["TCC_MISS_sum"]
        out.append(f"l2_hit_rate = {h / (h + m):.4f}")
    out.append(f"kernel_source_hash = {kernel_source_hash(kernel)}")
    return "\n".join(out)


def main(argv) -> str:
    last = 0
    if "--last" in argv:
        i = argv.index("--last")
        last = int(argv[i + 1])
        rest = argv[i + 2:]
        argv = argv[:i] + rest
    if argv[0] == "trace":
        return trace(argv[1], last, " ".join(argv[2:3]) if last else "")
    if argv[0] == "pmc":
        return pmc(argv[1], argv[2], argv[3], last)
    if argv[0] == "counters":
        return counters(argv[1], argv[2], argv[3:], last)
    raise SystemExit(__doc__)


if __name__ == "__main__":
    print(main(sys.argv[1:]))
