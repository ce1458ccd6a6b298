"""Summaries of rocprofv3 result databases (kernel trace and counter runs).

    python -m paper_2608_21826_amd.profsum trace <results.db>
    python -m paper_2608_21826_amd.profsum pmc <fetch.db> <write.db> <kernel-substring>
    python -m paper_2608_21826_amd.profsum counters <db> <kernel-substring> <counter>...

`trace` prints per-kernel call counts and average / min / max durations.
`counters` prints a kernel's counter values per dispatch and their means, and
the L2 hit rate when TCC_HIT_sum and TCC_MISS_sum are among them.
`pmc` prints FETCH_SIZE and WRITE_SIZE per dispatch (KiB, as the counters
read), scales each by what the same counter reads for the calibration copy
kernel (k_probe_copy: 1 GiB read and 1 GiB written), and prints HBM bytes per
launch of the kernel named by the substring, plus the hash of the solver
sources the run was taken on.
"""
from __future__ import annotations

import collections
import hashlib
import os
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CALIB_BYTES = 1 << 30


KERNEL_SOURCES = ("bq_device.hpp", "sssp_device.hpp", "sssp_kernels.hpp")


def kernel_source_hash() -> str:
    """Hash of the sources the single-query solver kernels are built from;
    a counter summary taken on other sources no longer describes them."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(HERE, "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def _short(name: str) -> str:
    name = name.replace("(anonymous namespace)::", "")
    return name.split("(")[0] if "(" in name else name


def trace(db: str) -> str:
    c = sqlite3.connect(db)
    rows = list(c.execute("select name, duration from kernels"))
    agg = collections.defaultdict(list)
    for n, d in rows:
        agg[_short(n)].append(d)
    lines = [f"{'kernel':48s} {'calls':>6s} {'avg_us':>12s} {'min_us':>12s} {'max_us':>12s}"]
    for n, ds in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
        lines.append(f"{n[:48]:48s} {len(ds):6d} {sum(ds) / len(ds) / 1e3:12.3f} "
                     f"{min(ds) / 1e3:12.3f} {max(ds) / 1e3:12.3f}")
    return "\n".join(lines)


def _counter(db: str, cname: str):
    c = sqlite3.connect(db)
    agg = collections.defaultdict(list)
    for k, n, v in c.execute("select kernel_name, counter_name, value from counters_collection"):
        if n == cname:
            agg[_short(k)].append(float(v))
    return agg


def pmc(fetch_db: str, write_db: str, kernel: str) -> str:
    f = _counter(fetch_db, "FETCH_SIZE")
    w = _counter(write_db, "WRITE_SIZE")
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
        f"kernel_source_hash = {kernel_source_hash()}",
    ]
    return "\n".join(out)


def counters(db: str, kernel: str, names) -> str:
    """Per-dispatch values and means of counters of one kernel; with
    TCC_HIT_sum and TCC_MISS_sum also the L2 hit rate."""
    out = [f"kernel = {kernel}"]
    means = {}
    for cname in names:
        vals = [v for k, v in _counter(db, cname).items() if kernel in k][0]
        means[cname] = sum(vals) / len(vals)
        out.append(f"{cname}_per_dispatch = {[round(x) for x in vals]}")
        out.append(f"{cname}_mean = {means[cname]:.0f}")
    if "TCC_HIT_sum" in means and "TCC_MISS_sum" in means:
        h, m = means["TCC_HIT_sum"], means["TCC_MISS_sum"]
        out.append(f"l2_hit_rate = {h / (h + m):.4f}")
    out.append(f"kernel_source_hash = {kernel_source_hash()}")
    return "\n".join(out)


if __name__ == "__main__":
    if sys.argv[1] == "trace":
        print(trace(sys.argv[2]))
    elif sys.argv[1] == "pmc":
        print(pmc(sys.argv[2], sys.argv[3], sys.argv[4]))
    elif sys.argv[1] == "counters":
        print(counters(sys.argv[2], sys.argv[3], sys.argv[4:]))
    else:
        raise SystemExit(__doc__)
