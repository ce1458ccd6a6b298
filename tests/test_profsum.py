"""The rocprofv3 summary tool (paper_2608_21826_amd/profsum.py) on small
databases built here with the columns it reads: per-kernel aggregation, the
last-N selection by dispatch order, exact instantiation names, the byte
calibration against the copy kernel, and the per-kernel source hashes."""
import sqlite3

import pytest

from paper_2608_21826_amd import profsum


def _trace_db(path, rows):
    c = sqlite3.connect(path)
    c.execute("create table kernels (dispatch_id integer, name text, duration integer)")
    c.executemany("insert into kernels values (?, ?, ?)", rows)
    c.commit()
    c.close()


def _counter_db(path, rows):
    c = sqlite3.connect(path)
    c.execute("create table counters_collection (dispatch_id integer, kernel_name text, "
              "counter_name text, value real)")
    c.executemany("insert into counters_collection values (?, ?, ?, ?)", rows)
    c.commit()
    c.close()


def test_trace_aggregates_and_last(tmp_path):
    db = str(tmp_path / "t.db")
    # a search of 3 launches, then 2 timed ones, of the same kernel
    rows = [(i, "k_bench_mixed(int*)", d) for i, d in enumerate([9000, 8000, 7000, 1000, 3000])]
    rows.append((9, "void k_solve<128>(SolveArgs)", 2000))
    _trace_db(db, rows)
    out = profsum.trace(db)
    assert "k_bench_mixed" in out and " 5 " in out.splitlines()[1]
    last = profsum.main(["trace", db, "--last", "2", "k_bench_mixed"]).splitlines()
    assert len(last) == 2 and "2.000" in last[1]  # mean of 1000 and 3000 ns


def test_pmc_scales_by_the_copy_kernel_and_keeps_instantiations_apart(tmp_path):
    f, w = str(tmp_path / "f.db"), str(tmp_path / "w.db")
    gib_kib = (1 << 30) / 1024
    # FETCH_SIZE reads half of a copy's bytes, WRITE_SIZE all of them
    _counter_db(f, [(1, "k_probe_copy(long*)", "FETCH_SIZE", gib_kib / 2),
                    (2, "void k_solve<64>(SolveArgs)", "FETCH_SIZE", 999.0),
                    (3, "void k_solve<128>(SolveArgs)", "FETCH_SIZE", 100.0),
                    (4, "void k_solve<128>(SolveArgs)", "FETCH_SIZE", 300.0)])
    _counter_db(w, [(1, "k_probe_copy(long*)", "WRITE_SIZE", gib_kib),
                    (2, "void k_solve<64>(SolveArgs)", "WRITE_SIZE", 999.0),
                    (3, "void k_solve<128>(SolveArgs)", "WRITE_SIZE", 10.0),
                    (4, "void k_solve<128>(SolveArgs)", "WRITE_SIZE", 30.0)])
    rec = dict(line.split(" = ") for line in profsum.pmc(f, w, "k_solve<128>").splitlines())
    assert float(rec["fetch_scale"]) == pytest.approx(2.0)
    assert float(rec["hbm_fetch_bytes_per_launch"]) == pytest.approx(200.0 * 1024 * 2)
    assert float(rec["hbm_write_bytes_per_launch"]) == pytest.approx(20.0 * 1024)
    last = dict(line.split(" = ") for line in
                profsum.main(["pmc", f, w, "k_solve<128>", "--last", "1"]).splitlines())
    assert float(last["hbm_fetch_bytes_per_launch"]) == pytest.approx(300.0 * 1024 * 2)


def test_counters_l2_rate(tmp_path):
    db = str(tmp_path / "c.db")
    _counter_db(db, [(1, "k_bsolve", "TCC_HIT_sum", 30.0), (1, "k_bsolve", "TCC_MISS_sum", 10.0),
                     (2, "k_bsolve", "TCC_HIT_sum", 50.0), (2, "k_bsolve", "TCC_MISS_sum", 10.0)])
    out = profsum.counters(db, "k_bsolve", ["TCC_HIT_sum", "TCC_MISS_sum"])
    assert "l2_hit_rate = 0.8000" in out
    assert f"kernel_source_hash = {profsum.kernel_source_hash('k_bsolve')}" in out


def test_source_hashes_follow_the_kernel():
    h = profsum.kernel_source_hash
    assert h() == h("k_solve<128>") == h("k_solve<64>")
    assert len({h(), h("k_bsolve"), h("k_bench_mixed")}) == 3


def test_source_hash_ignores_comments_not_code():
    code = profsum._code_of
    a = "int f(int x) {  // doubles\n  return 2 * x; /* the\n value */ }\n"
    b = "int f(int x) {\n    return 2 * x;\n}\n"
    c = "int f(int x) { return 3 * x; }"
    assert code(a) == code(b)
    assert code(a) != code(c)
