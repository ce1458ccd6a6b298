"""The C-ABI library builds for gfx950, loads, and exports every entry point
that include/bq.h declares (no device calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bq.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*[A-Za-z_][\w\s\*]*?\b(\w+)\s*\([^;]*\)\s*;", text, flags=re.M)
    return sorted(set(names))


def test_header_parses():
    names = declared_functions()
    assert "sssp_bf" in names and "bq_create" in names and "bq_bench_mixed" in names


def test_library_exports_every_declared_symbol():
    import paper_2608_21826_amd as pkg
    lib = ctypes.CDLL(pkg.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"
    assert sorted(pkg.EXPORTS) == declared_functions()


def test_strerror_is_host_only():
    import paper_2608_21826_amd as pkg
    assert pkg.strerror(pkg.BQ_ERANGE).startswith("distances")
    assert pkg.strerror(pkg.BQ_OK) == "ok"


def test_built_for_gfx950():
    import paper_2608_21826_amd as pkg
    data = open(pkg.LIB_PATH, "rb").read()
    assert b"gfx950" in data


def test_no_cpu_fallback_when_library_missing(tmp_path):
    import paper_2608_21826_amd as pkg
    with pytest.raises(ImportError):
        pkg.lib(str(tmp_path / "missing.so"))


STRUCTS = [("Launch", "bq_launch"), ("BenchStats", "bq_bench_stats"), ("SsspStats", "sssp_stats"),
           ("RoundsStats", "sssp_rounds_stats"), ("Instance", "sssp_instance"),
           ("Request", "bq_request"), ("Response", "bq_response"),
           ("ServerStats", "bq_server_stats")]


def test_struct_layouts_match_the_header(tmp_path):
    """The binding's ctypes mirrors have the size and field offsets of the
    header's structs, as a C compiler lays them out."""
    import shutil
    import subprocess
    import paper_2608_21826_amd as pkg
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "bq.h"', "int main(void) {"]
    want = []
    for py, c in STRUCTS:
        cls = getattr(pkg, py)
        lines.append(f'printf("%zu\\n", sizeof({c}));')
        want.append(ctypes.sizeof(cls))
        for name, _ in cls._fields_:
            lines.append(f'printf("%zu\\n", offsetof({c}, {name}));')
            want.append(getattr(cls, name).offset)
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True,
                                          text=True).stdout.split()]
    assert got == want


def test_status_codes_match_the_header():
    """bq_status values in the header equal the binding's constants."""
    import paper_2608_21826_amd as pkg
    text = open(HEADER).read()
    body = text[text.index("typedef enum {"):text.index("} bq_status;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    vals = {k: int(v) for k, v in re.findall(r"(BQ_\w+)\s*=\s*(-?\d+)", body)}
    assert vals and all(getattr(pkg, k) == v for k, v in vals.items())
    assert len(set(vals.values())) == len(vals)
    for k in vals:
        assert pkg.strerror(vals[k]) != "unknown status", k


def test_null_handles_are_rejected_on_the_host():
    """Every entry point called with NULL pointers and zero sizes returns
    before any HIP call (so this runs without a GPU): the *_destroy calls
    accept NULL, every other call gives BQ_EINVAL."""
    import paper_2608_21826_amd as pkg
    L = pkg.lib()
    host_only = {"bq_strerror", "bq_device_cus"}
    for name in pkg.EXPORTS:
        if name in host_only:
            continue
        f = getattr(L, name)
        args = [None if (t is ctypes.c_void_p or hasattr(t, "contents")) else 0
                for t in f.argtypes]
        want = pkg.BQ_OK if name.endswith("_destroy") else pkg.BQ_EINVAL
        assert f(*args) == want, name
