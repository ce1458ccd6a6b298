"""Host-only code under the sanitizers (CPU, no GPU): the Broker Queue's
host model (oracle/queue_cpu.c, C11 atomics on threads) under
ThreadSanitizer, and the served engine's admission arena
(paper_2608_21826_amd/csrc/arena_host.hpp) under AddressSanitizer and
UndefinedBehaviorSanitizer. Each is built with its own driver
(tests/sanitize/) that checks results too; a sanitizer report fails the
test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")


def _build(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip(f"sanitizer build not available: {r.stderr[-300:]}")


def _run(exe, env_extra):
    env = dict(os.environ, **env_extra)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    report = r.stdout + r.stderr
    assert r.returncode == 0, report[-3000:]
    assert "Sanitizer" not in report and "runtime error" not in report, report[-3000:]
    return report


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no gcc")
def test_queue_model_under_thread_sanitizer(tmp_path):
    exe = str(tmp_path / "queue_tsan")
    _build(["gcc", "-O1", "-g", "-std=c11", "-fsanitize=thread", "-pthread", "-D_GNU_SOURCE",
            os.path.join(ROOT, "oracle", "queue_cpu.c"), os.path.join(SAN, "queue_main.c"),
            "-o", exe])
    out = _run(exe, {"TSAN_OPTIONS": "halt_on_error=1 exitcode=66"})
    assert "queue model ok" in out


@pytest.mark.skipif(shutil.which("g++") is None, reason="no g++")
def test_arena_under_address_sanitizer(tmp_path):
    exe = str(tmp_path / "arena_asan")
    _build(["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
            "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "include"),
            "-I", os.path.join(ROOT, "paper_2608_21826_amd", "csrc"),
            os.path.join(SAN, "arena_main.cpp"), "-o", exe])
    out = _run(exe, {"ASAN_OPTIONS": "detect_leaks=1 halt_on_error=1"})
    assert "arena ok" in out
