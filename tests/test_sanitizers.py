"""Host code under the address and undefined-behaviour sanitizers (CPU only).

Two drivers are built with gcc / g++ and -fsanitize=address,undefined and
run: tests/sanitize/oracle_driver.c over the FP64 oracle (oracle/oracle.c)
and tests/sanitize/mvc_driver.cpp over the library's host-only cover solver
and its argument checks (paper_2512_20178_amd/csrc/mvc.hpp).  Any
out-of-bounds access, use after free, leak or undefined behaviour aborts the
driver with a sanitizer report; the drivers' own checks must all pass.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _run(cmd, **kw):
    return subprocess.run(cmd, capture_output=True, text=True, timeout=300, **kw)


def _build_and_run(tmp_path, compiler, std, srcs, extra):
    if shutil.which(compiler) is None:
        pytest.skip(f"{compiler} not available")
    exe = str(tmp_path / "driver")
    b = _run([compiler, std, *SAN, *srcs, "-o", exe, *extra])
    assert b.returncode == 0, b.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="4")
    r = _run([exe], env=env)
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    assert "0 failed checks" in r.stdout
    return r.stdout


def test_oracle_under_sanitizers(tmp_path):
    out = _build_and_run(tmp_path, "gcc", "-std=c11",
                         [os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"),
                          os.path.join(ROOT, "oracle", "oracle.c")], ["-fopenmp", "-lm"])
    assert "oracle driver" in out


def test_cover_solver_under_sanitizers(tmp_path):
    out = _build_and_run(tmp_path, "g++", "-std=c++17",
                         [os.path.join(ROOT, "tests", "sanitize", "mvc_driver.cpp")], [])
    assert "mvc driver" in out
