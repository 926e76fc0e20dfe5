"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the CPU code
(no GPU): the C oracle (oracle/fe_oracle.c) and the library's host-side
algorithms (csrc/fe_hostalgo.h: candidate generation, key sorting, tiling),
each driven over random inputs by a small checker under tests/sanitize/
that also compares them with plain definitions.  Any memory error, leak or
undefined behaviour fails the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
       "-fno-omit-frame-pointer", "-Wall", "-Wextra"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _build_and_run(tmp_path, compiler, args, name):
    if shutil.which(compiler) is None:
        pytest.skip("%s not available" % compiler)
    exe = str(tmp_path / name)
    r = subprocess.run([compiler] + SAN + args + ["-o", exe], capture_output=True, text=True)
    if r.returncode != 0 and ("asan" in r.stderr or "ubsan" in r.stderr):
        pytest.skip("sanitizer runtime not available: " + r.stderr[-200:])
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    return r.stdout


def test_oracle_under_sanitizers(tmp_path):
    out = _build_and_run(tmp_path, "gcc",
                         ["-std=c11", "-fopenmp", os.path.join(ROOT, "oracle", "fe_oracle.c"),
                          os.path.join(ROOT, "tests", "sanitize", "oracle_check.c")], "oc")
    assert "all checks passed" in out


def test_host_algorithms_under_sanitizers(tmp_path):
    out = _build_and_run(tmp_path, "g++",
                         ["-std=c++17", "-pthread",
                          "-I" + os.path.join(ROOT, "paper_0905_2200_amd", "csrc"),
                          os.path.join(ROOT, "tests", "sanitize", "host_algo_check.cpp")], "hac")
    assert "all checks passed" in out
