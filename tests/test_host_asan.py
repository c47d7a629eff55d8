"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Two small drivers are compiled with the sanitizers and run as subprocesses:
- tests/asan/host_tree_driver.cpp with the library's host tree build and
  walks (paper_1206_1199_amd/csrc/host_tree.cpp; g++, no device code);
- tests/asan/oracle_driver.c with the FP64 oracle (oracle/oracle.c; gcc).
A sanitizer report or a failed check ends the driver with a non-zero status.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-O1", "-g", "-fopenmp", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
       "-fno-omit-frame-pointer"]
ENV = dict(os.environ, OMP_NUM_THREADS="4", ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")


def _build_and_run(cmd, exe):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-4000:]
    r = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=600, env=ENV)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout[-4000:]


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ is not available")
def test_host_tree_and_walks_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_tree_asan")
    _build_and_run(["g++", "-std=c++17", *SAN, "-I", os.path.join(ROOT, "include"),
                    os.path.join(HERE, "asan", "host_tree_driver.cpp"),
                    os.path.join(ROOT, "paper_1206_1199_amd", "csrc", "host_tree.cpp"), "-o", exe], exe)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc is not available")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_asan")
    _build_and_run(["gcc", "-std=c11", *SAN, os.path.join(HERE, "asan", "oracle_driver.c"),
                    os.path.join(ROOT, "oracle", "oracle.c"), "-o", exe, "-lm"], exe)
