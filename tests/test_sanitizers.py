"""AddressSanitizer + UndefinedBehaviorSanitizer builds of the host code
(CPU only): the oracle (oracle/oracle.c) and the library's host setup
(csrc/setup.cpp + csrc/common.cpp), each linked with a driver that calls
every entry point on small inputs (tests/sanitize/).  The sanitizers abort on
the first out-of-bounds access, use after free, leak or undefined operation;
the drivers check the return codes.  Built with gcc/g++ only (no device code).
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2")


def _build_and_run(tmp_path, cmd, exe):
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    return r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    cmd = ["gcc", "-std=c99", "-fopenmp"] + SAN + [
        os.path.join(HERE, "oracle_driver.c"), os.path.join(ROOT, "oracle", "oracle.c"),
        "-o", exe, "-lm"]
    assert "oracle driver ok" in _build_and_run(tmp_path, cmd, exe)


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_host_setup_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "setup_driver")
    csrc = os.path.join(ROOT, "paper_2103_07329_amd", "csrc")
    cmd = ["g++", "-std=c++17"] + SAN + [
        "-I" + os.path.join(ROOT, "include"), "-I" + csrc,
        os.path.join(HERE, "setup_driver.cpp"), os.path.join(csrc, "setup.cpp"),
        os.path.join(csrc, "common.cpp"), "-o", exe]
    assert "setup driver ok" in _build_and_run(tmp_path, cmd, exe)
