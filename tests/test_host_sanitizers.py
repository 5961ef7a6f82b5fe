"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU):
the library's plain C++ (pattern parsing, plans, images, expected hits, the
FASTA parser) and the oracle's C, built with g++ into one checking program
(tests/sanitize/host_check.cpp) and run over seeded random and edge-case
inputs.  Any sanitizer report or failed check fails the test."""
import os
import shutil
import subprocess

import pytest

from conftest import ROOT


@pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None, reason="no host compiler")
def test_host_code_is_clean_under_asan_and_ubsan(tmp_path):
    csrc = os.path.join(ROOT, "paper_1611_06115_amd", "csrc")
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
    obj = str(tmp_path / "oracle.o")
    subprocess.check_call(["gcc", "-std=c11", "-pthread", *san, "-c", os.path.join(ROOT, "oracle", "oracle.c"),
                           "-o", obj])
    exe = str(tmp_path / "host_check")
    subprocess.check_call(["g++", "-std=c++17", "-pthread", *san, "-I", os.path.join(ROOT, "include"),
                           os.path.join(ROOT, "tests", "sanitize", "host_check.cpp"),
                           os.path.join(csrc, "plan.cpp"), os.path.join(csrc, "fasta.cpp"), obj, "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    out = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert out.returncode == 0, out.stderr[-4000:]
    assert "host check ok" in out.stdout
    assert "runtime error" not in out.stderr and "AddressSanitizer" not in out.stderr
