"""The oracle's C code and the library's host-side input checks built with AddressSanitizer and
UndefinedBehaviorSanitizer (g++/gcc, host code only) and run on small random sets: Pass-Join
against brute force for every selection method, the banded against the full edit distance, and
good and malformed string sets through the checks every host entry point runs first."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]


@pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None,
                    reason="needs gcc and g++")
def test_oracle_and_host_checks_under_sanitizers(tmp_path):
    obj = str(tmp_path / "pj_oracle.o")
    exe = str(tmp_path / "san_driver")
    subprocess.run(["gcc", *SAN, "-std=gnu11", "-c", os.path.join(ROOT, "oracle", "pj_oracle.c"),
                    "-o", obj], check=True)
    subprocess.run(["g++", *SAN, "-std=c++17", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "sanitize", "san_driver.cpp"),
                    os.path.join(ROOT, "paper_1111_7171_amd", "csrc", "pj_validate.cpp"), obj,
                    "-o", exe, "-pthread"], check=True)
    env = dict(os.environ,
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "sanitized host checks passed" in r.stdout
