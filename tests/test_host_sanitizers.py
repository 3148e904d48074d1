"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU
only): the oracle's C code, and the library's host-side canonicaliser,
result aggregation, tensor-train decomposition and blocked-annealer work
schedule, each driven over seeded random inputs by a small driver
(tests/sanitize/); any sanitizer report, failed check or non-zero exit fails
the test.  Built with gcc / g++, no device code."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None or shutil.which("g++") is None,
                                reason="needs gcc and g++")


def _run(cmd, tmp_path):
    r = subprocess.run(cmd, capture_output=True, text=True, cwd=tmp_path)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", *SAN, os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(HERE, "sanitize", "oracle_driver.c"),
          "-o", exe, "-lm"], tmp_path)
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV)
    assert r.returncode == 0 and "ERROR" not in r.stderr and "runtime error" not in r.stderr, r.stdout + r.stderr


def test_library_host_code_under_sanitizers(tmp_path):
    csrc = os.path.join(ROOT, "paper_2407_19987_amd", "csrc")
    exe = str(tmp_path / "host_driver")
    _run(["g++", "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I", csrc,
          os.path.join(csrc, "canon.cpp"), os.path.join(csrc, "results.cpp"), os.path.join(csrc, "tt.cpp"),
          os.path.join(HERE, "sanitize", "host_driver.cpp"), "-o", exe], tmp_path)
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV)
    assert r.returncode == 0 and "ERROR" not in r.stderr and "runtime error" not in r.stderr, r.stdout + r.stderr


def test_block_schedule_under_sanitizers(tmp_path):
    csrc = os.path.join(ROOT, "paper_2407_19987_amd", "csrc")
    exe = str(tmp_path / "schedule_driver")
    _run(["g++", "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I", csrc,
          os.path.join(csrc, "schedule.cpp"), os.path.join(HERE, "sanitize", "schedule_driver.cpp"), "-o", exe],
         tmp_path)
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV)
    assert r.returncode == 0 and "ERROR" not in r.stderr and "runtime error" not in r.stderr, r.stdout + r.stderr
