"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):

* the library's tile planner and footprint rasteriser, walked over every
  dtype, disc radius 0..123 and other windows, with every LDS and scratch
  region checked for bounds and for overlap with regions live in the same
  phase of a tile (tests/native/planner_check.cpp);
* the brute-force oracle's entry points on small ragged planes
  (tests/native/oracle_check.cpp).

The two programs are built separately: the oracle and the library share no
code."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")
CSRC = os.path.join(ROOT, "paper_2505_22938_amd", "csrc")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
SAN = ["-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
       "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


def _run(exe):
    env = dict(os.environ, ASAN_OPTIONS="abort_on_error=0:detect_leaks=1",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    return r.stdout


def test_planner_layouts_under_sanitizers(tmp_path):
    hip = os.path.join(ROCM, "lib", "libamdhip64.so")
    if not os.path.exists(hip):
        pytest.skip("needs the HIP runtime library to link the planner")
    exe = str(tmp_path / "planner_check")
    subprocess.check_call(["g++"] + SAN + [
        "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROCM, "include"), "-I", CSRC,
        os.path.join(NATIVE, "planner_check.cpp"), os.path.join(CSRC, "plan.cpp"),
        os.path.join(CSRC, "footprint.cpp"), "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
        "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-o", exe])
    out = _run(exe)
    assert " 0 failures" in out, out


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_check")
    subprocess.check_call(["g++"] + SAN + [
        "-fopenmp", os.path.join(NATIVE, "oracle_check.cpp"),
        os.path.join(ROOT, "oracle", "median_oracle.cpp"), "-o", exe])
    out = _run(exe)
    assert "0 failures" in out, out
