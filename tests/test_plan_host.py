"""Charge-block planner on the host (no GPU): the C++ checker in
tests/host/plan_check.cpp is compiled against csrc/plan.hip with g++ and
run. It evaluates every planned launch through its offset tables (bounds
checked) and compares the environments and the projection (pure and both
impurity placements, one chunk and several) with dense contractions, for
U(1), Z2 and trivial labels."""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2609_20536_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_charge_plans_match_dense_contractions(tmp_path):
    exe = tmp_path / "plan_check"
    cmd = ["g++", "-O2", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I", CSRC, os.path.join(HERE, "host", "plan_check.cpp"),
           "-x", "c++", os.path.join(CSRC, "plan.hip"), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-4000:]
    assert "fails 0" in r.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_charge_plans_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    """The same checker built with AddressSanitizer and UBSan (host code
    only): the planner's table construction makes no out-of-bounds access,
    use after free or undefined arithmetic on these cases."""
    exe = tmp_path / "plan_check_san"
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
           "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I", CSRC,
           os.path.join(HERE, "host", "plan_check.cpp"),
           "-x", "c++", os.path.join(CSRC, "plan.hip"), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "fails 0" in r.stdout
