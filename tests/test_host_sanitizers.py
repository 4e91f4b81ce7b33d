"""Host code under the address and undefined-behaviour sanitizers (CPU, no GPU).

* The launch-planning arithmetic (chunking, workspace bounds, layout; csrc/rad_plan.h)
  compiled with g++ -fsanitize=address,undefined and checked by tests/planner_check.cpp.
* The whole library's host code (argument validation, planning, bindings) built with the
  host sanitizers (GPU code as usual) and driven through the C ABI by tests/test_abi.py
  in a process that preloads the sanitizer runtime; any report fails the run.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1910_10391_amd", "csrc")


def test_planner_arithmetic_under_sanitizers(tmp_path):
    exe = str(tmp_path / "planner_check")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-I", CSRC, os.path.join(ROOT, "tests", "planner_check.cpp"), "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout[-2000:], r.stderr[-2000:])
    assert r.returncode == 0 and r.stdout.strip().endswith("ok")


def test_library_host_code_under_sanitizers():
    from paper_1910_10391_amd import build
    if not os.path.exists(build.HIPCC):
        pytest.skip("hipcc not available")
    lib = build.build_sanitized()
    env = dict(os.environ, LD_PRELOAD=build.sanitizer_runtime(), ASAN_OPTIONS="detect_leaks=0",
               RAD_LIBRARY=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi.py")], capture_output=True, text=True, env=env,
                       timeout=600, cwd="/tmp")
    out = r.stdout + r.stderr
    print(out[-4000:])
    assert r.returncode == 0
    assert "runtime error" not in out and "AddressSanitizer" not in out
