"""Host code of the library built with g++ under AddressSanitizer and
UndefinedBehaviorSanitizer and run without a GPU:

* the serving admission policy (``csrc/sched.h``) driven by a simulated
  executor (arena, slots, footprint budget, waiting for memory, the
  starvation rule, cancellation);
* the C ABI's argument checks, launch plans and workspace sizes over a wide
  range of shapes, against the library's own host sources (``api.cpp``,
  ``plan.cpp``, ``server.cpp``) with stand-in kernel launchers.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2512_15187_amd", "csrc")
NATIVE = os.path.join(HERE, "native")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def _build_and_run(tmp_path, name, sources, extra=()):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ is not installed")
    exe = str(tmp_path / name)
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-w", *SAN, *sources, "-o", exe, *extra]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, f"build failed:\n{' '.join(cmd)}\n{r.stderr[-4000:]}"
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, f"{name} failed:\n{r.stdout[-2000:]}\n{r.stderr[-4000:]}"
    return r.stdout


def test_sched_policy_under_sanitizers(tmp_path):
    out = _build_and_run(tmp_path, "sched_policy_test", [os.path.join(NATIVE, "sched_policy_test.cpp")])
    assert "all checks passed" in out


def test_api_checks_under_sanitizers(tmp_path):
    if not os.path.exists(os.path.join(ROCM, "include", "hip", "hip_runtime.h")):
        pytest.skip("HIP headers are not installed")
    srcs = [os.path.join(NATIVE, "api_checks_test.cpp"), os.path.join(NATIVE, "launch_stubs.cpp"),
            os.path.join(CSRC, "api.cpp"), os.path.join(CSRC, "plan.cpp"), os.path.join(CSRC, "server.cpp")]
    out = _build_and_run(tmp_path, "api_checks_test", ["-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include", *srcs],
                         extra=(f"-L{ROCM}/lib", "-lamdhip64", f"-Wl,-rpath,{ROCM}/lib", "-lpthread"))
    assert "all passed" in out
