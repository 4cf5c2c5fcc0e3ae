"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

- The engine's host sources (planner, executor's dry schedules, C ABI)
  are compiled with the sanitizers on their host code only (hipcc's
  -Xarch_host), linked with the regular device objects, and driven by
  tests/native/sanitize_plan.cpp: plan creation over several graphs,
  precisions, orders and options, every query, the argument checks, and
  host allocation failures injected at every point of a plan creation.
- The oracle's C routines are compiled with the same sanitizers (gcc)
  and driven by tests/native/sanitize_oracle.c.
Any sanitizer report fails the run (halt_on_error).
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2508_12627_amd", "csrc")
OBJ = os.path.join(ROOT, "paper_2508_12627_amd", "_build")
HIPCC = "/opt/rocm/bin/hipcc"
SAN_ENV = {"ASAN_OPTIONS": "halt_on_error=1:detect_leaks=0:verify_asan_link_order=0",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, (" ".join(cmd), r.stdout[-3000:], r.stderr[-3000:])
    return r


@pytest.mark.slow
def test_planner_and_abi_under_sanitizers(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    device_objs = [os.path.join(OBJ, f) for f in sorted(os.listdir(OBJ))
                   if f.endswith(".hip.o")] if os.path.isdir(OBJ) else []
    if not device_objs:
        pytest.skip("engine not built (run build() first)")
    host = ["plan.cpp", "costmodel.cpp", "profile.cpp", "exec.cpp", "capi.cpp", "inject.cpp",
            "lowrank.cpp"]
    flags = ["-x", "hip", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I" + os.path.join(ROOT, "include")]
    objs = []
    for src in host:
        o = str(tmp_path / (src + ".o"))
        _run([HIPCC] + flags + ["-c", os.path.join(CSRC, src), "-o", o])
        objs.append(o)
    drv = str(tmp_path / "drv.o")
    _run([HIPCC, "-O1", "-g", "-std=c++17", "-fsanitize=address", "-fsanitize=undefined",
          "-I" + os.path.join(ROOT, "include"), "-c",
          os.path.join(ROOT, "tests", "native", "sanitize_plan.cpp"), "-o", drv])
    exe = str(tmp_path / "sanitize_plan")
    _run([HIPCC, "--offload-arch=gfx950", "-fsanitize=address", "-fsanitize=undefined", "-o", exe,
          drv] + objs + device_objs)
    env = dict(os.environ, **SAN_ENV)
    r = _run([exe], env=env, timeout=600)
    assert "0 failures" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr


def test_oracle_under_sanitizers(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    exe = str(tmp_path / "sanitize_oracle")
    _run(["gcc", "-O1", "-g", "-fopenmp", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
          "-o", exe, os.path.join(ROOT, "tests", "native", "sanitize_oracle.c"),
          os.path.join(ROOT, "oracle", "oracle.c")])
    env = dict(os.environ, OMP_NUM_THREADS="4", **SAN_ENV)
    r = _run([exe], env=env, timeout=300)
    assert "0 failures" in r.stdout
    assert "runtime error" not in r.stderr
