"""Build libustat.so (HIP kernels for gfx950 + host planner + C ABI) in-tree.

Every translation unit is compiled by hipcc; packed-fp32 instruction
selection is disabled for all device code.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libustat.so")
BUILD = os.path.join(HERE, "_build")
SOURCES = ["k_rowred_mixed.hip", "k_rowred_int.hip", "k_colred_mixed.hip", "k_colred_int.hip",
           "k_rowred_f64.hip", "k_colred_fp.hip", "k_rowred_f32.hip", "k_gemm.hip", "k_reduce.hip",
           "kernels.hip", "k_lowrank.hip", "k_peak.hip", "mlp.hip", "exec.cpp", "capi.cpp", "plan.cpp",
           "lowrank.cpp", "costmodel.cpp", "profile.cpp", "inject.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
DEVICE_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
                "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "-I" + os.path.join(HERE, "..", "include")]


# Per-source code generation options: the low-rank outer-product kernel and
# the MFMA peak kernels keep their accumulators in ordinary VGPRs (no copies
# between accumulation and vector registers around every MFMA group of
# their loops).
EXTRA = {"k_lowrank.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=1"],
         "k_peak.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=1"]}


def _compile(src: str) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD, src + ".o")
    lang = ["-x", "hip"]
    cmd = [HIPCC] + lang + DEVICE_FLAGS + COMMON + EXTRA.get(src, []) + ["-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stderr)
        raise RuntimeError("compile failed: " + src)
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC] + DEVICE_FLAGS + ["-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stderr)
        raise RuntimeError("link failed")
    os.replace(tmp, LIB)
    if verbose:
        print(LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
