"""Builds the HIP library libsf.so in-tree for gfx950 with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = ["csrc/sf_api.hip", "csrc/sf_kernels.hip", "csrc/sf_cnn.hip", "csrc/sf_train.hip"]
LIB = os.path.join(HERE, "libsf.so")
ARCH = "gfx950"


def hipcc():
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def command(out=LIB):
    return [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
            "-shared", "-Wall", "-Wno-unused-function",
            # no packed-FP32 instructions in device code
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            # multiply-adds fused only within a source expression, so every
            # instantiation of a kernel (single frame, batched) rounds alike
            "-ffp-contract=on",
            "-I", os.path.join(ROOT, "include"),
            "-I", os.path.join(HERE, "csrc"),
            "-o", out] + [os.path.join(HERE, s) for s in SOURCES]


def build(verbose=True):
    """Compiles every HIP source into libsf.so (always recompiles)."""
    cmd = command(LIB + ".tmp")
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libsf.so")
    if verbose and res.stderr.strip():
        # keep warnings visible but short
        lines = [l for l in res.stderr.splitlines() if "warning" in l]
        for l in lines[:20]:
            print(l)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build()
