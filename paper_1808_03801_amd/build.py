"""Builds libusp.so (gfx950 HIP kernels + C-ABI runtime) in the package tree."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libusp.so")
ARCH = os.environ.get("USP_OFFLOAD_ARCH", "gfx950")

FLAGS = ["-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
         # no implicit FMA contraction: results must not depend on which
         # kernel instantiation (particles per thread) ran a cell
         "-ffp-contract=off",
         # packed FP32 instructions stay off (see the design notes)
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(HERE, "..", "include")]


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, f) for f in ("usp_cell.hip", "usp_kernels.hip", "usp_runtime.hip")]
    cmd = ["hipcc", *FLAGS, *srcs, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stdout + r.stderr)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
