"""Build libmhd.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libmhd.so")
SOURCES = ["mhd_kernels.hip", "mhd_flux.hip", "mhd_mlp.hip", "mhd_gravity.hip", "mhd_nbody.hip",
           "mhd_abi.hip"]
HEADERS = ["mhd_kernels.hpp", "mhd_physics.hpp", "mhd_mlp.hpp", "mhd_span.hpp"]
ARCH = os.environ.get("MHD_OFFLOAD_ARCH", "gfx950")

# Packed FP32 instructions are disabled: the compiler would otherwise form
# v_pk_* from ordinary float code.
HIPCC_FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics", "-Wall",
    # matrix-core results in ordinary VGPRs rather than accumulation
    # registers: the in-step MLP would otherwise copy every result out
    # before its activation (36 extra instructions per 16 samples)
    "-mllvm", "-amdgpu-mfma-vgpr-form=1",
]


# roctx: the step's host-side ranges (rocprofv3 --marker-trace)
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
LINK_FLAGS = ["-L" + os.path.join(ROCM, "lib"), "-Wl,-rpath," + os.path.join(ROCM, "lib"),
              "-lrocprofiler-sdk-roctx"]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc, *HIPCC_FLAGS, "-I", INCLUDE, "-I", CSRC,
           *[os.path.join(CSRC, s) for s in SOURCES], *LINK_FLAGS, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
