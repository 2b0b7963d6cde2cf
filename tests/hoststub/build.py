"""Build the library's host code against the CPU stand-in runtime
(hip_stub.cpp) into a shared library, with g++ (no GPU, no hipcc)."""
from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2608_03778_amd", "csrc")
HOST_SOURCES = ["dp_api.cpp", "dp_compile.cpp", "dp_cells.cpp", "dp_server.cpp"]


def available() -> bool:
    return shutil.which("g++") is not None and os.path.exists("/opt/rocm/include/hip/hip_runtime.h")


def build(out_dir: str) -> str:
    out = os.path.join(out_dir, "libdp_stub.so")
    kernels_h = os.path.join(CSRC, "dp_kernels.h")
    abi_h = os.path.join(ROOT, "include", "diffpower.h")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fPIC", "-shared", "-D__HIP_PLATFORM_AMD__",
           "-I/opt/rocm/include", f'-DDP_KERNELS_H="{kernels_h}"', f'-DDP_ABI_H="{abi_h}"',
           "-o", out,
           os.path.join(HERE, "hip_stub.cpp")] + [os.path.join(CSRC, s) for s in HOST_SOURCES]
    cmd += ["-lpthread"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return out
