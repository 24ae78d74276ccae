"""Build of the HIP library libvdwxc_gpu.so (gfx950) in-tree, with hipcc, and of the default
kernel-table file beside it.

    python -m paper_1703_06999_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SRC = os.path.join(PKG, "csrc", "vdwxc_gpu.hip")
DEPS = [SRC, os.path.join(PKG, "csrc", "kernels.h"), os.path.join(PKG, "csrc", "fft_lds.h"),
        os.path.join(ROOT, "include", "vdwxc_gpu.h")]
LIB_DIR = os.path.join(PKG, "lib")
LIB = os.path.join(LIB_DIR, "libvdwxc_gpu.so")

HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    return os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def build(verbose: bool = True) -> str:
    """Compile libvdwxc_gpu.so; always recompiles.  Returns the library path."""
    os.makedirs(LIB_DIR, exist_ok=True)
    tmp = LIB + ".tmp"
    cmd = [hipcc()] + HIP_FLAGS + ["-I", os.path.join(ROOT, "include"), SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(line for line in (res.stdout + res.stderr).splitlines()
                    if "packed-fp32-ops" not in line)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{out}")
    if verbose and out.strip():
        print(out)
    os.replace(tmp, LIB)
    write_default_table()
    return LIB


DEFAULT_TABLE = os.path.join(LIB_DIR, "vdw_kernel_table.vdwk")


def write_default_table() -> str:
    """The table file the library reads when vdwxc_init gets a NULL path: the package's synthetic
    kernel table (inputs.synthetic_kernel_table), next to the library."""
    sys.path.insert(0, ROOT)
    from paper_1703_06999_amd import inputs
    inputs.synthetic_kernel_table().save(DEFAULT_TABLE + ".tmp")
    os.replace(DEFAULT_TABLE + ".tmp", DEFAULT_TABLE)
    return DEFAULT_TABLE


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
