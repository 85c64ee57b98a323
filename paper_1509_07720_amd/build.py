"""Build libsimproj.so and the mbench peak-measurement program for gfx950
with hipcc (in-tree, no JIT cache)."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "simproj.hip")
OUT = os.path.join(HERE, "libsimproj.so")
MBENCH_SRC = os.path.join(HERE, "csrc", "mbench.hip")
MBENCH = os.path.join(HERE, "mbench")

COMMON_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950",
    # packed FP32 instructions stay off (only the compiler's scalar/vector
    # FP32 forms are used)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]
HIPCC_FLAGS = COMMON_FLAGS + [
    "-fPIC", "-shared",
    # the machine scheduler's instruction-level-parallelism strategy: the
    # FP64 clip kernel measured 2-3 % faster with it, FP32C unchanged
    "-mllvm", "-amdgpu-sched-strategy=max-ilp",
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.isabs(c) and os.path.exists(c) or not os.path.isabs(c)):
            return c
    return "hipcc"


def build_library(out: str = OUT, extra=()) -> str:
    cmd = [hipcc(), *HIPCC_FLAGS, *extra, "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
           "-o", out + ".tmp", SRC]
    subprocess.check_call(cmd)
    os.replace(out + ".tmp", out)
    return out


KERNEL_SOURCES = ("simproj.hip", "sp_poly.h", "sp_setup.h", "sp_wave.h", "sp_corner.h")


def kernel_source_hash() -> str:
    """SHA-256 of the projection kernels' sources and compiler flags: counter
    figures taken on one version of the kernels are only valid while this
    stays the same."""
    import hashlib

    h = hashlib.sha256(" ".join(HIPCC_FLAGS).encode())
    for name in KERNEL_SOURCES:
        with open(os.path.join(HERE, "csrc", name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def build_mbench(out: str = MBENCH) -> str:
    subprocess.check_call([hipcc(), *COMMON_FLAGS, "-o", out + ".tmp", MBENCH_SRC])
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build_library())
    print(build_mbench())
