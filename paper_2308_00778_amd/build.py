"""Build liblsqr.so (the HIP library behind include/lsqr.h) in place for gfx950."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "liblsqr.so")
SOURCES = [os.path.join(HERE, "csrc", "lsqr.hip")]
DEPENDS = SOURCES + [os.path.join(HERE, "csrc", "kernels.hpp"),
                     os.path.join(ROOT, "include", "lsqr.h")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-munsafe-fp-atomics",
    # no packed-FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


# Streaming read/write/copy kernels that measure the practical HBM ceiling
# (benchmark only; the solver library does not use them)
STREAM_LIB = os.path.join(HERE, "libstreamceil.so")
STREAM_SOURCES = [os.path.join(HERE, "csrc", "stream_ceiling.hip")]


def build(verbose: bool = False, extra: list[str] | None = None) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    cmd = [hipcc, *HIPCC_FLAGS, *(extra or []), "-I", os.path.join(ROOT, "include"),
           "-o", LIB + ".tmp", *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    cmd = [hipcc, *HIPCC_FLAGS, "-o", STREAM_LIB + ".tmp", *STREAM_SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(STREAM_LIB + ".tmp", STREAM_LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
