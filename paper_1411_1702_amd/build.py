"""Build the HIP library (gfx950) in-tree: paper_1411_1702_amd/libpf_hip.so."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpf_hip.so")
SOURCES = ["pf_runtime.hip", "pf_server.cpp"]
DEPS = ["pf_runtime.hip", "pf_kernels.hip", "pf_advdiff.hip", "pf_device.hpp", "pf_types.hpp", "pf_server.cpp"]
ARCH = os.environ.get("PF_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed FP32 instructions: some of their forms have given wrong
    # results on this target without any error
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def build(verbose: bool = False, extra_flags=None) -> str:
    """Compile every HIP source into one shared library; always rebuilds."""
    tmp = LIB + ".tmp"
    cmd = [hipcc()] + HIPCC_FLAGS + list(extra_flags or []) + ["-o", tmp] + \
        [os.path.join(CSRC, s) for s in SOURCES]
    res = subprocess.run(cmd, cwd=CSRC, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed")
    if verbose:
        sys.stderr.write("\n".join(l for l in res.stderr.splitlines() if "packed-fp32" not in l))
    os.replace(tmp, LIB)
    return LIB


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(os.path.join(CSRC, d)) > t for d in DEPS)


if __name__ == "__main__":
    print(build(verbose=True))
