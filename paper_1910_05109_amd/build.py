"""Build libb64hip.so in-tree with hipcc for gfx950.

Usage: python -m paper_1910_05109_amd.build   (or call build()).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SOURCES = [os.path.join(CSRC, f) for f in ("b64_single.hip", "b64_batch.hip", "b64_validate.hip",
                                            "b64_variants.hip", "b64_fused.hip", "b64_abi.hip",
                                            "b64_pipeline.hip")]
LIB = os.path.join(HERE, "libb64hip.so")
INCLUDE = os.path.join(ROOT, "include")
ARCH = "gfx950"

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Wall", "-Wextra", "-Wno-unused-parameter",
    # no packed-FP32 instructions anywhere
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    cand = os.path.join(rocm, "bin", "hipcc")
    return cand if os.path.exists(cand) else "hipcc"


def build(extra: list[str] | None = None, out: str = LIB) -> str:
    """Compile every HIP source of the package into `out` (always recompiles)."""
    tmp = out + ".tmp"
    cmd = [hipcc(), *FLAGS, *(extra or []), *SOURCES, "-o", tmp]
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(sys.argv[1:]))
