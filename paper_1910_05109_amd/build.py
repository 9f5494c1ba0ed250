"""Build libb64hip.so in-tree with hipcc for gfx950, and its CPython
fast-call binding (_b64fast) with the host C compiler.

Usage: python -m paper_1910_05109_amd.build   (or call build()).
"""
from __future__ import annotations

import os
import subprocess
import sys
import sysconfig
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SOURCES = [os.path.join(CSRC, f) for f in ("b64_single.hip", "b64_batch.hip", "b64_validate.hip",
                                            "b64_variants.hip", "b64_fused.hip", "b64_abi.hip",
                                            "b64_pipeline.hip", "b64_serve.hip",
                                            "b64_yardstick.hip")]
LIB = os.path.join(HERE, "libb64hip.so")
FAST = os.path.join(HERE, "_b64fast" + (sysconfig.get_config_var("EXT_SUFFIX") or ".so"))
INCLUDE = os.path.join(ROOT, "include")
ARCH = "gfx950"

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Wall", "-Wextra", "-Wno-unused-parameter",
    # no packed-FP32 instructions anywhere
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    cand = os.path.join(rocm, "bin", "hipcc")
    return cand if os.path.exists(cand) else "hipcc"


def build(extra: list[str] | None = None, out: str = LIB, jobs: int | None = None) -> str:
    """Compile every HIP source of the package into `out` (always recompiles):
    one object per source, compiled in parallel, then linked."""
    extra = list(extra or [])
    jobs = jobs or min(len(SOURCES), max(1, min(os.cpu_count() or 1, 8)))
    with tempfile.TemporaryDirectory(prefix="b64hip_build_") as tmpdir:
        objs = [os.path.join(tmpdir, os.path.basename(src) + ".o") for src in SOURCES]

        def compile_one(pair):
            src, obj = pair
            subprocess.check_call([hipcc(), *FLAGS, *extra, "-c", src, "-o", obj])

        with ThreadPoolExecutor(max_workers=jobs) as pool:
            list(pool.map(compile_one, zip(SOURCES, objs)))
        tmp = out + ".tmp"
        subprocess.check_call([hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *extra,
                               *objs, "-o", tmp])
    os.replace(tmp, out)
    if out == LIB:
        build_fast()
    return out


def build_fast() -> str:
    """The CPython fast-call binding (csrc/b64_pyfast.c), compiled for the host
    with the interpreter's own headers; it needs libb64hip.so only at run time
    (the ctypes binding hands it the entry points)."""
    py_inc = sysconfig.get_paths()["include"]
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    tmp = FAST + ".tmp"
    subprocess.check_call([os.environ.get("CC", "gcc"), "-O2", "-shared", "-fPIC", "-Wall", "-Wextra",
                           "-Wno-unused-parameter", "-D__HIP_PLATFORM_AMD__",
                           f"-I{py_inc}", f"-I{INCLUDE}", f"-I{os.path.join(rocm, 'include')}",
                           os.path.join(CSRC, "b64_pyfast.c"), "-o", tmp])
    os.replace(tmp, FAST)
    return FAST


if __name__ == "__main__":
    print(build(sys.argv[1:]))
