"""Builds libdrtopk.so in place with hipcc for gfx950 (no GPU needed)."""
from __future__ import annotations

import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libdrtopk.so")
CSRC = os.path.join(HERE, "csrc")
# host API + batched kernels, the serving dispatcher, and one translation unit
# per key codec of the single-problem path (compiled in parallel)
SOURCES = [os.path.join(CSRC, "drtopk.hip"), os.path.join(CSRC, "server.cpp"), os.path.join(CSRC, "wide.hip")] + sorted(
    os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.startswith("codec_") and f.endswith(".hip"))
HEADERS = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h"))
HEADERS.append(os.path.join(ROOT, "include", "drtopk.h"))
BUILD_DIR = os.path.join(HERE, "_build")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed fp32 instructions in the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build(verbose: bool = False, jobs: int | None = None) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(BUILD_DIR, exist_ok=True)
    tag = f".{os.getpid()}"
    objs = [os.path.join(BUILD_DIR, os.path.basename(src) + tag + ".o") for src in SOURCES]

    def compile_one(i: int) -> None:
        cmd = [hipcc, *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), "-c", "-o", objs[i], SOURCES[i]]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)

    jobs = jobs or min(len(SOURCES), max(1, os.cpu_count() or 1), 16)
    try:
        with ThreadPoolExecutor(max_workers=jobs) as pool:
            list(pool.map(compile_one, range(len(SOURCES))))
        tmp = LIB + f".tmp{os.getpid()}"
        cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    finally:
        for o in objs:
            if os.path.exists(o):
                os.remove(o)
    return LIB


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(f) > t for f in SOURCES + HEADERS)


if __name__ == "__main__":
    print(build(verbose=True))
