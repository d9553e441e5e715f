"""Builds the gfx950 library ``libbbe.so`` from ``csrc/`` with hipcc.

Flags: every arithmetic step of the race model is one IEEE single-precision
rounding, so no contraction into fused multiply-add (-ffp-contract=off) and
no fast-math; packed-FP32 instructions are disabled.
"""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libbbe.so")
SOURCES = ["race_kernels.hip", "race_kernels_paced.hip", "batch_kernels.hip",
           "batch_kernels_paced.hip", "mlp_kernels.hip", "order_kernels.hip",
           "bettor_kernels.hip", "bbe_api.hip", "bbe_batch.hip", "bbe_mlp.hip",
           "bbe_bettors.hip"]
ARCH = os.environ.get("BBE_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def kernel_hash() -> str:
    """Hash of the kernel sources (keys the persistent tuning cache)."""
    import hashlib
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".hpp")):
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def compile_flags() -> list[str]:
    return [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
            "-fno-fast-math", "-fvisibility=hidden", "-Wall",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            f'-DBBE_KERNEL_HASH="{kernel_hash()}"',
            "-I", INCLUDE, "-I", CSRC]


def build(verbose: bool = False, extra: list[str] | None = None, out: str = LIB) -> str:
    """Compile every source and link ``libbbe.so`` (always recompiles)."""
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    objs = [os.path.join(build_dir, src.replace(".hip", ".o")) for src in SOURCES]

    def compile_one(src, obj):
        cmd = [hipcc(), *compile_flags(), *(extra or []), "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)

    # one compiler process per source, a few at a time
    workers = max(1, min(len(SOURCES), os.cpu_count() or 1, 8))
    with concurrent.futures.ThreadPoolExecutor(workers) as pool:
        for f in [pool.submit(compile_one, s, o) for s, o in zip(SOURCES, objs)]:
            f.result()
    tmp = out + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
