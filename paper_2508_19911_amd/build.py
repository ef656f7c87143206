"""Build libcgks.so (hand-written HIP for gfx950) in-tree with hipcc.

    python -m paper_2508_19911_amd.build

Regenerates the reconstruction tables when their generator changed, then compiles
``csrc/cgks_api.hip`` into ``paper_2508_19911_amd/libcgks.so``.  Packed FP32 instructions are
disabled (-packed-fp32-ops); no fast-math.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcgks.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("CGKS_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def generate_tables(force: bool = False) -> None:
    tables = os.path.join(CSRC, "recon_tables.hpp")
    gen = os.path.join(HERE, "gen_recon.py")
    if force or not os.path.exists(tables) or os.path.getmtime(tables) < os.path.getmtime(gen):
        from . import gen_recon
        gen_recon.main()


def count_flops(verbose: bool = True) -> dict:
    """Compile csrc/flopcount.hip (host program over the device templates), run it, write flops.json."""
    import json
    bdir = os.path.join(os.path.dirname(HERE), "_build")
    os.makedirs(bdir, exist_ok=True)
    exe = os.path.join(bdir, "flopcount")
    cmd = [HIPCC, "-O1", "-std=c++17", f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-o", exe, os.path.join(CSRC, "flopcount.hip")]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True, capture_output=not verbose)
    out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    counts = json.loads(out)
    with open(os.path.join(HERE, "flops.json"), "w") as f:
        json.dump(counts, f, indent=1, sort_keys=True)
        f.write("\n")
    return counts


def build(verbose: bool = True, extra=None) -> str:
    generate_tables()
    src = os.path.join(CSRC, "cgks_api.hip")
    cmd = [HIPCC] + FLAGS + (extra or []) + ["-o", LIB + ".tmp", src]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    count_flops(verbose)
    return LIB


if __name__ == "__main__":
    extra = sys.argv[1:]
    build(extra=extra)
