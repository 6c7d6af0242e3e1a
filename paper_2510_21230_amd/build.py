"""Build libatm3.so (HIP, gfx950) in-tree with hipcc.

Every translation unit is compiled for gfx950 with packed FP32 instructions
disabled; the binning unit additionally with -ffp-contract=off (its FP64 cell
decisions must equal the plain C expression bit for bit).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libatm3.so")
BUILD = os.path.join(ROOT, "_build")

SOURCES = {
    "atm3_api.hip": [],
    "atm3_binning.hip": ["-ffp-contract=off"],
    "atm3_forces.hip": [],
    "atm3_surrogate.hip": [],
    "atm3_md.hip": [],
    "atm3_variants.hip": [],
}

COMMON = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # atomics of a wave to one address: a DPP wave reduction and one atomic,
    # not a loop over the active lanes
    "-mllvm", "-amdgpu-atomic-optimizer-strategy=DPP",
    "-Wall", "-Wno-unused-function",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def hipcc() -> str:
    return os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    procs = []
    for src, extra in SOURCES.items():
        obj = os.path.join(BUILD, src.replace(".hip", ".o"))
        cmd = [hipcc(), "-c", os.path.join(CSRC, src), "-o", obj] + COMMON + extra
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
    for src, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            sys.stderr.write(out.decode(errors="replace"))
            raise RuntimeError(f"hipcc failed on {src}")
        elif verbose and out:
            sys.stderr.write(out.decode(errors="replace"))
    tmp = OUT + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs
    subprocess.check_call(cmd)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
