"""Compile the HIP library (gfx950) in-tree: paper_2201_04622_amd/libeamfe.so."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libeamfe.so")
SOURCES = [os.path.join(HERE, "csrc", n) for n in ("eamfe_kernels.hip", "eamfe_barostat.hip", "eamfe_host.cpp")]
HEADERS = [os.path.join(HERE, "csrc", "eamfe_internal.h"), os.path.join(ROOT, "include", "eamfe.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed-FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # multiply-adds fused only within one source expression: the same
    # expression then compiles to the same rounding wherever it is inlined
    "-ffp-contract=on",
    "-I", os.path.join(ROOT, "include"),
]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS]
    for s in SOURCES:
        cmd += ["-x", "hip", s]
    cmd += ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l]
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + "\n".join(msgs))
    if verbose and msgs:
        print("\n".join(msgs))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
