"""Builds libeselbm.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2203_12946_amd.build

Every HIP source is compiled for gfx950 only, with packed-FP32 instruction
selection disabled, and linked into one shared library next to this file.
"""
from __future__ import annotations

import os
import pathlib
import shutil
import subprocess
import sys

HERE = pathlib.Path(__file__).resolve().parent
CSRC = HERE / "csrc"
LIB = HERE / "libeselbm.so"
SOURCES = ["eselbm_step.hip", "eselbm_adjoint.hip", "eselbm_api.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def flags() -> list[str]:
    return [
        "-O3", "-std=c++17", "-fPIC", "-shared",
        f"--offload-arch={ARCH}",
        # no packed-FP32 instruction selection on this target
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        # hardware FP64 atomics for the diagnostic reductions
        "-munsafe-fp-atomics",
        "-Wno-unused-command-line-argument",
    ]


def build(verbose: bool = False) -> pathlib.Path:
    tmp = LIB.with_suffix(".so.tmp%d" % os.getpid())
    cmd = [hipcc(), *flags(), "-I", str(HERE.parent / "include"),
           *[str(CSRC / s) for s in SOURCES], "-o", str(tmp)]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libeselbm.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
