"""Builds libeselbm.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2203_12946_amd.build

Every HIP source is compiled for gfx950 only, with packed-FP32 instruction
selection disabled, to objects in parallel (the step kernel is instantiated
once per storage type in its own source), and linked into one shared
library next to this file.
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
SOURCES = ["eselbm_step.hip", "step_f64.hip", "step_f32.hip", "step_f16s.hip", "step_f32s.hip",
           "eselbm_adjoint.hip", "eselbm_api.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def flags() -> list[str]:
    return [
        "-O3", "-std=c++17", "-fPIC",
        f"--offload-arch={ARCH}",
        # no packed-FP32 instruction selection on this target
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        # hardware FP64 atomics for the diagnostic reductions
        "-munsafe-fp-atomics",
        "-Wno-unused-command-line-argument",
    ]


def build(verbose: bool = False) -> pathlib.Path:
    """Compiles every source to an object (in parallel), then links."""
    from concurrent.futures import ThreadPoolExecutor
    tmpdir = HERE / f"_build_{os.getpid()}"
    tmpdir.mkdir(exist_ok=True)
    try:
        def compile_one(src: str):
            obj = tmpdir / (pathlib.Path(src).stem + ".o")
            cmd = [hipcc(), *flags(), "-I", str(HERE.parent / "include"), "-c", str(CSRC / src), "-o", str(obj)]
            if verbose:
                print(" ".join(cmd), flush=True)
            return subprocess.run(cmd, capture_output=True, text=True), obj

        jobs = min(len(SOURCES), max(1, os.cpu_count() or 1))
        with ThreadPoolExecutor(max_workers=jobs) as ex:
            results = list(ex.map(compile_one, SOURCES))
        for res, _ in results:
            if res.returncode != 0:
                sys.stderr.write(res.stdout + res.stderr)
                raise RuntimeError("hipcc failed building libeselbm.so")
        tmp = LIB.with_suffix(".so.tmp%d" % os.getpid())
        cmd = [hipcc(), *flags(), "-shared", *[str(o) for _, o in results], "-o", str(tmp)]
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("hipcc failed linking libeselbm.so")
        os.replace(tmp, LIB)
    finally:
        shutil.rmtree(tmpdir, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
