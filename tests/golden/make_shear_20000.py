"""Writes tests/golden/shear_layer_1024_20000.json: the FP64 oracle's run of the
1024^2 doubly periodic shear layer (Sec. V B initial condition, nu = 1e-5)
over its full 20000 steps, summarised at checkpoints 1000, 2000, 5000, 10000
and 20000: mass, momentum, kinetic energy, the L2 norms of u and of rho - 1,
and rho and u at 64 seeded cells.

Calls only the oracle and the seeded input generators (about seven minutes
of host time on eight cores):

    python tests/golden/make_shear_20000.py
"""
import json
import os
import pathlib
import sys
import time

import numpy as np

ROOT = pathlib.Path(__file__).resolve().parents[2]
sys.path.insert(0, str(ROOT))

import oracle  # noqa: E402
from paper_2203_12946_amd import workloads as W  # noqa: E402

CHECKPOINTS = (1000, 2000, 5000, 10000, 20000)
NCELLS = 64
SEED = 20000


def main():
    wl = W.SHEAR_1024
    rho0, u0 = W.fields_for(wl)
    ny, nx = wl.shape
    rng = np.random.default_rng(SEED)
    cells = [(int(y), int(x)) for y, x in zip(rng.integers(0, ny, NCELLS), rng.integers(0, nx, NCELLS))]
    f = oracle.init_equilibrium(rho0, u0)
    out = {"workload": wl.name, "tau": wl.tau, "steps": list(CHECKPOINTS), "cells": cells,
           "note": "FP64 oracle (oracle/eselbm_oracle.c) from the seeded fields of workloads.fields_for",
           "checkpoints": {}}
    done = 0
    t0 = time.time()
    for c in CHECKPOINTS:
        f = oracle.step(f, c - done, wl.tau)
        done = c
        rho, u = oracle.moments(f)
        j = rho[None] * u
        out["checkpoints"][str(c)] = {
            "mass": float(rho.sum()),
            "mom": [float(v) for v in j.reshape(2, -1).sum(1)],
            "kinetic": 0.5 * float(np.sum(rho * (u * u).sum(0))),
            "u_l2": float(np.linalg.norm(u)),
            "drho_l2": float(np.linalg.norm(rho - 1.0)),
            "rho": [float(rho[y, x]) for y, x in cells],
            "u": [[float(u[0, y, x]), float(u[1, y, x])] for y, x in cells],
        }
        print(f"{c} steps, {time.time() - t0:.0f} s", flush=True)
    path = pathlib.Path(__file__).resolve().parent / "shear_layer_1024_20000.json"
    tmp = path.with_suffix(".json.tmp%d" % os.getpid())
    tmp.write_text(json.dumps(out, indent=1) + "\n")
    os.replace(tmp, path)
    print(path)


if __name__ == "__main__":
    main()
