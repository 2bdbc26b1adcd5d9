"""Per-step path-length statistics of a run, as JSON lines.

The 64^2 D2Q9 Taylor-Green workload logs the statistics of alpha after every
step.  Each step runs with the fused FP64 diagnostics of eselbm_alpha_stats
on: alpha min/max/mean over the collided cells, the gated, guarded, exact-path
and alpha < 2 counts, mass, momentum, kinetic energy and, optionally, the H
function of the step's output state (Eq. hdef).

    python -m paper_2203_12946_amd.alpha_log [--workload d2q9_tgv_64] [--dtype f64]
                                             [--steps 1000] [--no-H] [--out FILE]

Every computation runs in the HIP library; this module only steps the
solver and writes one JSON object per step.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import torch

from . import eselbm as es
from . import workloads as W

_KEYS = ("alpha_min", "alpha_max", "alpha_mean", "n_cells", "n_gated", "n_guard", "n_alpha_lt2", "n_exact",
         "n_nonpos", "mass", "mom", "kinetic", "H")


def run(wl: W.Workload, dtype: str = "f64", steps: int | None = None, with_H: bool = True, out=None,
        mode: str = "higher") -> tuple[list[dict], float]:
    """Steps workload ``wl`` one step at a time with statistics on; returns
    (records, wall seconds) and writes each record as a JSON line to the
    text stream ``out`` if given."""
    nsteps = wl.steps if steps is None else int(steps)
    rho, u = W.fields_for(wl)
    s = es.Solver(wl.lattice, wl.shape, dtype=dtype, mode=mode)
    a = s.init_equilibrium(torch.from_numpy(rho).cuda(), torch.from_numpy(u).cuda())
    b = s.empty_state()
    s.set_stats(True)
    recs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for n in range(1, nsteps + 1):
        s.step(a, b, 1, wl.tau)
        a, b = b, a
        st = s.stats(with_H=with_H)
        rec = {"step": n}
        rec.update({k: st[k] for k in _KEYS})
        if not with_H:
            rec.pop("H")
        recs.append(rec)
        if out is not None:
            out.write(json.dumps(rec) + "\n")
        if st["n_nonpos"]:
            break
    wall = time.perf_counter() - t0
    return recs, wall


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--workload", default=W.TGV2D_64.name)
    ap.add_argument("--dtype", default="f64")
    ap.add_argument("--mode", default="higher")
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--no-H", action="store_true")
    ap.add_argument("--out", default="-")
    args = ap.parse_args()
    wl = {w.name: w for w in (W.TGV2D_64, W.SHEAR_1024, W.TGV3D_256, W.ADJ2D_256, W.ADJ3D_128)}[args.workload]
    torch.cuda.set_device(0)
    if args.out == "-":
        run(wl, args.dtype, args.steps, not args.no_H, sys.stdout, args.mode)
    else:
        with open(args.out, "w") as fh:
            run(wl, args.dtype, args.steps, not args.no_H, fh, args.mode)


if __name__ == "__main__":
    main()
