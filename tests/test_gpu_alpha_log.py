"""Per-step path-length statistics of the 64^2 D2Q9 Taylor-Green workload
(FP64, 1000 steps; the workload logs alpha statistics every step) against
the oracle stepped one step at a time: every step's alpha min/max/mean over
the cells, the gated and guarded counts, mass, kinetic energy and H.
"""
import io
import json
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2203_12946_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def es():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2203_12946_amd import eselbm
    return eselbm


def test_tgv64_alpha_log_every_step(es):
    from paper_2203_12946_amd import alpha_log
    wl = W.TGV2D_64
    buf = io.StringIO()
    recs, wall = alpha_log.run(wl, "f64", wl.steps, with_H=True, out=buf)
    lines = buf.getvalue().splitlines()
    assert len(recs) == len(lines) == wl.steps
    assert json.loads(lines[-1])["step"] == wl.steps
    rho, u = W.fields_for(wl)
    f = oracle.init_equilibrium(rho, u)
    worst = {"alpha": 0.0, "mass": 0.0, "ke": 0.0, "H": 0.0}
    for rec in recs:
        f, alpha, (ngated, nguard, _) = oracle.step(f, 1, wl.tau, want_alpha=True)
        r, v = oracle.moments(f)
        ke = 0.5 * float(np.sum(r * (v ** 2).sum(0)))
        H = oracle.H(f)
        assert rec["n_cells"] == alpha.size and rec["n_nonpos"] == 0
        assert rec["n_gated"] == ngated and rec["n_guard"] == nguard, rec["step"]
        assert rec["n_alpha_lt2"] == int(np.sum(alpha < 2.0)), rec["step"]
        da = max(abs(rec["alpha_min"] - alpha.min()), abs(rec["alpha_max"] - alpha.max()),
                 abs(rec["alpha_mean"] - alpha.mean()))
        worst["alpha"] = max(worst["alpha"], da)
        worst["mass"] = max(worst["mass"], abs(rec["mass"] - r.sum()) / r.sum())
        worst["ke"] = max(worst["ke"], abs(rec["kinetic"] - ke) / ke)
        worst["H"] = max(worst["H"], abs(rec["H"] - H) / abs(H))
    print(f"[alpha log {wl.name} f64, {wl.steps} steps, {wall:.2f} s] worst per-step differences {worst}; "
          f"last step alpha in [{recs[-1]['alpha_min']:.8f}, {recs[-1]['alpha_max']:.8f}], "
          f"gated {recs[-1]['n_gated']}/{recs[-1]['n_cells']}", file=sys.stderr, flush=True)
    assert worst["alpha"] <= 1e-9
    assert worst["mass"] <= 1e-13
    assert worst["ke"] <= 1e-9
    assert worst["H"] <= 1e-12
    # the kinetic energy decays (nu = 0.01) and H never increases
    assert recs[-1]["kinetic"] < recs[0]["kinetic"]
    assert all(b["H"] <= a["H"] + 1e-12 * abs(a["H"]) for a, b in zip(recs, recs[1:]))
