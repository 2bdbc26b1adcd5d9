"""Mutation check of the oracle's pins.

Each case plants one plausible mistake in a copy of the oracle's C source (a
wrong sign, coefficient, index or dropped term, of the kind a transcription
of the paper could make), builds that copy, and runs the CPU pin suites
against it in a child process.  At least one pin must fail for every
mutant: a mutant that survives would mean that part of the oracle is not
pinned.  Only the copy is broken; the oracle itself is untouched."""
import os
import pathlib
import subprocess
import sys

import pytest

ROOT = pathlib.Path(__file__).resolve().parents[1]
SRC = ROOT / "oracle" / "eselbm_oracle.c"

SUITES = ("tests/test_oracle_pins.py", "tests/test_oracle_adjoint_ref.py")
PINS_ONLY = ("tests/test_oracle_pins.py",)

# (name, original text, mutated text[, suites]): the original must occur in
# the source; the first occurrence is replaced.  The suites default to both
# pin files.
MUTANTS = [
    ("weights", "return c == 0 ? 2.0 / 3.0 : 1.0 / 6.0;", "return c == 0 ? 1.0 / 2.0 : 1.0 / 4.0;"),
    ("equilibrium z", "z[a] = (2.0 * u[a] + s) / (1.0 - u[a]);", "z[a] = (2.0 * u[a] + s) / (1.0 + u[a]);"),
    ("equilibrium Upsilon", "ups[a] = 2.0 - s;", "ups[a] = 1.0;"),
    ("velocity", "u[a] = j[a] / r;", "u[a] = j[a];"),
    ("departure", "x[i] = feq[i] / g[i] - 1.0; /* Eq. xdef */", "x[i] = g[i] / feq[i] - 1.0;"),
    ("gate", "if (xmax_abs < 1.0e-3) {", "if (xmax_abs < 1.0e-2) {"),
    ("a1", "if (x[i] < 0.0) a1 += g[i] * x[i] * x[i] * x[i] / 2.0;\n            b1",
     "if (x[i] < 0.0) a1 += g[i] * x[i] * x[i] * x[i] / 3.0;\n            b1"),
    ("c1", "c1 += g[i] * 2.0 * x[i] * x[i] / (2.0 + x[i]);\n        }\n        double aL",
     "c1 += g[i] * 2.0 * x[i] * x[i] / (2.0 - x[i]);\n        }\n        double aL"),
    ("conjugate root", "return 2.0 * c / (b + sqrt(b * b - 4.0 * a * c));",
     "return 2.0 * c / (b + sqrt(b * b - 2.0 * a * c));"),
    ("b Omega+ term", "(2.0 / (4.0 + aL * xi) +", "(1.0 / (4.0 + aL * xi) +"),
    ("c rational", "60.0 * xi * xi * xi + 11.0", "66.0 * xi * xi * xi + 11.0"),
    ("a of alpha_Higher", "h * beta * x4 / 12.0", "h * beta * x4 / 10.0"),
    ("guard", "alpha = (1.0 + amax) / 2.0;", "alpha = amax;"),
    ("beta", "double beta = 1.0 / (2.0 * tau + 1.0);", "double beta = 1.0 / (2.0 * tau + 0.5);"),
    ("relaxation", "nxt[(long long)i * N + cell] = g[i] + alpha * beta * (feq[i] - g[i]);",
     "nxt[(long long)i * N + cell] = g[i] + alpha * (feq[i] - g[i]);"),
    ("streaming direction", "long long sx = wrap(xx - c[3 * i + 0], nx);", "long long sx = wrap(xx + c[3 * i + 0], nx);"),
    # the forcing term has no counterpart in the paper: its mutants must be
    # caught by the moment pins alone, not by the torch reference (the same
    # reading written a second time)
    ("force", "uf[a] = u[a] + force[(long long)a * N + cell] / rho;", "uf[a] = u[a] + force[(long long)a * N + cell];",
     PINS_ONLY),
    ("force sign", "nxt[(long long)i * N + cell] += feqf[i] - feq[i];", "nxt[(long long)i * N + cell] += feq[i] - feqf[i];",
     PINS_ONLY),
    ("H", "part += v * (log(v / w[i]) - 1.0);", "part += v * log(v);"),
    ("Delta H", "s2 += g[i] * x * log1p(x);", "s2 += g[i] * x * x;"),
    ("alpha_Iterate1", "return a0 - orc_dH_mirror(Q, g, feq, a0) / dH_mirror_prime(Q, g, x, a0);",
     "return a0 + orc_dH_mirror(Q, g, feq, a0) / dH_mirror_prime(Q, g, x, a0);"),
    ("wall mass balance", "double rho_w = out_mass / in_eq;", "double rho_w = 1.0;"),
    ("polynomial equilibrium", "q / (2.0 * th * th)", "q / (th * th)"),
    ("ES-BGK target", "T[k] = cpr * sig;", "T[k] = -cpr * sig;"),
    ("ES-BGK factor", "return (1.0 - 1.0 / prandtl) / (1.0 + 1.0 / (2.0 * tau1 * prandtl));",
     "return (1.0 - 1.0 / prandtl);"),
]


def _run(case, tmp):
    name, orig, mut = case[:3]
    suites = case[3] if len(case) > 3 else SUITES
    src = SRC.read_text()
    if orig not in src:
        return name, None, "mutation site not found"
    d = tmp / name.replace(" ", "_")
    d.mkdir()
    bad = d / "mutant.c"
    bad.write_text(src.replace(orig, mut, 1))
    lib = d / "libmutant.so"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", str(lib), str(bad), "-lm"])
    env = dict(os.environ, ESELBM_ORACLE_LIB=str(lib), OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu", "-p", "no:cacheprovider",
                        *suites],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    caught = [ln.split(" ")[1] for ln in r.stdout.splitlines() if ln.startswith("FAILED ")]
    return name, r.returncode, caught[0] if caught else r.stdout[-1500:]


@pytest.mark.slow
def test_pins_catch_every_mutant(tmp_path):
    """Every planted mistake is caught by some pin (mutants run in parallel
    child processes, one core each)."""
    from concurrent.futures import ThreadPoolExecutor
    workers = max(1, min(8, os.cpu_count() or 1))
    with ThreadPoolExecutor(workers) as ex:
        results = list(ex.map(lambda c: _run(c, tmp_path), MUTANTS))
    survivors = []
    for name, rc, info in results:
        print(f"[mutant {name}] " + ("caught by " + info if rc else f"SURVIVED: {info}"), file=sys.stderr)
        if not rc:
            survivors.append(name)
    assert not survivors, f"mutants not caught by any pin: {survivors}"
