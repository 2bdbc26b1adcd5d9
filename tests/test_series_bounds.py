"""The truncation bounds behind the kernels' series forms, checked on the CPU
against the constants in the headers (so that a change of a range or an order
there that the rounding of the type no longer covers fails here).

* expm1 by its Taylor polynomial for |v| <= kSmallExpArg (quasi_eq.hpp,
  SmallExpm1<float/double>::N): the first dropped term relative to v.
* phi(y) = (1 + y) log(1 + y) - y by its series for |y| < Y and log(1 + y)
  by the derivative of that series (lattice.hpp, MirrorCfg<float/double>):
  the polynomials evaluated as the kernels do, in extended precision,
  against the series to 60 terms (itself checked against the closed form
  where that does not cancel) and against log1p over the whole range.
"""
import math
import pathlib
import re

import numpy as np
import pytest

CSRC = pathlib.Path(__file__).resolve().parents[1] / "paper_2203_12946_amd" / "csrc"
EPS = {"float": 2.0 ** -24, "double": 2.0 ** -53}


def _src(name):
    return (CSRC / name).read_text()


def _small_expm1():
    s = _src("quasi_eq.hpp")
    arg = s.split("constexpr double kSmallExpArg =")[1].split(";")[0]
    num, den = (float(t) for t in arg.split("/"))
    n = {t: int(re.search(r"struct SmallExpm1<%s> \{\s*static constexpr int N = (\d+);" % t, s).group(1))
         for t in ("float", "double")}
    return num / den, n


def _mirror_cfg():
    s = _src("lattice.hpp")
    out = {}
    for t in ("float", "double"):
        m = re.search(r"struct MirrorCfg<%s> \{\s*static constexpr double Y = ([0-9.]+);.*?"
                      r"static constexpr int K = (\d+);" % t, s, re.S)
        out[t] = (float(m.group(1)), int(m.group(2)))
    return out


@pytest.mark.parametrize("t", ["float", "double"])
def test_small_expm1_truncation_below_rounding(t):
    x, n = _small_expm1()
    # Taylor remainder relative to expm1(v) ~ v: below |v|^N / (N+1)! for |v| <= x (alternating tail bound
    # times a factor 1 / (1 - x) for the geometric rest)
    bound = x ** n[t] / math.factorial(n[t] + 1) / (1.0 - x)
    assert bound < EPS[t] / 8, (t, bound)
    # and the polynomial, evaluated by Horner as the kernel does, against expm1 on the range
    v = np.linspace(-x, x, 4001, dtype=np.longdouble)
    p = np.full_like(v, 1.0 / math.factorial(n[t]))
    for k in range(n[t] - 1, 0, -1):
        p = p * v + np.longdouble(1.0 / math.factorial(k))
    p = p * v
    ref = np.expm1(v)
    nz = v != 0
    rel = np.max(np.abs((p[nz] - ref[nz]) / ref[nz]))
    assert float(rel) < 2 * EPS[t], (t, float(rel))


@pytest.mark.parametrize("t", ["float", "double"])
def test_mirror_series_truncation_below_rounding(t):
    Y, K = _mirror_cfg()[t]
    y = np.linspace(-Y, Y, 8001, dtype=np.longdouble)[1:-1]
    y = y[np.abs(y) > 1e-4]
    # phi by its series: sum_{k=2}^{K} (-1)^k y^k / (k (k - 1)), Horner as in phi_series
    s = np.full_like(y, (-1.0 if K % 2 else 1.0) / (K * (K - 1.0)))
    for k in range(K - 1, 1, -1):
        s = s * y + np.longdouble((-1.0 if k % 2 else 1.0) / (k * (k - 1.0)))
    phi = s * y * y
    # the reference: the same series to 60 terms (the closed form cancels for
    # small y; the series converges far below the extended precision here)
    r = np.zeros_like(y)
    for k in range(60, 1, -1):
        r = r * y + np.longdouble((-1.0 if k % 2 else 1.0) / (k * (k - 1.0)))
    phi_ref = r * y * y
    assert np.allclose(phi_ref[np.abs(y) > 0.01], ((1 + y) * np.log1p(y) - y)[np.abs(y) > 0.01], rtol=1e-12)
    # log(1 + y) by the derivative series, Horner as in log1p_series
    q = np.full_like(y, (-1.0 if (K - 2) % 2 else 1.0) / (K - 1.0))
    for j in range(K - 3, -1, -1):
        q = q * y + np.longdouble((-1.0 if j % 2 else 1.0) / (j + 1.0))
    l = q * y
    l_ref = np.log1p(y)
    e_phi = float(np.max(np.abs((phi - phi_ref) / phi_ref)))
    e_log = float(np.max(np.abs((l - l_ref) / l_ref)))
    # the series' truncation stays within a few roundings of the type (the
    # kernels' own arithmetic rounds at the same level)
    assert e_phi < 4 * EPS[t], (t, e_phi)
    assert e_log < 4 * EPS[t], (t, e_log)
