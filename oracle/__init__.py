"""FP64 CPU oracle for the ESELBM stream-collide step (arXiv:2203.12946).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package; the product
library never does, and it shares no code with it.

The arithmetic lives in ``eselbm_oracle.c`` (plain C, double precision, one
cell at a time, the paper's formulas in the paper's order).  This module only
builds that file with gcc, loads it with ctypes and marshals NumPy arrays.

Parity status of each function is stated in its docstring; every function
here is pinned by ``tests/test_oracle_*.py`` against closed forms, limits,
invariants or brute force (none of them re-types the oracle's formulas).
"""
from __future__ import annotations

import ctypes
import os
import pathlib
import subprocess

import numpy as np

_HERE = pathlib.Path(__file__).resolve().parent
_SRC = _HERE / "eselbm_oracle.c"
_LIB_PATH = _HERE / "liboracle.so"
# ESELBM_ORACLE_LIB names another build of the C file to load instead (the
# mutation check of the pins builds deliberately broken copies); it is then
# loaded as it is, never rebuilt.
_LIB_OVERRIDE = os.environ.get("ESELBM_ORACLE_LIB")
_lib = None

MODES = {"higher": 0, "bgk": 1, "lower": 2, "elbm": 3, "iterate1": 4, "lbgk": 5}


def build() -> pathlib.Path:
    """Compile the oracle shared library with gcc (no GPU needed)."""
    tmp = _LIB_PATH.with_suffix(".so.tmp%d" % os.getpid())
    subprocess.check_call(
        ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", str(tmp), str(_SRC), "-lm"]
    )
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if _LIB_OVERRIDE:
        lib = ctypes.CDLL(_LIB_OVERRIDE)
    else:
        if not _LIB_PATH.exists() or _LIB_PATH.stat().st_mtime < _SRC.stat().st_mtime:
            build()
        lib = ctypes.CDLL(str(_LIB_PATH))
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    llp = ctypes.POINTER(ctypes.c_longlong)
    lib.orc_lattice.argtypes = [ctypes.c_int, ip, dp]
    lib.orc_lattice.restype = ctypes.c_int
    lib.orc_equilibrium.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp]
    lib.orc_equilibrium.restype = None
    lib.orc_equilibrium_poly.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp]
    lib.orc_equilibrium_poly.restype = None
    lib.orc_cell_moments.argtypes = [ctypes.c_int, dp, dp, dp]
    lib.orc_cell_moments.restype = None
    lib.orc_path_length.argtypes = [ctypes.c_int, dp, dp, ctypes.c_double, ctypes.c_int, dp]
    lib.orc_path_length.restype = ctypes.c_int
    lib.orc_H.argtypes = [ctypes.c_int, ctypes.c_longlong, dp]
    lib.orc_H.restype = ctypes.c_double
    lib.orc_dH_step.argtypes = [ctypes.c_int, dp, dp, ctypes.c_double, ctypes.c_double]
    lib.orc_dH_step.restype = ctypes.c_double
    lib.orc_dH_mirror.argtypes = [ctypes.c_int, dp, dp, ctypes.c_double]
    lib.orc_dH_mirror.restype = ctypes.c_double
    lib.orc_alpha_elbm.argtypes = [ctypes.c_int, dp, dp]
    lib.orc_alpha_elbm.restype = ctypes.c_double
    lib.orc_alpha_iterate1.argtypes = [ctypes.c_int, dp, dp]
    lib.orc_alpha_iterate1.restype = ctypes.c_double
    lib.orc_step.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp,
                             ctypes.c_int, ctypes.c_double, ctypes.c_int, dp, dp, llp]
    lib.orc_step.restype = ctypes.c_int
    lib.orc_step_walls.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp,
                                   dp, ctypes.c_int, ctypes.c_double, ctypes.c_int, dp, llp]
    lib.orc_step_walls.restype = ctypes.c_int
    lib.orc_esbgk_cpr.argtypes = [ctypes.c_double, ctypes.c_double]
    lib.orc_esbgk_cpr.restype = ctypes.c_double
    lib.orc_quasi_equilibrium.argtypes = [ctypes.c_int, dp, dp, ctypes.c_double, dp, ip]
    lib.orc_quasi_equilibrium.restype = ctypes.c_int
    lib.orc_step_esbgk.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp,
                                   ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int, dp, llp]
    lib.orc_step_esbgk.restype = ctypes.c_int
    lib.orc_init_equilibrium.argtypes = [ctypes.c_int, ctypes.c_longlong, dp, dp, dp]
    lib.orc_init_equilibrium.restype = None
    lib.orc_moments.argtypes = [ctypes.c_int, ctypes.c_longlong, dp, dp, dp]
    lib.orc_moments.restype = None
    lib.orc_num_threads.argtypes = []
    lib.orc_num_threads.restype = ctypes.c_int
    lib.orc_set_threads.argtypes = [ctypes.c_int]
    lib.orc_set_threads.restype = None
    _lib = lib
    return lib


def _dp(a):
    if a is None:
        return ctypes.POINTER(ctypes.c_double)()
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleError(RuntimeError):
    """Raised when a pre-collision population is non-positive or not finite."""


def lattice(D: int):
    """Velocities c [Q,3] and weights w [Q] of the D1Q3 tensor-product lattice."""
    lib = _load()
    c = np.zeros((27, 3), dtype=np.int32)
    w = np.zeros(27)
    Q = lib.orc_lattice(D, c.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(w))
    if Q < 0:
        raise ValueError("D must be 1, 2 or 3")
    return c[:Q].copy(), w[:Q].copy()


def equilibrium(D: int, rho: float, u) -> np.ndarray:
    """Product-form entropic equilibrium for one cell (Sec. II)."""
    lib = _load()
    u = _f64(np.resize(np.asarray(u, dtype=np.float64), 3))
    feq = np.zeros(3 ** D)
    lib.orc_equilibrium(D, float(rho), _dp(u), _dp(feq))
    return feq


def equilibrium_poly(D: int, rho: float, u) -> np.ndarray:
    """Polynomial equilibrium of Eq. histeq for one cell (classic LBGK)."""
    lib = _load()
    u = _f64(np.resize(np.asarray(u, dtype=np.float64), 3))
    feq = np.zeros(3 ** D)
    lib.orc_equilibrium_poly(D, float(rho), _dp(u), _dp(feq))
    return feq


def cell_moments(D: int, f):
    lib = _load()
    f = _f64(f)
    rho = np.zeros(1)
    u = np.zeros(3)
    lib.orc_cell_moments(D, _dp(f), _dp(rho), _dp(u))
    return rho[0], u[:D].copy()


_DETAIL_KEYS = ("alpha", "alpha_lower", "h", "a", "b", "c", "a1", "b1", "c1", "a2",
                "x_min", "x_absmax", "gated", "guarded", "alpha_unguarded", "no_root")


def path_length(g, feq, beta: float, mode: str = "higher") -> dict:
    """Per-cell path length with every intermediate (Sec. IV, App. D)."""
    lib = _load()
    g = _f64(g)
    feq = _f64(feq)
    det = np.zeros(16)
    rc = lib.orc_path_length(g.size, _dp(g), _dp(feq), float(beta), MODES[mode], _dp(det))
    if rc != 0:
        raise OracleError("non-positive or non-finite population")
    d = dict(zip(_DETAIL_KEYS, det.tolist()))
    d["gated"] = bool(d["gated"])
    d["guarded"] = bool(d["guarded"])
    d["no_root"] = bool(d["no_root"])
    return d


def dH_step(g, feq, alpha: float, beta: float) -> float:
    """Exact per-cell entropy change of the collision (Eq. deltaH3)."""
    g = _f64(g)
    feq = _f64(feq)
    return _load().orc_dH_step(g.size, _dp(g), _dp(feq), float(alpha), float(beta))


def dH_mirror(g, feq, alpha: float) -> float:
    """Entropy change to the mirror state (Eq. deltaH_)."""
    g = _f64(g)
    feq = _f64(feq)
    return _load().orc_dH_mirror(g.size, _dp(g), _dp(feq), float(alpha))


def alpha_elbm(g, feq) -> float:
    """Iterative ELBM path length: root of the mirror condition (NaN if none)."""
    g = _f64(g)
    feq = _f64(feq)
    return _load().orc_alpha_elbm(g.size, _dp(g), _dp(feq))


def alpha_iterate1(g, feq) -> float:
    """One Newton step of the mirror condition from alpha_Lower (Sec. V C)."""
    g = _f64(g)
    feq = _f64(feq)
    return _load().orc_alpha_iterate1(g.size, _dp(g), _dp(feq))


def _grid(f):
    """(D, nx, ny, nz) of an SoA state shaped [3, nx], [9, ny, nx] or
    [27, nz, ny, nx]."""
    if f.ndim == 2:
        Q, nx = f.shape
        if Q != 3:
            raise ValueError("a 1-D state must have 3 populations")
        return 1, nx, 1, 1
    if f.ndim == 3:
        Q, ny, nx = f.shape
        if Q != 9:
            raise ValueError("a 2-D state must have 9 populations")
        return 2, nx, ny, 1
    if f.ndim == 4:
        Q, nz, ny, nx = f.shape
        if Q != 27:
            raise ValueError("a 3-D state must have 27 populations")
        return 3, nx, ny, nz
    raise ValueError("state must be [Q,nx], [Q,ny,nx] or [Q,nz,ny,nx]")


def step(f, nsteps: int, tau: float, mode: str = "higher", force=None,
         want_alpha: bool = False):
    """Run nsteps periodic pull-stream + collide steps; returns the new state.

    With ``want_alpha`` returns ``(state, alpha_field, (n_gated, n_guarded,
    n_no_root))`` for the last step.  ``force`` is a [D, ...grid] body-force density.
    """
    lib = _load()
    f = _f64(f)
    D, nx, ny, nz = _grid(f)
    out = np.empty_like(f)
    alpha = np.empty(f.shape[1:]) if want_alpha else None
    counts = np.zeros(3, dtype=np.int64)
    F = None if force is None else _f64(force)
    if F is not None and F.shape != (D,) + f.shape[1:]:
        raise ValueError("force must be [D, ...grid]")
    rc = lib.orc_step(D, nx, ny, nz, _dp(f), _dp(out), int(nsteps), float(tau), MODES[mode],
                      _dp(F), _dp(alpha),
                      counts.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)))
    if rc == -1:
        raise OracleError("non-positive or non-finite pre-collision population")
    if rc != 0:
        raise MemoryError("oracle allocation failed")
    if want_alpha:
        return out, alpha, (int(counts[0]), int(counts[1]), int(counts[2]))
    return out


def esbgk_cpr(tau1: float, prandtl: float) -> float:
    """The ES-BGK stress factor c_Pr = (1 - 1/Pr) / (1 + 1/(2 tau1 Pr))."""
    return float(_load().orc_esbgk_cpr(float(tau1), float(prandtl)))


def quasi_equilibrium(g, feq, cpr: float):
    """(f^QE, converged, Newton steps) of one cell: the minimiser of H with the
    mass and momentum of g and pressure tensor P(feq) + cpr (P(g) - P(feq))."""
    lib = _load()
    g = _f64(g)
    feq = _f64(feq)
    D = {3: 1, 9: 2, 27: 3}[g.size]
    out = np.empty_like(g)
    it = ctypes.c_int(0)
    rc = lib.orc_quasi_equilibrium(D, _dp(g), _dp(feq), float(cpr), _dp(out), ctypes.byref(it))
    return out, rc == 0, int(it.value)


def step_esbgk(f, nsteps: int, tau1: float, prandtl: float, mode: str = "higher",
               want_alpha: bool = False):
    """Periodic entropic ES-BGK steps (mode higher, lower or bgk).  With
    ``want_alpha`` returns ``(state, alpha, (n_gated, n_guarded, n_qe_fallback))``."""
    lib = _load()
    f = _f64(f)
    D, nx, ny, nz = _grid(f)
    out = np.empty_like(f)
    alpha = np.empty(f.shape[1:]) if want_alpha else None
    counts = np.zeros(3, dtype=np.int64)
    rc = lib.orc_step_esbgk(D, nx, ny, nz, _dp(f), _dp(out), int(nsteps), float(tau1), float(prandtl),
                            MODES[mode], _dp(alpha), counts.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)))
    if rc == -1:
        raise OracleError("non-positive or non-finite pre-collision population")
    if rc == -3:
        raise ValueError("ES-BGK steps take mode higher, lower or bgk")
    if rc != 0:
        raise MemoryError("oracle allocation failed")
    if want_alpha:
        return out, alpha, (int(counts[0]), int(counts[1]), int(counts[2]))
    return out


def step_walls(f, nsteps: int, tau: float, walls, wall_velocity=None, mode: str = "higher",
               want_alpha: bool = False):
    """Steps with diffuse walls (the boundary rule of the cavity, Sec. V C).

    ``walls``: per axis (x, y[, z]) True for walls at -1/2 and n - 1/2, False
    for periodic.  ``wall_velocity``: {(axis, side): velocity} with side 0
    the low and 1 the high wall (default: every wall at rest).  With
    ``want_alpha`` returns ``(state, alpha, (n_gated, n_guarded, n_fallback))``.
    """
    lib = _load()
    f = _f64(f)
    D, nx, ny, nz = _grid(f)
    mask = sum(1 << a for a, on in enumerate(walls) if on)
    uw = np.zeros((3, 2, 3))
    for (a, sd), v in (wall_velocity or {}).items():
        uw[a, sd, :len(v)] = v
    uw = _f64(uw)
    out = np.empty_like(f)
    alpha = np.empty(f.shape[1:]) if want_alpha else None
    counts = np.zeros(3, dtype=np.int64)
    rc = lib.orc_step_walls(D, nx, ny, nz, mask, _dp(uw), _dp(f), _dp(out), int(nsteps), float(tau),
                            MODES[mode], _dp(alpha), counts.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)))
    if rc == -1:
        raise OracleError("non-positive or non-finite pre-collision population")
    if rc != 0:
        raise MemoryError("oracle allocation failed")
    if want_alpha:
        return out, alpha, (int(counts[0]), int(counts[1]), int(counts[2]))
    return out


def init_equilibrium(rho, u) -> np.ndarray:
    """State f = feq(rho, u) for every cell; rho [...grid], u [D, ...grid]."""
    lib = _load()
    rho = _f64(rho)
    u = _f64(u)
    D = u.shape[0]
    if u.shape[1:] != rho.shape or rho.ndim != D:
        raise ValueError("u must be [D, ...grid] with rho [...grid]")
    N = rho.size
    f = np.empty((3 ** D,) + rho.shape)
    lib.orc_init_equilibrium(D, N, _dp(rho), _dp(u), _dp(f))
    return f


def moments(f):
    """Density [...grid] and velocity [D, ...grid] fields of a state."""
    lib = _load()
    f = _f64(f)
    D = _grid(f)[0]
    rho = np.empty(f.shape[1:])
    u = np.empty((D,) + f.shape[1:])
    lib.orc_moments(D, rho.size, _dp(f), _dp(rho), _dp(u))
    return rho, u


def H(f) -> float:
    """Global H function sum_x <f, log(f/w) - 1> (Eq. hdef)."""
    f = _f64(f)
    D = _grid(f)[0]
    return _load().orc_H(D, f[0].size, _dp(f))


def num_threads() -> int:
    """OpenMP threads the oracle's cell loops use."""
    return int(_load().orc_num_threads())


def set_threads(n: int) -> None:
    """Cap the oracle's OpenMP threads at n (n < 1: back to the default)."""
    _load().orc_set_threads(int(n))


def beta_of_tau(tau: float) -> float:
    """beta = dt / (2 tau + dt), dt = 1 (Sec. II)."""
    return 1.0 / (2.0 * tau + 1.0)


def light_cone_block(f, center, k: int):
    """Periodic (2k+1)^D block of state ``f`` centred on cell ``center``.

    Running the oracle's periodic step k times on this block gives the exact
    value of the centre cell after k steps on the full grid: information
    travels one cell per step, so the wrap-around of the small block reaches
    the centre only after k + 1 steps.
    """
    D = _grid(np.asarray(f))[0]
    idx = []
    for a, cval in enumerate(center):
        n = f.shape[1 + a]
        idx.append((np.arange(-k, k + 1) + cval) % n)
    if D == 2:
        return np.ascontiguousarray(f[:, idx[0][:, None], idx[1][None, :]])
    return np.ascontiguousarray(f[:, idx[0][:, None, None], idx[1][None, :, None],
                                  idx[2][None, None, :]])
