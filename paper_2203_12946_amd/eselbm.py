"""Python binding of libeselbm.so (the C ABI in include/eselbm.h).

Argument marshalling only: every computation runs in the HIP library.
PyTorch provides device memory (tensors) and the stream (torch's current
HIP stream).  If the library is not built this module raises on import;
there is no fallback path.
"""
from __future__ import annotations

import contextlib
import ctypes
import pathlib

import torch

_LIB_PATH = pathlib.Path(__file__).resolve().parent / "libeselbm.so"

D2Q9, D3Q27 = 0, 1
F64, F32, F16_SHIFTED, F32_SHIFTED = 0, 1, 2, 3
MODE_HIGHER, MODE_BGK, MODE_LOWER, MODE_ELBM, MODE_ITERATE1, MODE_LBGK = 0, 1, 2, 3, 4, 5
OK, E_ARG, E_UNSUPPORTED, E_HIP, E_NONPOSITIVE = 0, 1, 2, 3, 4

DTYPES = {"f64": F64, "f32": F32, "f16s": F16_SHIFTED, "f32s": F32_SHIFTED}
MODES = {"higher": MODE_HIGHER, "bgk": MODE_BGK, "lower": MODE_LOWER, "elbm": MODE_ELBM,
         "iterate1": MODE_ITERATE1, "lbgk": MODE_LBGK}
LATTICES = {"D2Q9": D2Q9, "D3Q27": D3Q27}
TORCH_STORAGE = {F64: torch.float64, F32: torch.float32, F16_SHIFTED: torch.float16,
                 F32_SHIFTED: torch.float32}
TORCH_COMPUTE = {F64: torch.float64, F32: torch.float32, F16_SHIFTED: torch.float32,
                 F32_SHIFTED: torch.float32}


class EselbmError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"eselbm status {status}: {message}")
        self.status = status


class Stats(ctypes.Structure):
    _fields_ = [
        ("mass", ctypes.c_double), ("mom", ctypes.c_double * 3), ("kinetic", ctypes.c_double),
        ("H", ctypes.c_double), ("alpha_min", ctypes.c_double), ("alpha_max", ctypes.c_double),
        ("alpha_mean", ctypes.c_double), ("n_cells", ctypes.c_longlong), ("n_gated", ctypes.c_longlong),
        ("n_guard", ctypes.c_longlong), ("n_nonpos", ctypes.c_longlong),
        ("n_alpha_lt2", ctypes.c_longlong), ("n_exact", ctypes.c_longlong),
        ("n_newton", ctypes.c_longlong), ("n_mirror_fallback", ctypes.c_longlong),
    ]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["mom"] = list(self.mom)
        return d


_vp = ctypes.c_void_p
_SIGNATURES = {
    "eselbm_create": [ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int],
    "eselbm_destroy": [_vp],
    "eselbm_set_mode": [_vp, ctypes.c_int],
    "eselbm_set_stats": [_vp, ctypes.c_int],
    "eselbm_set_alpha_field": [_vp, _vp],
    "eselbm_set_nut_field": [_vp, _vp],
    "eselbm_set_velocity_field": [_vp, _vp],
    "eselbm_set_force": [_vp, _vp],
    "eselbm_set_walls": [_vp, ctypes.c_int, _vp],
    "eselbm_set_prandtl": [_vp, ctypes.c_double],
    "eselbm_init_equilibrium": [_vp, _vp, _vp, _vp, _vp],
    "eselbm_step": [_vp, _vp, _vp, ctypes.c_int, ctypes.c_double, _vp],
    "eselbm_alpha_stats": [_vp, ctypes.POINTER(Stats), ctypes.c_int, _vp],
    "eselbm_moments": [_vp, _vp, _vp, _vp, _vp],
    "eselbm_adjoint_step": [_vp, _vp, _vp, _vp, _vp, ctypes.c_double, _vp, _vp],
    "eselbm_adjoint_step_diss": [_vp, _vp, _vp, _vp, ctypes.c_double, _vp, ctypes.c_double, _vp, _vp],
    "eselbm_kinetic_loss": [_vp, _vp, _vp, _vp, ctypes.c_double, _vp],
    "eselbm_kinetic_loss_noalloc": [_vp, _vp, _vp, _vp, ctypes.c_double, _vp],
    "eselbm_dissipation_loss": [_vp, _vp, _vp, _vp, ctypes.c_double, _vp, _vp],
    "eselbm_dissipation_seed": [_vp, _vp, _vp, ctypes.c_double, _vp, _vp],
    "eselbm_dissipation_loss_uv": [_vp, _vp, _vp, _vp, _vp, ctypes.c_double, _vp, _vp],
    "eselbm_equilibrium_vjp": [_vp, _vp, _vp, _vp, _vp, _vp],
}
EXPORTS = tuple(_SIGNATURES) + ("eselbm_last_error",)


def _load() -> ctypes.CDLL:
    if not _LIB_PATH.exists():
        raise ImportError(
            f"{_LIB_PATH} is not built; run `python -m paper_2203_12946_amd.build` "
            "(there is no CPU fallback)")
    lib = ctypes.CDLL(str(_LIB_PATH))
    for name, argtypes in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = argtypes
        fn.restype = ctypes.c_int
    lib.eselbm_last_error.argtypes = []
    lib.eselbm_last_error.restype = ctypes.c_char_p
    return lib


lib = _load()


def _check(status: int):
    if status != OK:
        raise EselbmError(status, lib.eselbm_last_error().decode())


def _dev(t: torch.Tensor | None, dtype=None, numel=None, device=None) -> _vp:
    """Pointer of a contiguous device tensor (or NULL)."""
    if t is None:
        return _vp(None)
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if device is not None and t.device != device:
        raise ValueError(f"expected a tensor on {device}, got one on {t.device}")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"expected {numel} elements, got {t.numel()}")
    return _vp(t.data_ptr())


def _stream(stream=None) -> _vp:
    s = torch.cuda.current_stream() if stream is None else stream
    return _vp(s.cuda_stream)


class Solver:
    """One periodic grid: lattice, shape (ny, nx) or (nz, ny, nx), storage dtype.

    State tensors are [Q, *shape] in the storage dtype ("f16s" and "f32s"
    hold the shifted deviations f - w).  Adjoint tensors are [Q, *shape] in the
    compute dtype.
    """

    def __init__(self, lattice: str, shape, dtype: str = "f32", mode: str = "higher",
                 device: int | None = None):
        self.lattice = lattice
        self.D = 2 if lattice == "D2Q9" else 3
        self.Q = 9 if self.D == 2 else 27
        shape = tuple(int(s) for s in shape)
        if len(shape) != self.D:
            raise ValueError("shape must be (ny, nx) for D2Q9 and (nz, ny, nx) for D3Q27")
        self.shape = shape
        nx, ny, nz = (shape[1], shape[0], 1) if self.D == 2 else (shape[2], shape[1], shape[0])
        self.nx, self.ny, self.nz = nx, ny, nz
        self.cells = nx * ny * nz
        self.dtype_code = DTYPES[dtype]
        self.storage_dtype = TORCH_STORAGE[self.dtype_code]
        self.compute_dtype = TORCH_COMPUTE[self.dtype_code]
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self._h = _vp()
        # held by the instance: at interpreter exit the module global may be
        # cleared before the last solver is collected
        self._lib = lib
        with torch.cuda.device(self.device):
            _check(lib.eselbm_create(ctypes.byref(self._h), LATTICES[lattice], nx, ny, nz, self.dtype_code))
        self._alpha = None
        self._nut = None
        self._force = None
        self._uv = None
        self.set_mode(mode)

    def __del__(self):
        # no module globals here: at interpreter exit they may already be gone
        h, lib = getattr(self, "_h", None), getattr(self, "_lib", None)
        self._h = None
        if h is not None and h.value and lib is not None:
            lib.eselbm_destroy(h)

    def _p(self, t, dtype=None, numel=None) -> _vp:
        return _dev(t, dtype, numel, self.device)

    def _on(self):
        """Makes the solver's device current for one library call (the
        library rejects calls made with another device current)."""
        if torch.cuda.current_device() == self.device.index:
            return contextlib.nullcontext()
        return torch.cuda.device(self.device)

    # ---- configuration --------------------------------------------------
    def set_mode(self, mode: str):
        self.mode = mode
        _check(lib.eselbm_set_mode(self._h, MODES[mode]))

    def set_stats(self, on: bool):
        with self._on():
            _check(lib.eselbm_set_stats(self._h, int(bool(on))))

    def set_alpha_field(self, alpha: torch.Tensor | None):
        """Register a [*shape] compute-dtype tensor receiving per-cell alpha."""
        self._alpha = alpha
        with self._on():
            _check(lib.eselbm_set_alpha_field(self._h, self._p(alpha, self.compute_dtype, self.cells)))

    def set_nut_field(self, nut: torch.Tensor | None):
        """Register a [*shape] compute-dtype tensor receiving per-cell nu_T (Eq. nuT)."""
        self._nut = nut
        with self._on():
            _check(lib.eselbm_set_nut_field(self._h, self._p(nut, self.compute_dtype, self.cells)))

    def set_velocity_field(self, uv: torch.Tensor | None):
        """Register a [D + 1, *shape] float32 tensor receiving u (with the
        half-force shift) and rho of each step call's output state."""
        self._uv = uv
        with self._on():
            _check(lib.eselbm_set_velocity_field(self._h, self._p(uv, torch.float32, (self.D + 1) * self.cells)))

    def empty_velocity(self) -> torch.Tensor:
        return torch.empty((self.D + 1,) + self.shape, dtype=torch.float32, device=self.device)

    def set_walls(self, walls=None, velocity=None):
        """Diffuse walls: ``walls`` per axis (x, y[, z]) True/False (None: none);
        ``velocity`` {(axis, side): (ux, uy[, uz])}, side 0 low, 1 high."""
        mask = 0 if walls is None else sum(1 << a for a, on in enumerate(walls) if on)
        uw = (ctypes.c_double * 18)()
        for (a, sd), v in (velocity or {}).items():
            for k, comp in enumerate(v):
                uw[(2 * a + sd) * 3 + k] = float(comp)
        with self._on():
            _check(lib.eselbm_set_walls(self._h, mask, ctypes.cast(uw, _vp)))

    def set_prandtl(self, prandtl: float):
        """Entropic ES-BGK collision at Prandtl number ``prandtl`` (1: off)."""
        with self._on():
            _check(lib.eselbm_set_prandtl(self._h, float(prandtl)))

    def set_force(self, F: torch.Tensor | None):
        """Register a [D, *shape] float32 body-force density (F32 storage only)."""
        self._force = F
        with self._on():
            _check(lib.eselbm_set_force(self._h, self._p(F, torch.float32, self.D * self.cells)))

    # ---- state ----------------------------------------------------------
    def empty_state(self) -> torch.Tensor:
        return torch.empty((self.Q,) + self.shape, dtype=self.storage_dtype, device=self.device)

    def empty_adjoint(self) -> torch.Tensor:
        return torch.empty((self.Q,) + self.shape, dtype=self.compute_dtype, device=self.device)

    def init_equilibrium(self, rho: torch.Tensor, u: torch.Tensor, out: torch.Tensor | None = None,
                         stream=None) -> torch.Tensor:
        f = self.empty_state() if out is None else out
        with self._on():
            _check(lib.eselbm_init_equilibrium(
                self._h, self._p(rho, torch.float64, self.cells), self._p(u, torch.float64, self.D * self.cells),
                self._p(f, self.storage_dtype, self.Q * self.cells), _stream(stream)))
        return f

    def step(self, f_in: torch.Tensor, f_out: torch.Tensor, nsteps: int, tau: float, stream=None):
        n = self.Q * self.cells
        with self._on():
            _check(lib.eselbm_step(self._h, self._p(f_in, self.storage_dtype, n), self._p(f_out, self.storage_dtype, n),
                                   int(nsteps), float(tau), _stream(stream)))

    def stats(self, with_H: bool = False, stream=None) -> dict:
        """FP64 diagnostics of the last statistics-enabled step (synchronises
        the stream).  A step that met non-positive or non-finite populations
        is not an error here: the counts are returned with ``status`` set to
        E_NONPOSITIVE and ``n_nonpos`` > 0, so that a caller can stop a run
        that has lost positivity; every other failure raises EselbmError."""
        st = Stats()
        with self._on():
            status = lib.eselbm_alpha_stats(self._h, ctypes.byref(st), int(bool(with_H)), _stream(stream))
        if status not in (OK, E_NONPOSITIVE):
            _check(status)
        d = st.as_dict()
        d["status"] = status
        return d

    def moments(self, f: torch.Tensor, stream=None):
        rho = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        u = torch.empty((self.D,) + self.shape, dtype=torch.float64, device=self.device)
        with self._on():
            _check(lib.eselbm_moments(self._h, self._p(f, self.storage_dtype, self.Q * self.cells),
                                      self._p(rho), self._p(u), _stream(stream)))
        return rho, u

    # ---- adjoint ----------------------------------------------------------
    def empty_seed(self) -> torch.Tensor:
        """[1 + D, *shape] compute-dtype buffer for a compact loss seed."""
        return torch.empty((1 + self.D,) + self.shape, dtype=self.compute_dtype, device=self.device)

    def adjoint_step(self, f_n, lam_next, lam_n, tau: float, force_grad=None, seed_next=None, stream=None):
        n = self.Q * self.cells
        with self._on():
            _check(lib.eselbm_adjoint_step(
                self._h, self._p(f_n, self.storage_dtype, n), self._p(lam_next, self.compute_dtype, n),
                self._p(seed_next, self.compute_dtype, (1 + self.D) * self.cells) if seed_next is not None else _vp(None),
                self._p(lam_n, self.compute_dtype, n), float(tau),
                self._p(force_grad, torch.float32, self.D * self.cells) if force_grad is not None else _vp(None),
                _stream(stream)))

    def adjoint_step_diss(self, f_n, lam_next, uv_next, weight: float, lam_n, tau: float, force_grad=None,
                          stream=None):
        """adjoint_step with the dissipation seed of the state after the step
        formed in the kernel from that state's velocity field uv_next."""
        n = self.Q * self.cells
        with self._on():
            _check(lib.eselbm_adjoint_step_diss(
                self._h, self._p(f_n, self.storage_dtype, n), self._p(lam_next, self.compute_dtype, n),
                self._p(uv_next, torch.float32, (self.D + 1) * self.cells), float(weight),
                self._p(lam_n, self.compute_dtype, n), float(tau),
                self._p(force_grad, torch.float32, self.D * self.cells) if force_grad is not None else _vp(None),
                _stream(stream)))

    def kinetic_loss(self, f, loss=None, lam=None, scale: float = 1.0, stream=None):
        with self._on():
            _check(lib.eselbm_kinetic_loss(
                self._h, self._p(f, self.storage_dtype, self.Q * self.cells),
                self._p(loss, torch.float64, 1) if loss is not None else _vp(None),
                self._p(lam, self.compute_dtype, self.Q * self.cells) if lam is not None else _vp(None),
                float(scale), _stream(stream)))

    def kinetic_loss_noalloc(self, f, loss=None, lam=None, scale: float = 1.0, stream=None):
        """kinetic_loss without any allocation (a fixed per-device buffer;
        grids of at most 2^24 cells; overlapping calls on one device race)."""
        with self._on():
            _check(lib.eselbm_kinetic_loss_noalloc(
                self._h, self._p(f, self.storage_dtype, self.Q * self.cells),
                self._p(loss, torch.float64, 1) if loss is not None else _vp(None),
                self._p(lam, self.compute_dtype, self.Q * self.cells) if lam is not None else _vp(None),
                float(scale), _stream(stream)))

    def dissipation_loss(self, f, loss=None, lam=None, weight: float = 1.0, force_grad=None, stream=None):
        with self._on():
            _check(lib.eselbm_dissipation_loss(
                self._h, self._p(f, self.storage_dtype, self.Q * self.cells),
                self._p(loss, torch.float64, 1) if loss is not None else _vp(None),
                self._p(lam, self.compute_dtype, self.Q * self.cells) if lam is not None else _vp(None),
                float(weight),
                self._p(force_grad, torch.float32, self.D * self.cells) if force_grad is not None else _vp(None),
                _stream(stream)))

    def dissipation_seed(self, f, seed, weight: float = 1.0, force_grad=None, stream=None):
        with self._on():
            _check(lib.eselbm_dissipation_seed(
                self._h, self._p(f, self.storage_dtype, self.Q * self.cells),
                self._p(seed, self.compute_dtype, (1 + self.D) * self.cells), float(weight),
                self._p(force_grad, torch.float32, self.D * self.cells) if force_grad is not None else _vp(None),
                _stream(stream)))

    def dissipation_loss_uv(self, uv, loss=None, lam=None, seed=None, weight: float = 1.0, force_grad=None,
                            stream=None):
        """dissipation_loss / dissipation_seed from a velocity field written
        by a step (set_velocity_field) instead of the state."""
        with self._on():
            _check(lib.eselbm_dissipation_loss_uv(
                self._h, self._p(uv, torch.float32, (self.D + 1) * self.cells),
                self._p(loss, torch.float64, 1) if loss is not None else _vp(None),
                self._p(lam, self.compute_dtype, self.Q * self.cells) if lam is not None else _vp(None),
                self._p(seed, self.compute_dtype, (1 + self.D) * self.cells) if seed is not None else _vp(None),
                float(weight),
                self._p(force_grad, torch.float32, self.D * self.cells) if force_grad is not None else _vp(None),
                _stream(stream)))

    def equilibrium_vjp(self, rho, u, lam, stream=None) -> torch.Tensor:
        gu = torch.empty((self.D,) + self.shape, dtype=torch.float64, device=self.device)
        with self._on():
            _check(lib.eselbm_equilibrium_vjp(
                self._h, self._p(rho, torch.float64, self.cells), self._p(u, torch.float64, self.D * self.cells),
                self._p(lam, self.compute_dtype, self.Q * self.cells), self._p(gu), _stream(stream)))
        return gu


def beta_of_tau(tau: float) -> float:
    return 1.0 / (2.0 * tau + 1.0)


def rollout(solver: Solver, f0: torch.Tensor, tau: float, nsteps: int, ckpt_every: int,
            force: torch.Tensor | None = None, diss_weight: float | None = None,
            keep_segments: int | str | None = 1):
    """Differentiable checkpointed rollout: (state after nsteps, accumulated
    dissipation loss); see paper_2203_12946_amd.adjoint.rollout."""
    from .adjoint import rollout as _rollout
    return _rollout(solver, f0, tau, nsteps, ckpt_every, force=force, diss_weight=diss_weight,
                    keep_segments=keep_segments)


def equilibrium(solver: Solver, rho: torch.Tensor, u: torch.Tensor) -> torch.Tensor:
    """Differentiable equilibrium initial state f = feq(rho, u) (gradient
    w.r.t. u); see paper_2203_12946_amd.adjoint.equilibrium."""
    from .adjoint import equilibrium as _equilibrium
    return _equilibrium(solver, rho, u)
