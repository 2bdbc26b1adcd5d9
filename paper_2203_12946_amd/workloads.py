"""Seeded synthetic initial conditions shaped like the paper's test flows.

This module holds no lattice-Boltzmann arithmetic: it only produces density,
velocity and body-force fields (double precision NumPy arrays) from which both
the HIP library and the CPU oracle build their own initial states.  Every
random draw is seeded.

Grid coordinates are node based: cell index i sits at x = i / N in the
non-dimensional coordinates of the paper's shear layer (Sec. V B) and at
x = 2 pi i / N for the periodic Taylor-Green vortices.  Arrays are indexed
[y, x] in 2-D and [z, y, x] in 3-D; velocity arrays carry the component
first, [D, ...grid], with component 0 along x.

Relaxation times are the paper's tau (nu = tau theta0, theta0 = 1/3).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

THETA0 = 1.0 / 3.0


def tau_from_nu(nu: float) -> float:
    """Paper's tau for a kinematic viscosity nu (nu = tau * theta0)."""
    return nu / THETA0


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    lattice: str          # "D2Q9" | "D3Q27"
    shape: tuple          # (ny, nx) or (nz, ny, nx)
    nu: float
    steps: int

    @property
    def tau(self) -> float:
        return tau_from_nu(self.nu)

    @property
    def cells(self) -> int:
        return int(np.prod(self.shape))


def taylor_green_2d(n: int, u0: float = 0.05, dtype=np.float64):
    """2-D periodic Taylor-Green vortex on an n x n grid.

    u = -u0 cos(kx) sin(ky), v = u0 sin(kx) cos(ky), k = 2 pi / n, with the
    matching incompressible pressure carried by the density
    rho = 1 - (3 u0^2 / 4)(cos 2kx + cos 2ky).
    """
    k = 2.0 * math.pi / n
    i = np.arange(n, dtype=np.float64)
    X, Y = np.meshgrid(i * k, i * k, indexing="xy")  # [y, x]
    u = np.stack([-u0 * np.cos(X) * np.sin(Y), u0 * np.sin(X) * np.cos(Y)])
    rho = 1.0 - 0.75 * u0 * u0 * (np.cos(2.0 * X) + np.cos(2.0 * Y))
    return rho.astype(dtype), u.astype(dtype)


def shear_layer(n: int, u0: float = 0.04, width: float = 0.05, delta: float = 0.05,
                ny: int | None = None):
    """Doubly periodic shear layer of Sec. V B on an n (x) by ny (y) grid.

    u_x = U0 tanh((4y - 1)/w) for y <= 1/2, U0 tanh((3 - 4y)/w) otherwise;
    u_y = U0 delta sin(2 pi (x + 1/4)); rho = 1.  With w = 0.05 the layers
    read tanh(80 (y - 1/4)) and tanh(80 (3/4 - y)).
    """
    ny = n if ny is None else ny
    x = np.arange(n, dtype=np.float64) / n
    y = np.arange(ny, dtype=np.float64) / ny
    X, Y = np.meshgrid(x, y, indexing="xy")
    ux = np.where(Y <= 0.5, u0 * np.tanh((4.0 * Y - 1.0) / width),
                  u0 * np.tanh((3.0 - 4.0 * Y) / width))
    uy = u0 * delta * np.sin(2.0 * math.pi * (X + 0.25))
    return np.ones_like(X), np.stack([ux, uy])


def taylor_green_3d(n: int, u0: float = 0.1 / math.sqrt(3.0), noise: float = 1e-4,
                    seed: int = 1600, shape=None):
    """3-D periodic Taylor-Green vortex (Re 1600 set by nu), plus seeded noise.

    u = u0 sin x cos y cos z, v = -u0 cos x sin y cos z, w = 0 on the
    2 pi-periodic box, rho = 1 + 3 (u0^2/16)(cos 2x + cos 2y)(cos 2z + 2), and
    independent N(0, noise^2) perturbations on each velocity component.
    ``shape`` = (nz, ny, nx) overrides the cube (each axis stays 2 pi periodic).
    """
    nz, ny, nx = (n, n, n) if shape is None else shape
    kx, ky, kz = (2.0 * math.pi / m for m in (nx, ny, nz))
    z = np.arange(nz)[:, None, None] * kz
    y = np.arange(ny)[None, :, None] * ky
    x = np.arange(nx)[None, None, :] * kx
    u = u0 * np.sin(x) * np.cos(y) * np.cos(z)
    v = -u0 * np.cos(x) * np.sin(y) * np.cos(z)
    w = np.zeros_like(u * v)
    u = u + 0.0 * v
    rho = 1.0 + 3.0 * (u0 * u0 / 16.0) * (np.cos(2 * x) + np.cos(2 * y)) * (np.cos(2 * z) + 2.0)
    vel = np.stack([np.broadcast_to(u, (nz, ny, nx)), np.broadcast_to(v, (nz, ny, nx)), w])
    if noise > 0.0:
        rng = np.random.default_rng(seed)
        vel = vel + rng.normal(0.0, noise, size=vel.shape)
    return np.broadcast_to(rho, (nz, ny, nx)).copy(), np.ascontiguousarray(vel)


def random_divfree_2d(n: int, k_peak: float = 8.0, u_rms: float = 0.03, seed: int = 3):
    """Seeded divergence-free 2-D velocity from a random streamfunction.

    The energy spectrum is E(k) ~ (k/k_peak)^4 exp(-2 (k/k_peak)^2), the field
    is scaled to the requested r.m.s. speed, and rho = 1.
    """
    rng = np.random.default_rng(seed)
    kx = np.fft.fftfreq(n, d=1.0 / n)
    KX, KY = np.meshgrid(kx, kx, indexing="xy")
    K = np.sqrt(KX ** 2 + KY ** 2)
    E = (K / k_peak) ** 4 * np.exp(-2.0 * (K / k_peak) ** 2)
    amp = np.zeros_like(K)
    nz = K > 0
    # |psi_k|^2 k^2 ~ E(k) / k  (2-D shell)  =>  |psi_k| ~ sqrt(E / k^3)
    amp[nz] = np.sqrt(E[nz] / K[nz] ** 3)
    phase = np.exp(2j * math.pi * rng.random(K.shape))
    psi = np.real(np.fft.ifft2(amp * phase))
    # u = d psi / dy, v = -d psi / dx, spectrally
    psi_k = np.fft.fft2(psi)
    u = np.real(np.fft.ifft2(1j * KY * psi_k))
    v = np.real(np.fft.ifft2(-1j * KX * psi_k))
    vel = np.stack([u, v]) * (2.0 * math.pi / n)
    rms = math.sqrt(float(np.mean(vel[0] ** 2 + vel[1] ** 2)))
    vel *= u_rms / rms
    return np.ones((n, n)), vel


def sod_tube(n: int = 800, rho_left: float = 1.5, rho_right: float = 0.75):
    """The shock tube of Sec. V A: density step at the middle of an n-node
    tube (nodes 1..n/2 of the paper's 1-based numbering at rho_left, the rest
    at rho_right), fluid at rest.  Returns rho [n] and u [1, n]."""
    rho = np.where(np.arange(n) < n // 2, rho_left, rho_right).astype(np.float64)
    return rho, np.zeros((1, n))


def sod_lattice_nu(n: int = 800, nu: float = 1e-5) -> float:
    """Lattice viscosity of the shock tube.  The paper quotes nu = 1e-5; read
    in units where the tube has length 1 and the lattice speed is 1 (dx = dt
    = 1/n), the lattice value is nu * n.  This reading reproduces the
    turbulent-viscosity ratios the paper reports for the tube; nu = 1e-5 as a
    lattice value would make them several hundred times larger."""
    return nu * n


def random_force(shape, D: int, amplitude: float = 1e-6, seed: int = 7):
    """Seeded body-force density field [D, ...shape], amplitude * N(0, 1)."""
    rng = np.random.default_rng(seed)
    return amplitude * rng.standard_normal((D,) + tuple(shape))


# The five synthetic workloads, with the paper-shaped parameters.
TGV2D_64 = Workload("d2q9_tgv_64", "D2Q9", (64, 64), 0.01, 1000)
SHEAR_1024 = Workload("d2q9_shear_layer_1024", "D2Q9", (1024, 1024), 1e-5, 20000)
TGV3D_256 = Workload("d3q27_tgv_256_re1600", "D3Q27", (256, 256, 256),
                     (0.1 / math.sqrt(3.0)) * (256 / (2 * math.pi)) / 1600.0, 5000)
ADJ2D_256 = Workload("d2q9_adjoint_256", "D2Q9", (256, 256), 1e-4, 200)
ADJ3D_128 = Workload("d3q27_adjoint_128", "D3Q27", (128, 128, 128),
                     (0.1 / math.sqrt(3.0)) * (128 / (2 * math.pi)) / 1600.0, 500)


def fields_for(wl: Workload, shape=None, seed: int | None = None):
    """(rho, u) of a workload, optionally on another grid ``shape``."""
    shp = wl.shape if shape is None else tuple(shape)
    if wl.name.startswith("d2q9_tgv"):
        assert shp[0] == shp[1]
        return taylor_green_2d(shp[0])
    if wl.name.startswith("d2q9_shear"):
        return shear_layer(shp[1], ny=shp[0])
    if wl.name.startswith("d3q27_tgv") or wl.name.startswith("d3q27_adjoint"):
        return taylor_green_3d(shp[0], shape=shp, seed=1600 if seed is None else seed)
    if wl.name.startswith("d2q9_adjoint"):
        assert shp[0] == shp[1]
        return random_divfree_2d(shp[0], seed=3 if seed is None else seed)
    raise KeyError(wl.name)
