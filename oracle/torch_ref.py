"""FP64 PyTorch (CPU) reference of the ESELBM step, for gradient checks.

TEST INFRASTRUCTURE ONLY (see the package docstring).  A second, vectorised
transcription of the same algorithm as the C oracle, written on its own so
that torch autograd can differentiate it: the gradients it produces are the
reference for the library's hand-written adjoint.  Its forward pass is pinned
to the C oracle and its gradients to central finite differences of the C
oracle (tests/test_oracle_adjoint_ref.py).

Branches are torch.where selections: in a gated cell alpha = 2 carries no
gradient, the Omega+-/Omega- masks are fixed at the point, and the guard's
alpha_max takes its gradient through the smallest x_i.

Parity of the gradients with the paper: unpinned by the paper itself (it has
no adjoint); pinned by finite differences of the oracle.
"""
from __future__ import annotations

import itertools

import torch

THETA0 = 1.0 / 3.0


def lattice(D: int):
    """(c [Q, D] float64, w [Q]) with x fastest in the population index."""
    cs = [tuple(reversed(t)) for t in itertools.product((-1, 0, 1), repeat=D)]
    c = torch.tensor(cs, dtype=torch.float64)
    w1 = {-1: 1.0 / 6.0, 0: 2.0 / 3.0, 1: 1.0 / 6.0}
    w = torch.tensor([float(torch.tensor([w1[int(v)] for v in row], dtype=torch.float64).prod()) for row in c],
                     dtype=torch.float64)
    return c, w


def equilibrium(rho: torch.Tensor, u: torch.Tensor) -> torch.Tensor:
    """Product-form entropic equilibrium (Sec. II); rho [...], u [D, ...]."""
    D = u.shape[0]
    c, w = lattice(D)
    s = torch.sqrt(1.0 + 3.0 * u * u)
    ups = 2.0 - s
    z = (2.0 * u + s) / (1.0 - u)
    out = []
    for i in range(c.shape[0]):
        v = w[i] * rho
        for a in range(D):
            ca = int(c[i, a])
            v = v * ups[a] * (z[a] if ca > 0 else (1.0 / z[a] if ca < 0 else 1.0))
        out.append(v)
    return torch.stack(out)


def moments(f: torch.Tensor, force: torch.Tensor | None = None):
    D = f.dim() - 1
    c, _ = lattice(D)
    rho = f.sum(0)
    j = torch.einsum("i...,ia->a...", f, c.to(f.dtype))
    if force is not None:
        j = j + 0.5 * force
    return rho, j / rho


def _root(a, b, c):
    return 2.0 * c / (b + torch.sqrt(b * b - 4.0 * a * c))


def path_length(g: torch.Tensor, feq: torch.Tensor, beta: float, mode: str = "higher"):
    """alpha per cell (Sec. IV, App. D) for populations [Q, ...]."""
    if mode == "bgk":
        return torch.full_like(g[0], 2.0)
    x = feq / g - 1.0
    xabs = x.abs().max(0).values
    gated = xabs < 1e-3
    # In gated cells alpha = 2 and the closed form is not used; feed it a fixed
    # non-degenerate departure there so that no 0/0 reaches the backward pass.
    Q = x.shape[0]
    dummy = torch.tensor([0.01 * (1 + k % 3) * (1 if k % 2 else -1) for k in range(Q)],
                         dtype=x.dtype).reshape((Q,) + (1,) * (x.dim() - 1))
    xr = x
    x = torch.where(gated.unsqueeze(0), dummy.expand_as(x), x)
    neg = x < 0
    zero = torch.zeros_like(x)
    a1 = torch.where(neg, g * x ** 3 / 2, zero).sum(0)
    b1 = (g * x * x / 2).sum(0)
    c1 = (g * 2 * x * x / (2 + x)).sum(0)
    aL = _root(a1, b1, c1)
    if mode == "lower":
        alpha = aL
    else:
        aLx = aL.unsqueeze(0) * x
        # the Omega+ fractions are only evaluated where x >= 0 (safe values elsewhere)
        xs = torch.where(neg, zero, x)
        ys = torch.where(neg, zero, aLx)
        frac = 2 / (4 + ys) + 1 / (4 + 2 * ys) + 2 / (4 + 3 * ys)
        b = b1 - (2 * aL * beta ** 2 / 15) * torch.where(neg, zero, g * xs ** 3 * frac).sum(0)
        c = (g * (60 * x ** 2 + 60 * x ** 3 + 11 * x ** 4) / (60 + 90 * x + 36 * x ** 2 + 3 * x ** 3)).sum(0)
        a2 = beta ** 2 * torch.where(neg, g * x ** 3 / 6, zero).sum(0)
        h = _root(a2, b, c)
        hb = (h * beta).unsqueeze(0)
        a = beta ** 2 * torch.where(
            neg, g * (x ** 3 / 6 - hb * x ** 4 / 12 + hb ** 2 * x ** 5 / 20 - hb ** 3 * x ** 6 / 5), zero).sum(0)
        alpha = _root(a, b, c)
    alpha = torch.where(gated, torch.full_like(alpha, 2.0), alpha)
    xmin = xr.min(0).values
    safe = torch.where(xmin < 0, xmin, -torch.ones_like(xmin))
    amax = -1.0 / (beta * safe)
    guard = (xmin < 0) & (alpha > amax)
    return torch.where(guard, 0.5 * (1.0 + amax), alpha)


def stream(f: torch.Tensor) -> torch.Tensor:
    """Pull streaming g_i(x) = f_i(x - c_i) on a periodic grid (Eq. advection)."""
    D = f.dim() - 1
    c, _ = lattice(D)
    out = []
    for i in range(c.shape[0]):
        shift = tuple(int(c[i, a]) for a in reversed(range(D)))
        out.append(torch.roll(f[i], shifts=shift, dims=tuple(range(D))))
    return torch.stack(out)


def step(f: torch.Tensor, tau: float, mode: str = "higher", force: torch.Tensor | None = None):
    beta = 1.0 / (2.0 * tau + 1.0)
    g = stream(f)
    rho, u = moments(g)
    feq = equilibrium(rho, u)
    alpha = path_length(g, feq, beta, mode)
    out = g + alpha * beta * (feq - g)
    if force is not None:
        out = out + equilibrium(rho, u + force / rho) - feq
    return out


def kinetic_energy(f: torch.Tensor) -> torch.Tensor:
    rho, u = moments(f)
    return 0.5 * (rho * (u * u).sum(0)).sum()


def vorticity(u: torch.Tensor) -> torch.Tensor:
    """Periodic second-order central differences; [1 or 3, ...]."""
    D = u.shape[0]

    def d(field, axis):  # axis: 0 = x (last array dim)
        dim = field.dim() - 1 - axis
        return 0.5 * (torch.roll(field, -1, dims=dim) - torch.roll(field, 1, dims=dim))

    if D == 2:
        return (d(u[1], 0) - d(u[0], 1)).unsqueeze(0)
    return torch.stack([d(u[2], 1) - d(u[1], 2), d(u[0], 2) - d(u[2], 0), d(u[1], 0) - d(u[0], 1)])


def dissipation(f: torch.Tensor, weight: float, force: torch.Tensor | None = None) -> torch.Tensor:
    _, u = moments(f, force)
    return weight * (vorticity(u) ** 2).sum()
