"""Seeded single-cell test states for the oracle and parity tests."""
import numpy as np

import oracle


def null_space_direction(D, rng):
    """Random unit vector orthogonal to {1, c_x, ..., c_D} (moment preserving)."""
    c, _ = oracle.lattice(D)
    M = np.vstack([np.ones(len(c))] + [c[:, a] for a in range(D)]).T  # [Q, 1+D]
    v = rng.standard_normal(len(c))
    q, _ = np.linalg.qr(M)
    v = v - q @ (q.T @ v)
    return v / np.linalg.norm(v)


def perturbed_state(D, eps, rng, rho=None, u=None, direction=None):
    """g = feq(rho, u) * (1 + eps * d) with d moment-free after scaling.

    Returns (g, feq).  The perturbation keeps rho and u, so feq(g) = feq.
    """
    if rho is None:
        rho = 1.0 + 0.05 * rng.standard_normal()
    if u is None:
        u = 0.08 * rng.standard_normal(D)
    feq = oracle.equilibrium(D, rho, u)
    d = null_space_direction(D, rng) if direction is None else direction
    g = feq + eps * d * feq.max()
    return g, feq
