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


def unstream(g):
    """The state f whose pull-streamed image is g: f_i(y) = g_i(y + c_i).

    Streaming is a permutation (Eq. advection), so this builds lattices whose
    pulled populations have a prescribed distance from equilibrium."""
    D = g.ndim - 1
    c, _ = oracle.lattice(D)
    out = np.empty_like(g)
    for i in range(c.shape[0]):
        shift = tuple(-int(c[i, a]) for a in reversed(range(D)))
        out[i] = np.roll(g[i], shift, axis=tuple(range(D)))
    return out


def three_regime_state(D, shape, seed):
    """A lattice whose pulled cells fall, about a third each, inside the gate
    (max|x| < 1e-3), in the small-departure band (1e-3 <= max|x| < 5e-3) and
    far from equilibrium (max|x| up to ~0.06): per-cell relative amplitudes
    2e-4, 1.5e-3 and 3e-2 on an equilibrium with random rho and u."""
    rng = np.random.default_rng(seed)
    u = 0.03 * rng.standard_normal((D,) + tuple(shape))
    rho = 1 + 0.01 * rng.standard_normal(tuple(shape))
    g = oracle.init_equilibrium(rho, u)
    amp = rng.choice([2e-4, 1.5e-3, 3e-2], size=tuple(shape))
    g = g * (1 + amp * rng.uniform(-1, 1, g.shape))
    return unstream(g)


def mixed_mirror_lattice(D, shape, seed, sigma=1.2, amps=(2e-4, 4e-3, 1.2e-2, 0.05)):
    """Pulled cells in five kinds, about a fifth each: relative perturbations
    of an equilibrium (random rho, u) of uniform amplitude 2e-4 (gated),
    4e-3 and 1.2e-2 (max|x| from 1.4e-3 to 2.5e-2: the power-series range of
    the path-length sums), 0.05 (their exact range), and log-normal
    populations far from equilibrium (often without a mirror root);
    un-streamed so that one step collides exactly these cells."""
    rng = np.random.default_rng(seed)
    u = 0.03 * rng.standard_normal((D,) + tuple(shape))
    rho = 1 + 0.01 * rng.standard_normal(tuple(shape))
    g = oracle.init_equilibrium(rho, u)
    kind = rng.integers(0, len(amps) + 1, size=tuple(shape))
    pert = np.zeros(g.shape)
    for k, a in enumerate(amps):
        pert = np.where(kind == k, a * rng.uniform(-1, 1, g.shape), pert)
    g = g * (1 + pert)
    far = np.exp(rng.normal(0, sigma, g.shape))
    g = np.where(kind == len(amps), g * far, g)
    return unstream(g)
