"""Shared pieces of the shock-tube checks (Sec. V A).

``riemann_entropic`` solves the Riemann problem of the inviscid equations the
D1Q3 lattice carries at equilibrium: mass and momentum with the momentum flux
of the entropic equilibrium, rho P(u), P(u) = (2 sqrt(1 + 3u^2) - 1) / 3 (the
second moment of the D1Q3 closed form of Sec. II).  A left rarefaction is
integrated along the eigenvector of the slower characteristic, a right shock
follows from the Rankine-Hugoniot conditions, and the two meet at the plateau.
This is written from the conservation laws alone, not from the lattice code.
"""
import numpy as np
from scipy.integrate import solve_ivp
from scipy.optimize import brentq


def _P(u):
    return (2.0 * np.sqrt(1.0 + 3.0 * u * u) - 1.0) / 3.0


def _dP(u):
    return 2.0 * u / np.sqrt(1.0 + 3.0 * u * u)


def _lam1(u):
    # eigenvalues of d(m, rho P(m/rho)) / d(rho, m): l^2 - P' l - (P - u P') = 0
    a = _P(u) - u * _dP(u)
    b = _dP(u)
    return (b - np.sqrt(b * b + 4.0 * a)) / 2.0


def riemann_entropic(rho_l, rho_r):
    """(rho*, u*, shock speed) for fluid at rest on both sides, rho_l > rho_r."""
    def u_rare(r):
        # along the 1-wave, d u / d ln rho = lam1(u) - u
        sol = solve_ivp(lambda t, u: [_lam1(u[0]) - u[0]], [np.log(rho_l), np.log(r)], [0.0],
                        rtol=1e-12, atol=1e-14)
        return float(sol.y[0, -1])

    def u_shock(r):
        # S (r - rho_r) = r u ;  S r u = r P(u) - rho_r P(0)
        return brentq(lambda u: (r * u) ** 2 / (r - rho_r) - (r * _P(u) - rho_r / 3.0), 0.0, 1.0,
                      xtol=1e-15)

    rs = brentq(lambda r: u_rare(r) - u_shock(r), rho_r * 1.0001, rho_l * 0.9999, xtol=1e-14)
    us = u_shock(rs)
    return rs, us, rs * us / (rs - rho_r)


def shock_position(rho, plateau, rho_r, lo):
    """Where rho falls through the midpoint between the plateau and rho_r,
    searching from index ``lo`` (linear interpolation between nodes)."""
    mid = 0.5 * (plateau + rho_r)
    idx = int(np.flatnonzero(rho[lo:] > mid)[-1]) + lo
    return idx + (rho[idx] - mid) / (rho[idx] - rho[idx + 1])


def nut_ratio(alpha, beta, tau):
    """nu_T / nu_0 = (2 - alpha) / (2 alpha beta tau) (Eq. nuT over nu_0 = theta tau)."""
    return (2.0 - alpha) / (2.0 * alpha * beta * tau)


def total_variation(rho):
    return float(np.abs(np.diff(rho)).sum())
