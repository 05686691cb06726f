"""Closed forms the pins compare against (independent of the oracle and of the HIP library).

- Bulk pressure of the pseudopotential model: p(rho) = rho/3 + (G/6) psi^2, psi = 1 - exp(-rho)
  (Sec. 3.1, with the printed 0.166 read as G cs^2 / 2 = G/6).
- Spinodals: p'(rho) = 0  <=>  y (1 - y) = -1/G with y = exp(-rho).
- Flat-interface coexistence of the Shan-Chen force (Shan & Chen 1993; Shan 2008 mechanical
  stability condition): p(rho_g) = p(rho_l) = p0 and
  integral_{rho_g}^{rho_l} (p0 - p(rho)) psi'(rho) / psi(rho)^2 d rho = 0.
- Lattice Laplacian eigenvalue: for p = cos(k.x), 6 sum_i w_i (p(x + e_i) - p(x)) = lambda p with
  lambda = 6 sum_i w_i (cos(k.e_i) - 1).
- BGK shear-wave decay: kinematic viscosity nu = (tau - 1/2)/3.
"""
import math

import numpy as np
from scipy import integrate, optimize


def psi(rho):
    return 1.0 - np.exp(-rho)


def pressure(rho, G):
    return rho / 3.0 + (G / 6.0) * psi(rho) ** 2


def dpressure(rho, G):
    return 1.0 / 3.0 + (G / 3.0) * psi(rho) * np.exp(-rho)


def spinodals(G):
    """(lower, upper) spinodal densities, G < -4."""
    disc = math.sqrt(1.0 + 4.0 / G)
    y_hi, y_lo = (1.0 + disc) / 2.0, (1.0 - disc) / 2.0
    return -math.log(y_hi), -math.log(y_lo)


def coexistence(G):
    """(rho_g, rho_l, p0) of a flat interface by the mechanical-stability condition."""
    lo, hi = spinodals(G)

    def integrand(r, p0):
        dpsi = math.exp(-r)
        return (p0 - float(pressure(r, G))) * dpsi / float(psi(r)) ** 2

    def residual(v):
        rg, rl = v
        p0 = float(pressure(rl, G))
        r1 = float(pressure(rg, G)) - p0
        r2, _ = integrate.quad(integrand, rg, rl, args=(p0,), epsabs=1e-13, epsrel=1e-12,
                               limit=200)
        return [r1, r2]

    sol = optimize.fsolve(residual, [0.6 * lo, 1.4 * hi], xtol=1e-13)
    rg, rl = float(sol[0]), float(sol[1])
    return rg, rl, float(pressure(rl, G))


def maxwell(G):
    """Equal-area (Maxwell) densities in the p - 1/rho plane, for contrast only."""
    def residual(v):
        rg, rl = v
        p0 = float(pressure(rl, G))
        area, _ = integrate.quad(lambda r: (float(pressure(r, G)) - p0) / (r * r), rg, rl,
                                 epsabs=1e-13)
        return [float(pressure(rg, G)) - p0, area]

    lo, hi = spinodals(G)
    sol = optimize.fsolve(residual, [0.6 * lo, 1.4 * hi], xtol=1e-13)
    return float(sol[0]), float(sol[1])


def laplacian_eigenvalue(q, k):
    """lambda for the lattice Laplacian 6 sum w_i (p(x+e_i) - p(x)) on cos(k.x)."""
    if q == 9:
        vecs = [(ex, ey, 0) for ey in (-1, 0, 1) for ex in (-1, 0, 1)]
        wt = {0: 4 / 9, 1: 1 / 9, 2: 1 / 36}
    else:
        vecs = [(ex, ey, ez) for ez in (-1, 0, 1) for ey in (-1, 0, 1) for ex in (-1, 0, 1)
                if ex * ex + ey * ey + ez * ez <= 2]
        wt = {0: 1 / 3, 1: 1 / 18, 2: 1 / 36}
    lam = 0.0
    for e in vecs:
        m = sum(c * c for c in e)
        lam += wt[m] * (math.cos(sum(ki * ei for ki, ei in zip(k, e))) - 1.0)
    return 6.0 * lam
