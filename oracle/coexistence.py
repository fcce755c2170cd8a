"""Equation of state and flat-interface coexistence of the Shan-Chen model.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

In the pseudopotential model of Sec. II-A of Li & Zhang (arXiv 2504.10539)
the interaction force turns the ideal-gas pressure into a non-ideal one, which
is what lets two phases coexist.  With the D2Q9 weights and psi = 1 - exp(-rho)
that equation of state is

    p(rho) = rho / 3 + G psi(rho)^2 / 6                      (c_s^2 = 1/3)

and, expanding the force to fourth order for a flat interface, the bulk
densities of the two coexisting phases satisfy the mechanical-stability
condition

    p(rho_g) = p(rho_l) = p0,
    integral_{rho_g}^{rho_l} (p0 - p(rho)) psi'(rho) / psi(rho)^2 d rho = 0,

(the force's fourth-order term is an exact derivative once weighted by
psi'/psi^2).  The critical point is G_c = -4, rho_c = ln 2.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate, optimize


def psi(rho):
    return 1.0 - np.exp(-rho)


def dpsi(rho):
    return np.exp(-rho)


def pressure(rho, G):
    """Non-ideal EOS of the pseudopotential model."""
    return rho / 3.0 + G * psi(rho) ** 2 / 6.0


def _residual(x, G):
    rg, rl = x
    if not 0.0 < rg < rl:
        return [1.0, 1.0]
    p0 = pressure(rl, G)
    integral, _ = integrate.quad(lambda r: (p0 - pressure(r, G)) * dpsi(r) / psi(r) ** 2,
                                 rg, rl, epsabs=1e-14, epsrel=1e-13, limit=200)
    return [pressure(rg, G) - p0, integral]


def coexistence(G: float):
    """(rho_g, rho_l) for interaction strength G < -4."""
    if not G < -4.0:
        raise ValueError("no phase separation for G >= G_c = -4")
    # spinodal points bracket the solution: p'(rho) = 0
    dp = lambda r: 1.0 / 3.0 + G * psi(r) * dpsi(r) / 3.0
    rs1 = optimize.brentq(dp, 1e-9, math.log(2.0))
    rs2 = optimize.brentq(dp, math.log(2.0), 20.0)
    if G > -4.5:
        # near the critical point the binodal sits about sqrt(3) spinodal
        # half-widths from the centre (the cubic-EOS limit)
        mid, half = 0.5 * (rs1 + rs2), 0.5 * (rs2 - rs1)
        guess = [mid - 3.0 ** 0.5 * half, mid + 3.0 ** 0.5 * half]
    else:
        guess = [0.5 * rs1, min(2.0 * rs2, rs2 + 2.0)]
    sol, info, ier, msg = optimize.fsolve(_residual, guess, args=(G,), xtol=1e-13,
                                          full_output=True)
    if ier != 1:
        raise RuntimeError(f"coexistence solve failed for G={G}: {msg}")
    rg, rl = float(sol[0]), float(sol[1])
    if not (0.0 < rg < rs1 < rs2 < rl):
        raise RuntimeError(f"coexistence solve left the binodal for G={G}: {rg}, {rl}")
    return rg, rl
