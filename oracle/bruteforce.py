"""Literal pure-Python brute force of one Shan-Chen LBM step, for tiny grids.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  This is written
independently of ``sc_oracle.c`` so that the two pin each other:

* the lattice is built by enumerating the nine velocities and giving each the
  D2Q9 weight that belongs to its squared length (0 -> 4/9, 1 -> 1/9,
  2 -> 1/36) instead of a typed-in table;
* the equilibrium is the Hermite form with the sound speed written out,
  w rho (1 + e.u / c_s^2 + (e.u)^2 / (2 c_s^4) - u.u / (2 c_s^2)), c_s^2 = 1/3;
* streaming is done by pulling, f_i(x, t+1) = f*_i(x - e_i), where the C
  oracle pushes;
* the force is the neighbour sum of Sec. II-A read as a sum over lattice
  neighbours, F = -G psi(x) sum_i w_i psi(x + e_i) e_i, psi = 1 - exp(-rho).

Source: Li & Zhang, arXiv 2504.10539, Sec. II-A Eq. (1) and Sec. III-A
(periodic square domain).  Only the population ORDER is shared with the C
oracle, because arrays are compared element by element; it is passed in.
"""
from __future__ import annotations

import math

CS2 = 1.0 / 3.0


def weight_of(ex: int, ey: int) -> float:
    """D2Q9 weight from the squared speed of the velocity."""
    return {0: 4.0 / 9.0, 1: 1.0 / 9.0, 2: 1.0 / 36.0}[ex * ex + ey * ey]


def velocities(order):
    """order: list of (ex, ey) pairs; returns list of (ex, ey, w)."""
    assert sorted(order) == sorted((a, b) for a in (-1, 0, 1) for b in (-1, 0, 1))
    return [(ex, ey, weight_of(ex, ey)) for ex, ey in order]


def psi(rho: float) -> float:
    return 1.0 - math.exp(-rho)


def feq(w: float, ex: int, ey: int, rho: float, ux: float, uy: float) -> float:
    eu = ex * ux + ey * uy
    uu = ux * ux + uy * uy
    return w * rho * (1.0 + eu / CS2 + eu * eu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2))


def step(f, G: float, tau: float, order):
    """f: nested lists f[i][y][x]; returns the state after one step."""
    lat = velocities(order)
    q = len(lat)
    ny = len(f[0])
    nx = len(f[0][0])
    rho = [[sum(f[i][y][x] for i in range(q)) for x in range(nx)] for y in range(ny)]
    ps = [[psi(rho[y][x]) for x in range(nx)] for y in range(ny)]
    fstar = [[[0.0] * nx for _ in range(ny)] for _ in range(q)]
    for y in range(ny):
        for x in range(nx):
            r = rho[y][x]
            jx = sum(f[i][y][x] * lat[i][0] for i in range(q))
            jy = sum(f[i][y][x] * lat[i][1] for i in range(q))
            Fx = 0.0
            Fy = 0.0
            for ex, ey, w in lat:
                if ex == 0 and ey == 0:
                    continue
                pn = ps[(y + ey) % ny][(x + ex) % nx]
                Fx += w * pn * ex
                Fy += w * pn * ey
            Fx *= -G * ps[y][x]
            Fy *= -G * ps[y][x]
            ux = (jx + tau * Fx) / r
            uy = (jy + tau * Fy) / r
            for i, (ex, ey, w) in enumerate(lat):
                fi = f[i][y][x]
                fstar[i][y][x] = fi + (feq(w, ex, ey, r, ux, uy) - fi) / tau
    out = [[[0.0] * nx for _ in range(ny)] for _ in range(q)]
    for i, (ex, ey, _w) in enumerate(lat):
        for y in range(ny):
            for x in range(nx):
                out[i][y][x] = fstar[i][(y - ey) % ny][(x - ex) % nx]
    return out


def moments(f, G: float, order):
    """rho and u = (j + F/2)/rho of a state, as nested lists."""
    lat = velocities(order)
    q = len(lat)
    ny = len(f[0])
    nx = len(f[0][0])
    rho = [[sum(f[i][y][x] for i in range(q)) for x in range(nx)] for y in range(ny)]
    ps = [[psi(rho[y][x]) for x in range(nx)] for y in range(ny)]
    ux = [[0.0] * nx for _ in range(ny)]
    uy = [[0.0] * nx for _ in range(ny)]
    for y in range(ny):
        for x in range(nx):
            Fx = Fy = 0.0
            for ex, ey, w in lat:
                pn = ps[(y + ey) % ny][(x + ex) % nx]
                Fx += w * pn * ex
                Fy += w * pn * ey
            Fx *= -G * ps[y][x]
            Fy *= -G * ps[y][x]
            jx = sum(f[i][y][x] * lat[i][0] for i in range(q))
            jy = sum(f[i][y][x] * lat[i][1] for i in range(q))
            ux[y][x] = (jx + Fx / 2.0) / rho[y][x]
            uy[y][x] = (jy + Fy / 2.0) / rho[y][x]
    return rho, ux, uy


def metrics(rho):
    """Eqs. (9)-(16) with explicit loops over cells (nested-list density)."""
    ny = len(rho)
    nx = len(rho[0])
    grads = []
    for j in range(ny):
        for i in range(nx):
            dx = (rho[j][(i + 1) % nx] - rho[j][(i - 1) % nx]) / 2.0
            dy = (rho[(j + 1) % ny][i] - rho[(j - 1) % ny][i]) / 2.0
            grads.append(math.sqrt(dx * dx + dy * dy))
    flat = [v for row in rho for v in row]
    gmax = max(grads)
    n = nx * ny
    return {
        "W": sum(1 for g in grads if g > 0.01) / n,
        "Gmax": gmax,
        "drho": max(flat) - min(flat),
        "W_eff": (sum(grads) / (gmax * n)) if gmax > 0 else 0.0,
        "E_int": sum(g * g for g in grads),
    }
