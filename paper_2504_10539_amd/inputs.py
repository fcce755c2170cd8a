"""Seeded synthetic inputs shared by the GPU path's callers and the oracle tests.

This module holds random draws and workload recipes only; none of the
method's arithmetic (density profile, noise, collision, metrics) lives here,
so it can serve both sides of a parity test without coupling them.

The paper (Li & Zhang, arXiv 2504.10539, Sec. III-A) simulates a single
droplet in a square periodic domain; it uses no dataset.  The recipes below
are synthetic droplet workloads of that kind at several scales.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Fluid set-up of the droplet runs: liquid/gas densities near the G = -5
# coexistence pair, tanh interface width 2, uniform noise +-1e-3.
RHO_L = 2.0
RHO_G = 0.15
WIDTH = 2.0
NOISE = 1e-3


def single_droplet(n: int, radius: float) -> np.ndarray:
    """One droplet centred at (n/2, n/2)."""
    return np.array([[n / 2.0, n / 2.0, float(radius)]], dtype=np.float64)


def many_droplets(n: int, count: int, rmin: float, rmax: float, seed: int) -> np.ndarray:
    """`count` droplets, centres uniform in [0, n)^2, radii uniform in [rmin, rmax]."""
    rng = np.random.default_rng(seed)
    cx = rng.uniform(0.0, n, count)
    cy = rng.uniform(0.0, n, count)
    r = rng.uniform(rmin, rmax, count)
    return np.ascontiguousarray(np.stack([cx, cy, r], axis=1))


def random_positive_state(nx: int, ny: int, seed: int, lo: float = 0.02,
                          hi: float = 0.3) -> np.ndarray:
    """Arbitrary positive populations f[9][ny][nx] (not an equilibrium)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(9, ny, nx))


def sweep_grid(n_g: int = 32, n_tau: int = 16):
    """(G, tau) pairs of the parameter sweep: G on [-6.0, -4.5] x tau on [0.55, 1.5]."""
    gs = np.linspace(-6.0, -4.5, n_g)
    taus = np.linspace(0.55, 1.5, n_tau)
    return [(float(g), float(t)) for g in gs for t in taus]


@dataclass
class Request:
    """One droplet simulation request of the serving workload."""
    arrival: float
    n: int
    G: float
    tau: float
    steps: int
    drops: np.ndarray = field(repr=False)
    seed: int = 0


def serving_trace(count: int, rate: float, seed: int, nmin: int = 64, nmax: int = 2048,
                  smin: int = 500, smax: int = 20000) -> list[Request]:
    """Poisson arrivals of droplet requests.

    Grid N log-uniform in [nmin, nmax]; G uniform in [-6.0, -4.5]; tau uniform
    in [0.6, 1.2]; 1-8 droplets with R uniform in [6, N/6] and centres uniform
    in [0, N)^2; steps log-uniform in [smin, smax]."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for k in range(count):
        t += rng.exponential(1.0 / rate) if rate > 0 else 0.0
        n = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
        g = float(rng.uniform(-6.0, -4.5))
        tau = float(rng.uniform(0.6, 1.2))
        nd = int(rng.integers(1, 9))
        r = rng.uniform(6.0, max(6.0, n / 6.0), nd)
        cx = rng.uniform(0.0, n, nd)
        cy = rng.uniform(0.0, n, nd)
        steps = int(round(math.exp(rng.uniform(math.log(smin), math.log(smax)))))
        out.append(Request(t, n, g, tau, steps, np.ascontiguousarray(np.stack([cx, cy, r], 1)),
                           seed=1000 + k))
    return out
