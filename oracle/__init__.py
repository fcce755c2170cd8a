"""Plain FP64 CPU oracle of the D2Q9 Shan-Chen step and the interface metrics.

TEST INFRASTRUCTURE ONLY.  The test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` are the only code that may import this
package.  The GPU library and its Python binding never import it, and the two
share no code: the oracle is C in ``sc_oracle.c`` (compiled with gcc, no
fast-math) plus the literal Python brute force in ``bruteforce.py`` and the
coexistence solver in ``coexistence.py``.

Each function cites the passage of Li & Zhang, arXiv 2504.10539, that it
follows; see the header of ``sc_oracle.c`` for the conventions (population
order, weights, layout ``f[i][y][x]``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Iterable

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sc_oracle.c")
_LIB = os.path.join(_HERE, "_liboracle.so")

_dbl_p = ctypes.POINTER(ctypes.c_double)
_int_p = ctypes.POINTER(ctypes.c_int)


def build(force: bool = True) -> str:
    """Compile ``sc_oracle.c`` into ``_liboracle.so`` (gcc -O2, no fast-math)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + f".tmp{os.getpid()}"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
           "-fno-fast-math", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(_LIB)
        L.oracle_lattice.argtypes = [_int_p, _int_p, _dbl_p]
        L.oracle_psi.argtypes = [ctypes.c_double]
        L.oracle_psi.restype = ctypes.c_double
        L.oracle_equilibrium.argtypes = [ctypes.c_double] * 3 + [_dbl_p]
        L.oracle_density.argtypes = [ctypes.c_int, ctypes.c_int, _dbl_p, _dbl_p]
        L.oracle_force.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                   _dbl_p, _dbl_p, _dbl_p]
        L.oracle_step.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                  ctypes.c_double, _dbl_p, ctypes.c_long, ctypes.c_int]
        L.oracle_step.restype = ctypes.c_int
        L.oracle_moments.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                     _dbl_p, _dbl_p, _dbl_p, _dbl_p]
        L.oracle_moments.restype = ctypes.c_int
        L.oracle_conservation.argtypes = [ctypes.c_int, ctypes.c_int, _dbl_p, _dbl_p]
        L.oracle_grad_mag.argtypes = [ctypes.c_int, ctypes.c_int, _dbl_p, _dbl_p]
        L.oracle_metrics.argtypes = [ctypes.c_int, ctypes.c_int, _dbl_p, _dbl_p]
        L.oracle_metrics.restype = ctypes.c_int
        L.oracle_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.oracle_splitmix64.restype = ctypes.c_uint64
        L.oracle_uniform01.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.oracle_uniform01.restype = ctypes.c_double
        L.oracle_init_density.argtypes = [
            ctypes.c_int, ctypes.c_int, _dbl_p, ctypes.c_int, ctypes.c_double,
            ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
            ctypes.c_long, ctypes.c_long, ctypes.c_long, ctypes.c_long, _dbl_p]
        L.oracle_init_populations.argtypes = [ctypes.c_int, ctypes.c_int, _dbl_p, _dbl_p]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dbl_p)


def lattice():
    """Velocities e_i and weights w_i in the oracle's population order."""
    ex = (ctypes.c_int * 9)()
    ey = (ctypes.c_int * 9)()
    w = (ctypes.c_double * 9)()
    lib().oracle_lattice(ex, ey, w)
    return np.array(ex[:]), np.array(ey[:]), np.array(w[:])


def psi(rho: float) -> float:
    """psi(rho) = 1 - exp(-rho) (pseudopotential, Sec. II-A reading)."""
    return lib().oracle_psi(float(rho))


def equilibrium(rho: float, ux: float, uy: float) -> np.ndarray:
    """Second-order BGK equilibrium populations (Eq. (1) collision operator)."""
    out = np.zeros(9)
    lib().oracle_equilibrium(float(rho), float(ux), float(uy), _p(out))
    return out


def density(f: np.ndarray) -> np.ndarray:
    f = np.ascontiguousarray(f, dtype=np.float64)
    _, ny, nx = f.shape
    rho = np.zeros((ny, nx))
    lib().oracle_density(nx, ny, _p(f), _p(rho))
    return rho


def force(rho: np.ndarray, G: float):
    """Interaction force F = -G psi(x) sum_i w_i psi(x+e_i) e_i (Sec. II-A)."""
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    ny, nx = rho.shape
    Fx = np.zeros_like(rho)
    Fy = np.zeros_like(rho)
    lib().oracle_force(nx, ny, float(G), _p(rho), _p(Fx), _p(Fy))
    return Fx, Fy


def step(f: np.ndarray, G: float, tau: float, nsteps: int = 1, nthreads: int = 1) -> np.ndarray:
    """Advance the pre-collision state by ``nsteps`` steps of Eq. (1); returns a copy."""
    f = np.array(f, dtype=np.float64, order="C", copy=True)
    q, ny, nx = f.shape
    assert q == 9
    rc = lib().oracle_step(nx, ny, float(G), float(tau), _p(f), int(nsteps), int(nthreads))
    if rc != 0:
        raise RuntimeError(f"oracle_step failed ({rc})")
    return f


def moments(f: np.ndarray, G: float):
    """rho and the half-force-corrected velocity u = (j + F/2)/rho."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    _, ny, nx = f.shape
    rho, ux, uy = (np.zeros((ny, nx)) for _ in range(3))
    rc = lib().oracle_moments(nx, ny, float(G), _p(f), _p(rho), _p(ux), _p(uy))
    if rc != 0:
        raise RuntimeError("oracle_moments failed")
    return rho, ux, uy


def conservation(f: np.ndarray):
    """(total mass, total momentum x, total momentum y) of the state."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    _, ny, nx = f.shape
    out = np.zeros(3)
    lib().oracle_conservation(nx, ny, _p(f), _p(out))
    return float(out[0]), float(out[1]), float(out[2])


def grad_mag(rho: np.ndarray) -> np.ndarray:
    """Eq. (16) central-difference |grad rho| with periodic wrap."""
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    ny, nx = rho.shape
    g = np.zeros_like(rho)
    lib().oracle_grad_mag(nx, ny, _p(rho), _p(g))
    return g


METRIC_KEYS = ("W", "Gmax", "drho", "W_eff", "E_int", "n_above", "rho_max", "rho_min", "sum_grad")


def metrics(rho: np.ndarray) -> dict:
    """Interface metrics of Eqs. (9)-(15) on a density field."""
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    ny, nx = rho.shape
    out = np.zeros(9)
    rc = lib().oracle_metrics(nx, ny, _p(rho), _p(out))
    if rc != 0:
        raise RuntimeError("oracle_metrics failed")
    return dict(zip(METRIC_KEYS, (float(v) for v in out)))


def splitmix64(seed: int, k: int) -> int:
    return int(lib().oracle_splitmix64(seed, k))


def uniform01(seed: int, k: int) -> float:
    return float(lib().oracle_uniform01(seed, k))


def init_density(nx: int, ny: int, drops: Iterable, rho_l: float, rho_g: float,
                 width: float, noise_amp: float, seed: int,
                 period=(0, 0), origin=(0, 0)) -> np.ndarray:
    """Droplet initial density on an nx x ny window (Sec. III-A set-up)."""
    d = np.ascontiguousarray(np.asarray(list(drops) if not isinstance(drops, np.ndarray) else drops,
                                        dtype=np.float64).reshape(-1, 3))
    rho = np.zeros((ny, nx))
    n = d.shape[0]
    dp = _p(d) if n else ctypes.cast(0, _dbl_p)
    lib().oracle_init_density(nx, ny, dp, n, float(rho_l), float(rho_g), float(width),
                              float(noise_amp), int(seed) & (2**64 - 1), int(period[0]),
                              int(period[1]), int(origin[0]), int(origin[1]), _p(rho))
    return rho


def init_populations(rho: np.ndarray) -> np.ndarray:
    """f_i = w_i rho (fluid at rest)."""
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    ny, nx = rho.shape
    f = np.zeros((9, ny, nx))
    lib().oracle_init_populations(nx, ny, _p(rho), _p(f))
    return f


def droplet_state(nx: int, ny: int, drops, rho_l=2.0, rho_g=0.15, width=2.0,
                  noise_amp=1e-3, seed=1, period=(0, 0), origin=(0, 0)) -> np.ndarray:
    """Initial populations of a droplet run."""
    return init_populations(init_density(nx, ny, drops, rho_l, rho_g, width, noise_amp,
                                         seed, period, origin))
