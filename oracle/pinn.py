"""Plain FP64 oracle of the PINN surrogate and of the interface correction.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``): the tests, the smoke
check and the benchmark's CPU leg are the only code that may import it.

Li & Zhang, arXiv 2504.10539:
  - Sec. II-B, Eq. (2): the network N(x, y) = [rho, u_x, u_y] maps spatial
    coordinates to the fluid fields;
  - Sec. III-B: fully connected, 2 inputs, hidden layers of 64, 128, 128 and
    64 neurons with tanh activation, 3 outputs;
  - Sec. II-C: the network's prediction corrects the LBM state, with the
    emphasis on interface regions;
  - Sec. II-D, Eq. (9) and Sec. IV-E, Eq. (16): the interface criterion
    |grad rho| > 0.01 with central differences.

Readings where the paper is silent (each is stated where it is used):
  - the coordinates fed to the network are the cell centres scaled to
    (-1, 1): x_hat = (2 x + 1) / nx - 1, y_hat = (2 y + 1) / ny - 1;
  - the output layer is linear (tanh only on the hidden layers);
  - the correction acts on interface cells only (Eq. (9)'s criterion on the
    state's density): there rho' = rho + beta (rho_N - rho) and
    u' = u + beta (u_N - u), u = sum_i f_i e_i / rho the velocity of the
    populations; the populations become f_i + f_eq_i(rho', u') -
    f_eq_i(rho, u), which keeps their non-equilibrium part and gives the cell
    exactly the mass rho' and momentum rho' u'.  Every other cell is left as
    it is.

Everything is the plain definition in FP64 with numpy's matrix product as a
step; no blocking or fusion.
"""
from __future__ import annotations

import numpy as np

import oracle

# Sec. III-B: layer widths, input to output.
LAYERS = (2, 64, 128, 128, 64, 3)
# Eq. (9): the interface threshold on |grad rho|.
INTERFACE_THRESHOLD = 0.01


def param_count() -> int:
    """Weights and biases of the network, in the packed order of `unpack`."""
    return sum(o * i + o for i, o in zip(LAYERS[:-1], LAYERS[1:]))


def unpack(params: np.ndarray):
    """Split a flat parameter vector into [(W_1, b_1), ..., (W_5, b_5)]; W_l has
    shape (out, in) (a layer maps h to W_l h + b_l), in layer order, each W_l
    row-major followed by its b_l."""
    p = np.asarray(params, dtype=np.float64).ravel()
    assert p.size == param_count(), p.size
    out, o = [], 0
    for i, n in zip(LAYERS[:-1], LAYERS[1:]):
        W = p[o:o + n * i].reshape(n, i)
        o += n * i
        b = p[o:o + n]
        o += n
        out.append((W, b))
    return out


def coordinates(nx: int, ny: int) -> np.ndarray:
    """Network inputs of every cell, shape (ny * nx, 2), row-major in (y, x):
    the cell centres scaled to (-1, 1) (reading: the paper feeds "spatial
    coordinates" without a scale; raw lattice indices would saturate tanh)."""
    x = (2.0 * np.arange(nx) + 1.0) / nx - 1.0
    y = (2.0 * np.arange(ny) + 1.0) / ny - 1.0
    X, Y = np.meshgrid(x, y)
    return np.stack([X.ravel(), Y.ravel()], axis=1)


def mlp_forward(params: np.ndarray, xy: np.ndarray) -> np.ndarray:
    """Eq. (2) with the Sec. III-B network: h_0 = (x, y), h_l = tanh(W_l h_{l-1}
    + b_l) for the four hidden layers, N = W_5 h_4 + b_5 (linear output).
    xy: (n, 2); returns (n, 3) = (rho, u_x, u_y)."""
    layers = unpack(params)
    h = np.asarray(xy, dtype=np.float64)
    for k, (W, b) in enumerate(layers):
        h = h @ W.T + b
        if k < len(layers) - 1:
            h = np.tanh(h)
    return h


def predict_fields(params: np.ndarray, nx: int, ny: int):
    """The network's rho, u_x, u_y on every cell, each of shape (ny, nx)."""
    out = mlp_forward(params, coordinates(nx, ny))
    return tuple(out[:, k].reshape(ny, nx) for k in range(3))


def interface_mask(rho: np.ndarray) -> np.ndarray:
    """Cells that Eq. (9) counts as interface: |grad rho| > 0.01 (strict), with
    the central differences of Eq. (16) and the domain's periodic wrap."""
    return oracle.grad_mag(rho) > INTERFACE_THRESHOLD


def equilibrium_field(rho: np.ndarray, ux: np.ndarray, uy: np.ndarray) -> np.ndarray:
    """Second-order equilibrium of every cell, shape (9, ny, nx): f_eq_i =
    w_i rho (1 + 3 e_i.u + 4.5 (e_i.u)^2 - 1.5 u.u) in the oracle's population
    order."""
    ex, ey, w = oracle.lattice()
    usq = ux * ux + uy * uy
    out = np.empty((9,) + rho.shape)
    for i in range(9):
        eu = ex[i] * ux + ey[i] * uy
        out[i] = w[i] * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * usq)
    return out


def velocity(f: np.ndarray):
    """rho = sum_i f_i and the velocity of the populations u = sum_i f_i e_i / rho."""
    ex, ey, _ = oracle.lattice()
    rho = f.sum(axis=0)
    jx = np.tensordot(ex.astype(np.float64), f, axes=(0, 0))
    jy = np.tensordot(ey.astype(np.float64), f, axes=(0, 0))
    return rho, jx / rho, jy / rho


def correct(f: np.ndarray, params: np.ndarray, beta: float, mask: np.ndarray | None = None):
    """Sec. II-C correction of the pre-collision state f (9, ny, nx) by the
    network `params` with blending factor beta.  `mask` (bool, (ny, nx)) are
    the cells to correct; by default the interface cells of f's density.
    Returns (corrected f, mask)."""
    f = np.asarray(f, dtype=np.float64)
    _, ny, nx = f.shape
    rho, ux, uy = velocity(f)
    if mask is None:
        mask = interface_mask(rho)
    rn, uxn, uyn = predict_fields(params, nx, ny)
    r2 = rho + beta * (rn - rho)
    ux2 = ux + beta * (uxn - ux)
    uy2 = uy + beta * (uyn - uy)
    delta = equilibrium_field(r2, ux2, uy2) - equilibrium_field(rho, ux, uy)
    return np.where(mask[None], f + delta, f), mask
