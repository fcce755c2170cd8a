"""Training of the PINN surrogate and the coupling loop, in PyTorch.

Li & Zhang, arXiv 2504.10539:
  - Sec. II-B, Eq. (2): N(x, y) = [rho, u_x, u_y];
  - Sec. III-B: 2 -> 64 -> 128 -> 128 -> 64 -> 3, tanh, learning rate 3e-4,
    300 epochs per coupling step;
  - Eqs. (3)-(8): L = L_data + lambda_1 L_phys + lambda_2 L_interface;
  - Sec. II-C / III-C: LBM steps, train on the current state, correct the
    state at the interfaces, continue; evolution segments with decreasing
    epochs.

Training runs on PyTorch (outside the library's hot path); the trained
parameters are packed in the C-ABI order (include/lbm.h, LBM_PINN_PARAMS) and
the correction itself runs in the library's kernels (lbm_pinn_correct).

Readings where the paper is silent or garbled:
  - inputs are the cell centres scaled to (-1, 1); the output layer is linear;
  - the velocity the network learns and the correction blends is the
    populations' own u = sum_i f_i e_i / rho (the correction then sets a
    cell's mass and momentum exactly; the half-force velocity of
    lbm_moments differs from it by F / (2 rho));
  - the network has no time input, so the time derivatives of Eqs. (6)-(7)
    are taken as zero (steady residuals): continuity div(rho u) and momentum
    div(rho u u) + grad p - div sigma, with p the pseudopotential equation of
    state rho / 3 + G psi^2 / 6 and sigma = rho nu (grad u + grad u^T),
    nu = (tau - 1/2) / 3, derivatives in lattice units (d/dx = (2 / nx) d/dx_hat);
  - Eq. (8) as printed (alpha_1 |grad rho|^2 - alpha_2 |grad rho|^4) contradicts
    its own description (a negative quadratic term that rewards sharp
    gradients, a positive quartic term against oscillations); the description
    is taken: -alpha_1 |grad rho|^2 + alpha_2 |grad rho|^4, on the interface
    points (|grad rho| > 0.01 of the LBM data);
  - lambda_1, lambda_2, alpha_1, alpha_2, the optimiser and the collocation
    sets are not given: Adam, and the defaults below;
  - "decreasing training epochs" over the five evolution segments: 300, 240,
    180, 120, 60.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

LAYERS = (2, 64, 128, 128, 64, 3)
PARAM_COUNT = sum(o * i + o for i, o in zip(LAYERS[:-1], LAYERS[1:]))


def _torch():
    import torch
    return torch


def make_net(seed: int = 0, device="cpu", dtype=None):
    """The Sec. III-B network with PyTorch's default initialisation."""
    torch = _torch()
    torch.manual_seed(seed)
    mods = []
    for k, (i, o) in enumerate(zip(LAYERS[:-1], LAYERS[1:])):
        mods.append(torch.nn.Linear(i, o))
        if k < len(LAYERS) - 2:
            mods.append(torch.nn.Tanh())
    net = torch.nn.Sequential(*mods).to(device)
    if dtype is not None:
        net = net.to(dtype)
    return net


def pack(net):
    """The network's parameters as one FP32 tensor in the C-ABI order: per
    layer, W (out x in, row-major) then b."""
    torch = _torch()
    parts = []
    for m in net:
        if isinstance(m, torch.nn.Linear):
            parts += [m.weight.detach().reshape(-1), m.bias.detach().reshape(-1)]
    p = torch.cat(parts).to(torch.float32).contiguous()
    assert p.numel() == PARAM_COUNT
    return p


def coords(nx: int, ny: int, device="cpu", dtype=None):
    """(ny * nx, 2) cell centres scaled to (-1, 1), row-major in (y, x)."""
    torch = _torch()
    dtype = dtype or torch.float32
    x = (2.0 * torch.arange(nx, device=device, dtype=dtype) + 1.0) / nx - 1.0
    y = (2.0 * torch.arange(ny, device=device, dtype=dtype) + 1.0) / ny - 1.0
    Y, X = torch.meshgrid(y, x, indexing="ij")
    return torch.stack([X.reshape(-1), Y.reshape(-1)], 1)


@dataclass
class LossWeights:
    lambda_phys: float = 1e-2
    lambda_interface: float = 1e-3
    alpha1: float = 1.0
    alpha2: float = 1.0


def _grad(out, inp):
    torch = _torch()
    return torch.autograd.grad(out, inp, torch.ones_like(out), create_graph=True)[0]


def losses(net, xy, target, interface, nx, ny, G, tau, w: LossWeights):
    """(total, data, phys, interface) losses of Eqs. (3)-(8) at the points xy
    (requires_grad), with the LBM fields `target` (n, 3) there and the boolean
    `interface` selection of interface points."""
    torch = _torch()
    out = net(xy)
    rho, ux, uy = out[:, 0], out[:, 1], out[:, 2]
    l_data = ((out - target) ** 2).sum(1).mean()                      # Eq. (4)
    sx, sy = 2.0 / nx, 2.0 / ny                                       # d/dx = sx d/dx_hat

    def d(f):
        g = _grad(f, xy)
        return g[:, 0] * sx, g[:, 1] * sy

    nu = (tau - 0.5) / 3.0
    mx, my = rho * ux, rho * uy
    cont = d(mx)[0] + d(my)[1]                                        # Eq. (6), steady
    psi = 1.0 - torch.exp(-rho)
    p = rho / 3.0 + G * psi * psi / 6.0
    dpx, dpy = d(p)
    uxx, uxy = d(ux)
    uyx, uyy = d(uy)
    sxx, sxy, syy = rho * nu * 2 * uxx, rho * nu * (uxy + uyx), rho * nu * 2 * uyy
    ns_x = d(mx * ux)[0] + d(mx * uy)[1] + dpx - (d(sxx)[0] + d(sxy)[1])   # Eq. (7), steady
    ns_y = d(my * ux)[0] + d(my * uy)[1] + dpy - (d(sxy)[0] + d(syy)[1])
    l_phys = (cont ** 2 + ns_x ** 2 + ns_y ** 2).mean()               # Eq. (5)
    if interface.any():
        grx, gry = d(rho)
        g2 = (grx ** 2 + gry ** 2)[interface]
        l_int = (-w.alpha1 * g2 + w.alpha2 * g2 * g2).mean()          # Eq. (8), as described
    else:
        l_int = torch.zeros((), device=xy.device, dtype=xy.dtype)
    total = l_data + w.lambda_phys * l_phys + w.lambda_interface * l_int   # Eq. (3)
    return total, l_data, l_phys, l_int


def interface_cells(rho: np.ndarray) -> np.ndarray:
    """Eq. (9)'s criterion |grad rho| > 0.01 with the Eq. (16) periodic central
    differences, on a density field (ny, nx)."""
    gx = (np.roll(rho, -1, 1) - np.roll(rho, 1, 1)) / 2.0
    gy = (np.roll(rho, -1, 0) - np.roll(rho, 1, 0)) / 2.0
    return np.sqrt(gx * gx + gy * gy) > 0.01


def train(net, fields, G, tau, epochs=300, lr=3e-4, points=4096, seed=0,
          weights: LossWeights | None = None, device=None, log=None):
    """Trains `net` on the fields (rho, u_x, u_y), each (ny, nx), for `epochs`
    full-batch Adam steps on `points` cells drawn once (half of them interface
    cells where there are enough).  Returns the per-epoch total losses."""
    torch = _torch()
    w = weights or LossWeights()
    rho, ux, uy = (np.asarray(a, dtype=np.float64) for a in fields)
    ny, nx = rho.shape
    dev = device or next(net.parameters()).device
    dtype = next(net.parameters()).dtype
    rng = np.random.default_rng(seed)
    inter = interface_cells(rho).ravel()
    idx_i = np.flatnonzero(inter)
    idx_b = np.flatnonzero(~inter)
    n = min(points, nx * ny)
    ni = min(len(idx_i), n // 2)
    sel = np.concatenate([rng.choice(idx_i, ni, replace=False) if ni else idx_i[:0],
                          rng.choice(idx_b, n - ni, replace=len(idx_b) < n - ni)])
    xy_all = coords(nx, ny, dev, dtype)
    xy = xy_all[torch.as_tensor(sel, device=dev)].clone().requires_grad_(True)
    tgt = torch.as_tensor(np.stack([rho.ravel()[sel], ux.ravel()[sel], uy.ravel()[sel]], 1),
                          device=dev, dtype=dtype)
    isel = torch.as_tensor(inter[sel], device=dev)
    opt = torch.optim.Adam(net.parameters(), lr=lr)
    hist = []
    for e in range(epochs):
        opt.zero_grad()
        total, ld, lp, li = losses(net, xy, tgt, isel, nx, ny, G, tau, w)
        total.backward()
        opt.step()
        hist.append(total.item())
        if log and (e % 50 == 0 or e == epochs - 1):
            log(f"epoch {e}: total {float(total):.4e} data {float(ld):.4e} "
                f"phys {float(lp):.4e} interface {float(li):.4e}")
    return hist


def state_fields(sim):
    """rho and the populations' velocity sum_i f_i e_i / rho of a Simulation's
    current state, as FP64 numpy arrays (ny, nx); summed on the GPU."""
    torch = _torch()
    f = sim.get_state().double()
    ex = torch.tensor([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=torch.float64, device=f.device)
    ey = torch.tensor([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=torch.float64, device=f.device)
    rho = f.sum(0)
    ux = torch.tensordot(ex, f, 1) / rho
    uy = torch.tensordot(ey, f, 1) / rho
    return tuple(t.cpu().numpy() for t in (rho, ux, uy))


def couple(sim, params_net, G, tau, beta=0.5, init_steps=500, segment=100,
           epochs=(300, 240, 180, 120, 60), log=None):
    """The coupling protocol of Sec. II-C / III-C on a Simulation: `init_steps`
    pure LBM steps, then per evolution segment: train on the current fields,
    correct the state at its interfaces on the GPU (lbm_pinn_correct), and
    advance `segment` steps.  Returns the metrics after each segment."""
    sim.step(init_steps)
    out = []
    for k, ep in enumerate(epochs):
        train(params_net, state_fields(sim), G, tau, epochs=ep, seed=k, log=log)
        sim.pinn_correct(pack(params_net).to(sim.device), beta)
        sim.step(segment)
        out.append(sim.metrics())
    return out
