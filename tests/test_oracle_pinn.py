"""Pins of the PINN oracle (oracle/pinn.py) against what the paper and the
mathematics fix, on the CPU.

- The network is the one of Sec. III-B (2 -> 64 -> 128 -> 128 -> 64 -> 3).
- Its forward pass equals a literal per-neuron loop with math.tanh (brute
  force), and closed-form networks (biases only; one path through single
  neurons).
- The equilibrium field equals the C oracle's per-cell equilibrium.
- The correction keeps every non-interface cell, gives each corrected cell
  exactly the blended mass and momentum (closed form), keeps the populations'
  non-equilibrium part, and reduces to the identity for beta = 0 and for a
  network that reproduces the state.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import pinn
from paper_2504_10539_amd import inputs

E_LITERAL = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]


def random_params(seed, scale=0.4):
    rng = np.random.default_rng(seed)
    return rng.uniform(-scale, scale, pinn.param_count())


def test_layer_widths_are_the_papers():
    assert pinn.LAYERS == (2, 64, 128, 128, 64, 3)
    assert pinn.param_count() == 2 * 64 + 64 + 64 * 128 + 128 + 128 * 128 + 128 + 128 * 64 + 64 + 64 * 3 + 3
    shapes = [W.shape for W, _ in pinn.unpack(np.zeros(pinn.param_count()))]
    assert shapes == [(64, 2), (128, 64), (128, 128), (64, 128), (3, 64)]


def test_forward_equals_per_neuron_loop():
    """Brute force: every neuron as a Python sum and math.tanh, on a few points."""
    p = random_params(1)
    layers = pinn.unpack(p)
    pts = np.array([[-0.9, 0.3], [0.0, 0.0], [0.71, -0.55], [0.999, 0.999]])
    got = pinn.mlp_forward(p, pts)
    for n, (x, y) in enumerate(pts):
        h = [x, y]
        for k, (W, b) in enumerate(layers):
            z = [sum(W[o][i] * h[i] for i in range(len(h))) + b[o] for o in range(len(b))]
            h = [math.tanh(v) for v in z] if k < 4 else z
        assert np.allclose(got[n], h, rtol=0, atol=1e-13), (n, got[n], h)


def test_forward_of_a_biases_only_network():
    """All weights zero: every hidden layer outputs tanh(b_l), the output is b_5."""
    p = np.zeros(pinn.param_count())
    layers = pinn.unpack(p)
    layers[4][1][:] = [0.25, -0.5, 0.125]
    out = pinn.mlp_forward(p, pinn.coordinates(5, 3))
    assert np.array_equal(out, np.tile([0.25, -0.5, 0.125], (15, 1)))


def test_forward_through_single_neurons_closed_form():
    """One path of single neurons: N_0 = c tanh(a4 tanh(a3 tanh(a2 tanh(a1 x)))) + d."""
    p = np.zeros(pinn.param_count())
    (W1, b1), (W2, b2), (W3, b3), (W4, b4), (W5, b5) = pinn.unpack(p)
    a1, a2, a3, a4, c, d = 1.3, -0.7, 2.1, 0.9, 1.7, 0.05
    W1[5, 0] = a1
    W2[17, 5] = a2
    W3[100, 17] = a3
    W4[40, 100] = a4
    W5[0, 40] = c
    b5[0] = d
    xy = pinn.coordinates(7, 4)
    out = pinn.mlp_forward(p, xy)
    x = xy[:, 0]
    expect = c * np.tanh(a4 * np.tanh(a3 * np.tanh(a2 * np.tanh(a1 * x)))) + d
    assert np.allclose(out[:, 0], expect, rtol=0, atol=1e-15)
    assert np.all(out[:, 1:] == 0.0)


def test_coordinates_are_cell_centres_in_the_unit_square():
    xy = pinn.coordinates(4, 2)
    assert np.allclose(xy[:4, 0], [-0.75, -0.25, 0.25, 0.75])
    assert np.allclose(xy[::4, 1], [-0.5, 0.5])


def test_equilibrium_field_equals_the_c_oracle():
    rng = np.random.default_rng(3)
    rho = rng.uniform(0.1, 2.5, (5, 6))
    ux, uy = rng.uniform(-0.1, 0.1, (2, 5, 6))
    got = pinn.equilibrium_field(rho, ux, uy)
    for y in range(5):
        for x in range(6):
            assert np.allclose(got[:, y, x], oracle.equilibrium(rho[y, x], ux[y, x], uy[y, x]),
                               rtol=1e-15, atol=0)


def droplet_state():
    rho = oracle.init_density(48, 40, [(22.0, 19.0, 10.0)], 2.0, 0.15, 2.0, 1e-3, 5)
    f = oracle.init_populations(rho)
    return oracle.step(f, -5.0, 1.0, 30)


def test_correction_keeps_other_cells_and_sets_the_blended_moments():
    f = droplet_state()
    p = random_params(7)
    beta = 0.4
    g, mask = pinn.correct(f, p, beta)
    rho = f.sum(0)
    assert mask.any() and not mask.all()
    assert np.array_equal(mask, oracle.grad_mag(rho) > 0.01)
    assert np.array_equal(g[:, ~mask], f[:, ~mask])
    ex = np.array([e[0] for e in E_LITERAL], float)
    ey = np.array([e[1] for e in E_LITERAL], float)
    jx = (f * ex[:, None, None]).sum(0)
    jy = (f * ey[:, None, None]).sum(0)
    rn, uxn, uyn = pinn.predict_fields(p, 48, 40)
    r2 = rho + beta * (rn - rho)
    ux2 = jx / rho + beta * (uxn - jx / rho)
    uy2 = jy / rho + beta * (uyn - jy / rho)
    m = mask
    assert np.allclose(g.sum(0)[m], r2[m], rtol=1e-13, atol=0)
    assert np.allclose((g * ex[:, None, None]).sum(0)[m], (r2 * ux2)[m], rtol=0, atol=1e-13)
    assert np.allclose((g * ey[:, None, None]).sum(0)[m], (r2 * uy2)[m], rtol=0, atol=1e-13)
    # the non-equilibrium part is kept
    neq_before = f - pinn.equilibrium_field(rho, jx / rho, jy / rho)
    neq_after = g - pinn.equilibrium_field(r2, ux2, uy2)
    assert np.allclose(neq_after[:, m], neq_before[:, m], rtol=0, atol=1e-13)


def test_correction_identities():
    f = droplet_state()
    p = random_params(8)
    g, _ = pinn.correct(f, p, 0.0)
    assert np.allclose(g, f, rtol=0, atol=1e-15)
    # a network whose prediction is the state itself changes nothing
    rho, ux, uy = pinn.velocity(f)
    saved = pinn.predict_fields
    try:
        pinn.predict_fields = lambda params, nx, ny: (rho, ux, uy)
        g, _ = pinn.correct(f, p, 0.7)
    finally:
        pinn.predict_fields = saved
    assert np.allclose(g, f, rtol=0, atol=1e-14)
    # beta = 1 with an explicit full mask: every cell takes the network's fields
    mask = np.ones(rho.shape, bool)
    g, _ = pinn.correct(f, p, 1.0, mask)
    rn, uxn, uyn = pinn.predict_fields(p, 48, 40)
    r2, ux2, uy2 = pinn.velocity(g)
    assert np.allclose(r2, rn, rtol=1e-13, atol=0)
    assert np.allclose(ux2, uxn, rtol=0, atol=1e-12) and np.allclose(uy2, uyn, rtol=0, atol=1e-12)


def test_planted_sign_error_in_the_correction_is_caught():
    """A correction that subtracted the new equilibrium instead of adding it would
    not give the blended mass: the closed form above distinguishes the two."""
    f = droplet_state()
    p = random_params(9)
    g, mask = pinn.correct(f, p, 0.5)
    rho, ux, uy = pinn.velocity(f)
    rn, uxn, uyn = pinn.predict_fields(p, 48, 40)
    r2 = rho + 0.5 * (rn - rho)
    wrong = f - (pinn.equilibrium_field(r2, ux, uy) - pinn.equilibrium_field(rho, ux, uy))
    assert not np.allclose(wrong.sum(0)[mask], r2[mask], rtol=1e-6)
    assert np.allclose(g.sum(0)[mask], r2[mask], rtol=1e-13)
