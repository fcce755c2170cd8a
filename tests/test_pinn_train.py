"""The PyTorch side of the PINN (paper_2504_10539_amd/pinn.py) on the CPU.

- The packed parameters are in the C-ABI order: the FP64 oracle evaluating the
  packed vector gives the torch network's outputs.
- The interface selection used for training is Eq. (9)'s criterion (the
  oracle's mask, computed independently in C).
- Training on an oracle-produced droplet state lowers the composite loss of
  Eq. (3) and its data term, and the physics residuals of the steady reading
  vanish on a uniform state at rest.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from oracle import pinn as opinn
from paper_2504_10539_amd import pinn


def test_pack_order_matches_the_oracle():
    net = pinn.make_net(seed=3, dtype=torch.float64)
    p = pinn.pack(net).double().numpy()
    assert p.size == opinn.param_count() == pinn.PARAM_COUNT
    xy = pinn.coords(13, 7, dtype=torch.float64)
    with torch.no_grad():
        ref = net(xy).numpy()
    # the packed FP32 vector, evaluated by the oracle, against the torch network
    # with the same FP32-rounded weights
    net32 = pinn.make_net(seed=3)
    with torch.no_grad():
        got_t = net32.double()(xy).numpy()
    got_o = opinn.mlp_forward(pinn.pack(pinn.make_net(seed=3)).double().numpy(), opinn.coordinates(13, 7))
    assert np.allclose(got_o, got_t, rtol=0, atol=1e-12)
    assert np.allclose(ref, got_t, atol=1e-6)
    assert np.allclose(pinn.coords(13, 7, dtype=torch.float64).numpy(), opinn.coordinates(13, 7))


def test_interface_cells_match_the_oracle():
    rho = oracle.init_density(40, 30, [(15.0, 14.0, 8.0)], 2.0, 0.15, 2.0, 1e-3, 2)
    assert np.array_equal(pinn.interface_cells(rho), opinn.interface_mask(rho))


def test_steady_residuals_vanish_at_rest():
    """A network that outputs a uniform state at rest has zero physics residual."""
    net = pinn.make_net(seed=0, dtype=torch.float64)
    with torch.no_grad():
        for m in net:
            if isinstance(m, torch.nn.Linear):
                m.weight.zero_()
                m.bias.zero_()
        net[-1].bias.copy_(torch.tensor([0.8, 0.0, 0.0], dtype=torch.float64))
    xy = pinn.coords(8, 8, dtype=torch.float64).requires_grad_(True)
    tgt = torch.tensor([[0.8, 0.0, 0.0]], dtype=torch.float64).repeat(64, 1)
    total, ld, lp, li = pinn.losses(net, xy, tgt, torch.zeros(64, dtype=torch.bool), 8, 8, -5.0,
                                    1.0, pinn.LossWeights())
    assert ld.item() == 0.0 and lp.item() == 0.0 and li.item() == 0.0


def test_training_lowers_the_loss_on_a_droplet():
    f = oracle.step(oracle.droplet_state(32, 32, [(16.0, 16.0, 8.0)]), -5.0, 1.0, 50)
    rho, ux, uy = oracle.moments(f, -5.0)
    net = pinn.make_net(seed=1)
    hist = pinn.train(net, (rho, ux, uy), -5.0, 1.0, epochs=30, lr=3e-3, points=256)
    assert hist[-1] < 0.5 * hist[0]
