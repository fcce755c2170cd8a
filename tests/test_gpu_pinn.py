"""The PINN surrogate and the interface correction on the GPU against the FP64
oracle (oracle/pinn.py).

The kernel evaluates the network with the weights of layers 2-4 rounded to
FP16 and the hidden activations rounded to FP16 between layers (matrix cores,
FP32 accumulation), with tanh from the hardware exponential and reciprocal
(absolute error below 4e-7).  The oracle is handed the same FP16-rounded
weights, so the remaining difference is the activation rounding and the tanh
error plus FP32 arithmetic.  An activation error vector at layer l has 2-norm
at most u sqrt(n_l) (|tanh| <= 1), tanh is 1-Lipschitz and a layer multiplies
an error by at most the spectral norm of its weights, so every output differs
from the oracle by at most
    B = ||W5|| (u sqrt(64) + ||W4|| (u sqrt(128) + ||W3|| (u sqrt(128) + ||W2|| u sqrt(64)))),
u = 2^-11 + 4e-7, plus FP32 rounding (1e-5 covers it for these networks).  The
corrected populations move by at most 13 beta B (derivative of the
equilibrium with respect to rho and u for rho <= 3, |u| <= 0.3), plus FP32.
The interface mask is decided in FP64 from the same density on both sides
and must agree exactly; every other cell must be left bitwise as it was.
"""
import numpy as np
import pytest

import oracle
from oracle import pinn
from paper_2504_10539_amd import inputs
from tests.gpu_helpers import f32_state, lbm, need_gpu, set_state_from, to_np, torch

pytestmark = pytest.mark.gpu
U16 = 2.0 ** -11
TANH = 4e-7  # absolute error of the kernel's tanh


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def network(seed, gain=1.0):
    """A network with PyTorch's default initialisation of linear layers
    (uniform in +-1/sqrt(fan_in)), FP32; layers 2-4 rounded to FP16 as the
    kernel evaluates them.  Returns (FP32 parameters for the GPU, the FP64
    parameters of the network the GPU evaluates)."""
    rng = np.random.default_rng(seed)
    parts = []
    for i, o in zip(pinn.LAYERS[:-1], pinn.LAYERS[1:]):
        k = gain / np.sqrt(i)
        parts += [rng.uniform(-k, k, (o, i)).ravel(), rng.uniform(-k, k, o)]
    p32 = np.concatenate(parts).astype(np.float32)
    q = p32.astype(np.float64)
    for l, (W, _) in enumerate(pinn.unpack(q)):
        if l in (1, 2, 3):
            W[...] = W.astype(np.float16).astype(np.float64)  # views into q
    return p32, q


def bound(q):
    n = [np.linalg.norm(W, 2) for W, _ in pinn.unpack(q)]
    u = U16 + TANH
    return n[4] * (u * 8 + n[3] * (u * np.sqrt(128) + n[2] * (u * np.sqrt(128) + n[1] * u * 8))) + 1e-5


@pytest.mark.parametrize("nx,ny,seed", [(64, 64, 1), (100, 37, 2), (257, 3, 3), (31, 90, 4)])
def test_inference_matches_oracle(nx, ny, seed):
    L = lbm()
    p32, q = network(seed)
    params = torch.from_numpy(p32).cuda()
    sim = L.Simulation(nx, ny, -5.0, 1.0)
    got = np.stack([to_np(t) for t in sim.pinn_infer(params)])
    ref = np.stack(pinn.predict_fields(q, nx, ny))
    err = np.abs(got - ref).max()
    tol = bound(q)
    print(f"{nx}x{ny}: max |N_gpu - N_oracle| = {err:.2e}, bound {tol:.2e}")
    assert err <= tol
    # the outputs are not trivially small (the test network is not degenerate)
    assert np.abs(ref).max() > 0.05


def test_inference_single_neuron_path_is_exact_to_fp16():
    """A network with a single active path: an error in a fragment layout would
    route the wrong weight and show up far beyond the rounding bound."""
    L = lbm()
    p = np.zeros(pinn.param_count())
    (W1, b1), (W2, b2), (W3, b3), (W4, b4), (W5, b5) = pinn.unpack(p)
    W1[5, 0], W1[9, 1] = 1.3, -0.8
    W2[17, 5], W2[100, 9] = -0.75, 0.5
    W3[100, 17], W3[3, 100] = 2.0, 1.25
    W4[40, 100], W4[63, 3] = 0.875, -1.5
    W5[0, 40], W5[2, 63], b5[1] = 1.75, 0.625, 0.1
    nx, ny = 96, 70
    params = torch.from_numpy(p.astype(np.float32)).cuda()
    got = np.stack([to_np(t) for t in L.Simulation(nx, ny, -5.0, 1.0).pinn_infer(params)])
    ref = np.stack(pinn.predict_fields(p, nx, ny))
    assert np.abs(got - ref).max() <= 2e-3  # four FP16 roundings along one path
    assert np.all(got[1] == float(np.float32(0.1)))  # b_5 alone, in FP32


def droplet_sim(L, storage, nx=150, ny=97, steps=60):
    sim = L.Simulation(nx, ny, -5.0, 1.0, storage, 1.0 if storage == L.LBM_F16_SHIFTED else 0.0)
    sim.init_droplets([(70.0, 45.0, 22.0), (130.0, 80.0, 10.0)], seed=3)
    sim.step(steps)
    return sim


@pytest.mark.parametrize("beta", [0.3, 1.0])
def test_correction_matches_oracle_fp32(beta):
    L = lbm()
    p32, q = network(11)
    params = torch.from_numpy(p32).cuda()
    sim = droplet_sim(L, L.LBM_F32)
    nx, ny = sim.nx, sim.ny
    f0 = to_np(sim.get_state())
    mask_t = torch.zeros(nx * ny, dtype=torch.uint8, device="cuda")
    sim.pinn_correct(params, beta, mask_t)
    f1 = to_np(sim.get_state())
    mask = mask_t.cpu().numpy().reshape(ny, nx).astype(bool)
    ref, ref_mask = pinn.correct(f0, q, beta)
    assert np.array_equal(mask, ref_mask)
    assert 0 < mask.sum() < mask.size
    # untouched cells bitwise; corrected cells within the derived bound
    assert np.array_equal(f1[:, ~mask], f0[:, ~mask])
    tol = 13 * beta * bound(q) + 1e-5
    err = np.abs(f1[:, mask] - ref[:, mask]).max()
    print(f"beta {beta}: {mask.sum()} cells corrected, max |f_gpu - f_oracle| = {err:.2e} (bound {tol:.2e})")
    assert err <= tol
    # the correction moved the state by much more than the GPU's difference
    moved = np.abs(ref[:, mask] - f0[:, mask]).max()
    assert moved > 0.05 and moved > 1e3 * err


@pytest.mark.parametrize("storage", [1, 2])
def test_correction_in_fp16_storage(storage):
    """FP16 storage forms: the corrected values are the FP32 run's, rounded as
    the storage form rounds a stored value."""
    L = lbm()
    p32, _ = network(12)
    params = torch.from_numpy(p32).cuda()
    a = droplet_sim(L, storage)
    f0 = to_np(a.get_state())
    b = L.Simulation(a.nx, a.ny, -5.0, 1.0, L.LBM_F32)
    set_state_from(b, f0)  # the same state in FP32 storage
    a.pinn_correct(params, 0.5)
    b.pinn_correct(params, 0.5)
    fa, fb = to_np(a.get_state()), to_np(b.get_state())
    changed = np.any(fb != f0, axis=0)
    assert changed.any()
    assert np.array_equal(fa[:, ~changed], f0[:, ~changed])
    # one half-precision rounding of a value of size <= 1 around its shift
    assert np.abs(fa - fb).max() <= 2 * U16 * 1.0 + 1e-6


def test_correction_refuses_moment_storage_and_bad_beta():
    L = lbm()
    p32, _ = network(13)
    params = torch.from_numpy(p32).cuda()
    sim = L.Simulation(64, 64, -5.0, 1.0, L.LBM_F16_MOMENT).init_droplets(inputs.single_droplet(64, 16))
    with pytest.raises(L.LbmError) as e:
        sim.pinn_correct(params, 0.5)
    assert e.value.code == L.LBM_EINVAL
    s2 = L.Simulation(64, 64, -5.0, 1.0).init_droplets(inputs.single_droplet(64, 16))
    for beta in (-0.1, 1.5, float("nan")):
        with pytest.raises(L.LbmError):
            s2.pinn_correct(params, beta)


def test_correction_then_steps_stay_finite_and_conserve_beta_zero():
    """beta = 0 leaves the state bitwise unchanged; a corrected run keeps stepping."""
    L = lbm()
    p32, _ = network(14)
    params = torch.from_numpy(p32).cuda()
    sim = droplet_sim(L, L.LBM_F32)
    f0 = to_np(sim.get_state())
    sim.pinn_correct(params, 0.0)
    assert np.array_equal(to_np(sim.get_state()), f0)
    sim.pinn_correct(params, 0.2)
    sim.step(100)
    assert sim.metrics()["finite"] == 1


def test_coupling_protocol_runs_on_the_gpu_correction():
    """The Sec. II-C / III-C loop: pure LBM steps, then segments of training
    (PyTorch) and GPU correction; the corrected run stays finite, takes the same
    number of steps and departs from the pure LBM run of the same droplet.  (The
    correction moves interface cells toward the network's density by design, so
    with a briefly trained network their mass changes.)"""
    from paper_2504_10539_amd import pinn as tpinn
    L = lbm()
    N, G, tau = 64, -5.5, 1.0
    a = L.Simulation(N, N, G, tau).init_droplets(inputs.single_droplet(N, N / 6), seed=1)
    b = L.Simulation(N, N, G, tau).init_droplets(inputs.single_droplet(N, N / 6), seed=1)
    net = tpinn.make_net(seed=2, device="cuda")
    rec = tpinn.couple(a, net, G, tau, beta=0.5, init_steps=100, segment=40, epochs=(60, 30))
    assert len(rec) == 2 and all(m["finite"] == 1 for m in rec)
    b.step(100 + 2 * 40)
    assert a.steps == b.steps == 180
    fa, fb = to_np(a.get_state()), to_np(b.get_state())
    assert not np.array_equal(fa, fb)
    assert rec[-1]["drho"] > 0.0
