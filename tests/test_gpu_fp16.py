"""FP16-shifted population storage against the FP64 oracle.

Storage form: h_i = half_RNE(f_i - w_i rho0), read back as float(h_i) + w_i rho0
with FP32 arithmetic.  Bar: density within 1e-3 and each interface metric
within 2% after 1000 steps of the 64x64 droplet run.  Both density readings
are computed and printed: max |drho| / max rho (range-normalised) and the
per-cell max |drho| / rho.
"""
import numpy as np
import pytest

import oracle
from paper_2504_10539_amd import inputs
from tests.gpu_helpers import f32_state, lbm, need_gpu, set_state_from, to_np, torch

pytestmark = pytest.mark.gpu

W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4, dtype=np.float32)


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def test_storage_rounding_is_shifted_half():
    rho0 = np.float32(0.5)
    f = f32_state(inputs.random_positive_state(40, 24, seed=3)).astype(np.float32)
    sim = lbm().Simulation(40, 24, -5.0, 1.0, lbm().LBM_F16_SHIFTED, float(rho0))
    set_state_from(sim, f)
    got = sim.get_state().cpu().numpy()
    sh = (W * rho0).astype(np.float32)[:, None, None]
    expect = (f - sh).astype(np.float16).astype(np.float32) + sh
    assert np.array_equal(got, expect)


def test_one_step_error_is_one_fp16_rounding():
    """From an FP16-representable state, one step differs from the FP64 oracle by
    at most the final half-precision rounding of f* - w_i rho0 (plus FP32 noise)."""
    rho0 = np.float32(1.0)
    sh = (W * rho0).astype(np.float32)[:, None, None]
    f = oracle.droplet_state(48, 40, [(20.0, 22.0, 9.0)], seed=4)
    f0 = ((f.astype(np.float32) - sh).astype(np.float16).astype(np.float32) + sh).astype(np.float64)
    sim = lbm().Simulation(48, 40, -5.0, 0.9, lbm().LBM_F16_SHIFTED, float(rho0))
    set_state_from(sim, f0)
    sim.step(1)
    got = to_np(sim.get_state())
    ref = oracle.step(f0, -5.0, 0.9, 1)
    half_ulp = 0.5 * np.spacing(np.abs(ref - sh).astype(np.float16)).astype(np.float64)
    assert np.all(np.abs(got - ref) <= 1.01 * half_ulp + 1e-6 * np.abs(ref).max())


@pytest.mark.parametrize("rho0", [0.5, 1.0])
def test_config1_fp16_shifted_1000_steps(rho0):
    """Metrics meet the 2% bar.  The density does NOT meet 1e-3: half-precision
    rounding of f_i - w_i rho0 biases mass and momentum slightly each step, the
    droplet drifts by ~0.01 cell, and at the interface (slope ~0.5 per cell)
    that reads as ~1e-2 of rho_max.  The bounds below record the measured
    result (1.4e-2 and 7.9e-3 range-normalised for rho0 = 0.5 and 1.0) with
    margin, as a regression guard."""
    N = 64
    drops = inputs.single_droplet(N, 16)
    sim = lbm().Simulation(N, N, -5.0, 1.0, lbm().LBM_F16_SHIFTED, rho0).init_droplets(drops, seed=1)
    sim.step(1000)
    rho = to_np(sim.moments()[0])
    m = sim.metrics()
    ref = oracle.step(oracle.droplet_state(N, N, drops, seed=1), -5.0, 1.0, 1000, 8)
    rho_ref = oracle.density(ref)
    mref = oracle.metrics(rho_ref)
    err_range = float(np.max(np.abs(rho - rho_ref)) / rho_ref.max())
    err_cell = float(np.max(np.abs(rho - rho_ref) / rho_ref))
    rel = {k: abs(m[k] / mref[k] - 1) for k in ("Gmax", "drho", "W_eff", "E_int")}
    print(f"fp16 rho0={rho0}: max|drho|/max rho = {err_range:.2e}, per-cell max|drho|/rho = "
          f"{err_cell:.2e}, metric errors {rel}, W {m['W']} vs {mref['W']}")
    for k, v in rel.items():
        assert v <= 0.02, k
    assert abs(m["W"] - mref["W"]) <= 0.02 * mref["W"]
    assert err_range <= 3e-2 and err_cell <= 8e-2


@pytest.mark.xfail(strict=True, reason="one global shift cannot fit both phases: in the gas "
                   "(rho ~ 0.15) the stored f_i - w_i rho0 is of order w_i and its half-precision "
                   "rounding is ~1e-3 of the local density every step; measured 1.35e-2 (rho0 = 1) "
                   "and 1.6e-2 (rho0 = 0.5) of rho_max, 3.3e-2 and 3.9e-2 per cell")
@pytest.mark.parametrize("rho0", [0.5, 1.0])
def test_config1_fp16_shifted_density_bar(rho0):
    """The stated FP16 bar: density within 1e-3 in both readings after 1000 steps."""
    N = 64
    drops = inputs.single_droplet(N, 16)
    sim = lbm().Simulation(N, N, -5.0, 1.0, lbm().LBM_F16_SHIFTED, rho0).init_droplets(drops, seed=1)
    sim.step(1000)
    rho = to_np(sim.moments()[0])
    rho_ref = oracle.density(oracle.step(oracle.droplet_state(N, N, drops, seed=1), -5.0, 1.0,
                                         1000, 8))
    assert float(np.max(np.abs(rho - rho_ref)) / rho_ref.max()) <= 1e-3
    assert float(np.max(np.abs(rho - rho_ref) / rho_ref)) <= 1e-3


def test_fp16_mixed_with_fp32_in_one_batch_is_bitwise():
    """An FP16 run and an FP32 run in the same batch equal their solo runs."""
    L = lbm()
    a = L.Simulation(96, 64, -5.0, 1.0, L.LBM_F16_SHIFTED, 0.5).init_droplets([(40, 30, 14)], seed=2)
    b = L.Simulation(80, 80, -5.5, 0.9, L.LBM_F32).init_droplets([(40, 40, 15)], seed=3)
    sa = L.Simulation(96, 64, -5.0, 1.0, L.LBM_F16_SHIFTED, 0.5).init_droplets([(40, 30, 14)], seed=2)
    sb = L.Simulation(80, 80, -5.5, 0.9, L.LBM_F32).init_droplets([(40, 40, 15)], seed=3)
    bt = L.Batch([a, b], steps_per_graph=16)
    bt.step(70)
    sa.step(70)
    sb.step(70)
    assert np.array_equal(to_np(a.get_state()), to_np(sa.get_state()))
    assert np.array_equal(to_np(b.get_state()), to_np(sb.get_state()))
    bt.close()
