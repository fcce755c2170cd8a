"""FP16 storage shifted per cell (LBM_F16_CELL) against the FP64 oracle.

Storage form: the nine values a cell x stores, A_i(x), are kept as
h_i = half_RNE(A_i - w_i rhohat), rounded once from the exact value, with
rhohat = half(sum_i A_i) of that
cell stored in a tenth FP16 plane, and read back as fma(rhohat, w_i, h_i) in
FP32.  Only the non-equilibrium and velocity parts of the populations round
to half precision, so the density bar of the FP16 form (1e-3) is within
reach, which the single global shift (LBM_F16_SHIFTED) cannot reach.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2504_10539_amd import inputs
from tests.gpu_helpers import f32_state, lbm, need_gpu, round_half, set_state_from, to_np

pytestmark = pytest.mark.gpu

EX = [0, 1, 0, -1, 0, 1, -1, -1, 1]
EY = [0, 0, 1, 0, -1, 1, 1, -1, -1]
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4, dtype=np.float32)


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def _round_f32(q: Fraction) -> np.float32:
    """Nearest FP32 to the exact value q, ties to even."""
    c = np.float32(float(q))
    best = None
    for v in (np.nextafter(c, np.float32(-np.inf)), c, np.nextafter(c, np.float32(np.inf))):
        d = abs(Fraction(float(v)) - q)
        if best is None or d < best[0] or (d == best[0] and (v.view(np.uint32) & 1) == 0):
            best = (d, v)
    return best[1]


def _fma32(a, b, c) -> np.float32:
    return _round_f32(Fraction(float(a)) * Fraction(float(b)) + Fraction(float(c)))


def _expected_roundtrip(f):
    """get_state(set_state(f)) in the per-cell-shift form, computed exactly on the host."""
    A = np.stack([np.roll(f[i], (-EY[i], -EX[i]), axis=(0, 1)) for i in range(9)])  # A_i(x) = f_i(x + e_i)
    r = A[0].copy()
    for i in range(1, 9):
        r = (r + A[i]).astype(np.float32)
    rh = r.astype(np.float16)
    dec = np.empty_like(A)
    for i in range(9):
        for y in range(A.shape[1]):
            for x in range(A.shape[2]):
                q = np.float32(rh[y, x])
                h = round_half(-Fraction(float(W[i])) * Fraction(float(q)) + Fraction(float(A[i, y, x])))
                dec[i, y, x] = _fma32(q, W[i], np.float32(h))
    return np.stack([np.roll(dec[i], (EY[i], EX[i]), axis=(0, 1)) for i in range(9)])


def test_storage_roundtrip_is_cell_shifted_half():
    L = lbm()
    f = f32_state(inputs.random_positive_state(20, 12, seed=3)).astype(np.float32)
    sim = L.Simulation(20, 12, -5.0, 1.0, L.LBM_F16_CELL)
    set_state_from(sim, f)
    got = sim.get_state().cpu().numpy()
    assert np.array_equal(got, _expected_roundtrip(f))


def test_config1_fp16_cell_1000_steps():
    """Config 1: density within 1e-3 of rho_max (the FP16 bar) and every metric
    within 0.1%; the per-cell reading is reported."""
    L = lbm()
    N = 64
    drops = inputs.single_droplet(N, 16)
    sim = L.Simulation(N, N, -5.0, 1.0, L.LBM_F16_CELL).init_droplets(drops, seed=1)
    sim.step(1000)
    rho = to_np(sim.moments()[0])
    m = sim.metrics()
    ref = oracle.step(oracle.droplet_state(N, N, drops, seed=1), -5.0, 1.0, 1000, 8)
    rho_ref = oracle.density(ref)
    mref = oracle.metrics(rho_ref)
    err_range = float(np.max(np.abs(rho - rho_ref)) / rho_ref.max())
    err_cell = float(np.max(np.abs(rho - rho_ref) / rho_ref))
    rel = {k: abs(m[k] / mref[k] - 1) for k in ("Gmax", "drho", "W_eff", "E_int")}
    print(f"fp16 cell-shifted: max|drho|/max rho = {err_range:.2e}, per-cell max|drho|/rho = "
          f"{err_cell:.2e}, metric errors {rel}, mass drift "
          f"{m['mass'] / oracle.conservation(ref)[0] - 1:.2e}")
    assert err_range <= 1e-3
    assert err_cell <= 3e-3  # regression bound on the per-cell reading
    for k, v in rel.items():
        assert v <= 1e-3, k
    assert m["W"] == mref["W"]


@pytest.mark.xfail(strict=True, reason="the per-cell reading of the FP16 bar is missed: "
                   "1.9e-3 per cell (7.7e-4 of rho_max); the half-precision rounding of the "
                   "moving populations leaves mass and momentum errors that move the droplet")
def test_config1_fp16_cell_per_cell_density_bar():
    L = lbm()
    N = 64
    drops = inputs.single_droplet(N, 16)
    sim = L.Simulation(N, N, -5.0, 1.0, L.LBM_F16_CELL).init_droplets(drops, seed=1)
    sim.step(1000)
    rho = to_np(sim.moments()[0])
    rho_ref = oracle.density(oracle.step(oracle.droplet_state(N, N, drops, seed=1), -5.0, 1.0,
                                         1000, 8))
    assert float(np.max(np.abs(rho - rho_ref) / rho_ref)) <= 1e-3


def test_fp16_cell_tile_shapes_bitwise_identical():
    """Every tile shape, strip and paired, computes bitwise the same state."""
    L = lbm()
    nx, ny = 300, 77
    f0 = f32_state(oracle.droplet_state(nx, ny, [(150.0, 38.0, 20.0), (20.0, 70.0, 9.0)], seed=6))
    ref = None
    for t in L.tiles():
        sim = L.Simulation(nx, ny, -5.5, 0.8, L.LBM_F16_CELL)
        sim.set_tile(t["id"])
        set_state_from(sim, f0)
        sim.step(5)
        got = to_np(sim.get_state())
        if ref is None:
            ref = got
        assert np.array_equal(got, ref), t


def test_fp16_cell_in_a_mixed_batch_is_bitwise():
    L = lbm()
    mk = [lambda: L.Simulation(96, 64, -5.0, 1.0, L.LBM_F16_CELL).init_droplets([(40, 30, 14)], seed=2),
          lambda: L.Simulation(80, 80, -5.5, 0.9, L.LBM_F32).init_droplets([(40, 40, 15)], seed=3),
          lambda: L.Simulation(130, 50, -5.0, 1.0, L.LBM_F16_SHIFTED, 1.0).init_droplets([(60, 25, 12)], seed=4)]
    batch = [m() for m in mk]
    solo = [m() for m in mk]
    bt = L.Batch(batch, steps_per_graph=16)
    bt.step(53)
    for s in solo:
        s.step(53)
    for a, s in zip(batch, solo):
        assert np.array_equal(to_np(a.get_state()), to_np(s.get_state()))
    bt.close()
