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


def _twice(q) -> np.float16:
    """q rounded to FP32 and then to half (the double rounding the storage
    form does not do)."""
    return np.float16(_round_f32(Fraction(q)))


def _expected_roundtrip(f, to_half=None):
    """get_state(set_state(f)) in the per-cell-shift form, computed exactly on
    the host (to_half: the rounding of A_i - w_i rhohat to half, once from the
    exact value unless another is given for comparison)."""
    to_half = to_half or round_half
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
                h = to_half(-Fraction(float(W[i])) * Fraction(float(q)) + Fraction(float(A[i, y, x])))
                dec[i, y, x] = _fma32(q, W[i], np.float32(h))
    return np.stack([np.roll(dec[i], (EY[i], EX[i]), axis=(0, 1)) for i in range(9)])


def test_storage_roundtrip_is_cell_shifted_half():
    L = lbm()
    f = f32_state(inputs.random_positive_state(20, 12, seed=3)).astype(np.float32)
    sim = L.Simulation(20, 12, -5.0, 1.0, L.LBM_F16_CELL)
    set_state_from(sim, f)
    got = sim.get_state().cpu().numpy()
    assert np.array_equal(got, _expected_roundtrip(f))


def _tie_state(nx, ny, seed):
    """A state in which one stored difference per cell, A_i - w_i rhohat,
    lies within half an FP32 ulp of a midpoint between two halves, on the
    side away from the even one (one rounding and two roundings disagree)."""
    rng = np.random.default_rng(seed)
    A = np.empty((9, ny, nx), np.float32)
    crafted = 0
    for y in range(ny):
        for x in range(nx):
            i = (x + 2 * y) % 9
            w = Fraction(float(W[i]))
            for _ in range(400):
                a = rng.uniform(0.05, 0.3, 9).astype(np.float32)
                for _ in range(3):  # rhohat = half(rho) moves only if A_i crosses a half
                    r = np.float32(a[0])
                    for v in a[1:]:
                        r = np.float32(r + v)
                    q = Fraction(float(np.float16(r)))
                    lo = np.float16(-float(w * q) / 2)
                    hi = np.nextafter(lo, np.float16(1))
                    m = (Fraction(float(lo)) + Fraction(float(hi))) / 2
                    a[i] = np.float32(float(m + w * q))
                r = np.float32(a[0])
                for v in a[1:]:
                    r = np.float32(r + v)
                d = Fraction(float(a[i])) - w * Fraction(float(np.float16(r)))
                if d != m and _round_f32(d) == np.float32(float(m)) and round_half(d) != _twice(d):
                    crafted += 1
                    break
            A[:, y, x] = a
    f = np.stack([np.roll(A[i], (EY[i], EX[i]), axis=(0, 1)) for i in range(9)])
    return f, crafted


def test_cell_shifted_values_are_rounded_once():
    """Stored values are the nearest halves to the exact differences: on a
    state built so that one rounding and two roundings (via FP32) disagree in
    every cell, the round trip equals the single rounding bit for bit and not
    the double one."""
    L = lbm()
    nx, ny = 16, 8
    f, crafted = _tie_state(nx, ny, seed=22)
    assert crafted >= nx * ny * 3 // 4
    sim = L.Simulation(nx, ny, -5.0, 1.0, L.LBM_F16_CELL)
    set_state_from(sim, f)
    got = sim.get_state().cpu().numpy()
    once = _expected_roundtrip(f)
    twice = _expected_roundtrip(f, _twice)
    assert np.array_equal(got.view(np.uint32), once.view(np.uint32))
    assert np.sum(once.view(np.uint32) != twice.view(np.uint32)) >= crafted


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
        if t["steps"] >= 3:  # FP32 only
            continue
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
