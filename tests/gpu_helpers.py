"""Shared helpers for the GPU parity tests (inputs and comparisons only)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def lbm():
    from paper_2504_10539_amd import lbm as _lbm
    return _lbm


def to_np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def f32_state(f64: np.ndarray) -> np.ndarray:
    """FP64 populations rounded to FP32 and widened back: a state both sides hold exactly."""
    return f64.astype(np.float32).astype(np.float64)


def set_state_from(sim, f: np.ndarray):
    sim.set_state(torch.from_numpy(np.ascontiguousarray(f, dtype=np.float32)).cuda())


def rel_density_error(rho_gpu: np.ndarray, rho_ref: np.ndarray) -> float:
    return float(np.max(np.abs(rho_gpu - rho_ref) / np.abs(rho_ref)))


def round_half(q) -> np.float16:
    """Nearest half-precision value to the exact rational q, ties to even (the
    per-cell and moment storage forms round each stored deviation once, from
    the exact difference)."""
    from fractions import Fraction
    q = Fraction(q)
    c = np.float16(float(q))
    best = None
    for v in (np.nextafter(c, np.float16(-np.inf)), c, np.nextafter(c, np.float16(np.inf))):
        d = abs(Fraction(float(v)) - q)
        if best is None or d < best[0] or (d == best[0] and (v.view(np.uint16) & 1) == 0):
            best = (d, v)
    return best[1]
