"""The many-droplet error run: the [0, 512)^2 window of the 4096^2 2000-droplet
field (radii uniform in [8, 48], seed 3), treated as its own periodic domain,
G = -5.5, tau = 1.0, 5000 steps.  GPU FP32 and FP16-shifted storage against the
FP64 oracle, errors logged every 500 steps.

Measured (MI355X): FP32 per-cell max |drho|/rho grows to 7.5e-5 by step 5000
(2.6e-5 of rho_max) and every metric stays within 3e-5.  A numpy FP32
emulation of the kernel's arithmetic gives errors of the same size (7.0e-6
against the GPU's 8.1e-6 at step 500), so this is the FP32 arithmetic, not a
kernel defect; an FP32-ulp perturbation of the FP64 run grows only to 1.8e-6,
i.e. the field itself does not amplify rounding noise.
FP16-shifted storage keeps every metric within 0.9%, while the droplets
drift apart from the FP64 run (per-cell density errors of order one by step
2000); the density bar does not hold for this workload.  The exact-moment FP16
form (LBM_F16_MOMENT) stays within 1.5e-4 on every metric and ends at 1.07e-3
of rho_max (3.0e-3 per cell), ten times closer than the per-cell shift.
"""
import numpy as np
import pytest

import oracle
from paper_2504_10539_amd import inputs
from tests.gpu_helpers import lbm, need_gpu, to_np

pytestmark = pytest.mark.gpu

KEYS = ("W", "Gmax", "drho", "W_eff", "E_int")


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


@pytest.fixture(scope="module")
def window_series(nthreads):
    """Worst errors over the series (every 500 steps) of each storage form."""
    L = lbm()
    n, G, tau = 512, -5.5, 1.0
    drops = inputs.many_droplets(4096, 2000, 8, 48, seed=3)
    f = oracle.droplet_state(n, n, drops, seed=3, period=(4096, 4096))
    sims = {"f32": L.Simulation(n, n, G, tau, L.LBM_F32),
            "f16": L.Simulation(n, n, G, tau, L.LBM_F16_SHIFTED, 1.0),
            "f16c": L.Simulation(n, n, G, tau, L.LBM_F16_CELL),
            "f16m": L.Simulation(n, n, G, tau, L.LBM_F16_MOMENT)}
    for s in sims.values():
        s.init_droplets(drops, seed=3, period=(4096, 4096))
    worst = {"f32_cell": 0.0, "f32_range": 0.0, "f32_metric": 0.0, "f16_metric": 0.0,
             "f16_cell": 0.0, "f16_range": 0.0, "f16c_metric": 0.0, "f16c_range": 0.0,
             "f16c_cell": 0.0, "f16m_metric": 0.0, "f16m_range": 0.0, "f16m_cell": 0.0}
    for seg in range(1, 11):
        f = oracle.step(f, G, tau, 500, nthreads)
        rr = oracle.density(f)
        mr = oracle.metrics(rr)
        line = [f"step {500 * seg}"]
        for name, s in sims.items():
            s.step(500)
            rho = to_np(s.moments()[0])
            m = s.metrics()
            assert m["finite"] == 1, (name, seg)
            cell = float(np.max(np.abs(rho - rr) / rr))
            rng = float(np.max(np.abs(rho - rr)) / rr.max())
            met = max(abs(m[k] / mr[k] - 1) for k in KEYS)
            line.append(f"{name}: cell {cell:.2e} range {rng:.2e} metrics {met:.2e}")
            if name == "f32":
                worst["f32_cell"] = max(worst["f32_cell"], cell)
                worst["f32_range"] = max(worst["f32_range"], rng)
                worst["f32_metric"] = max(worst["f32_metric"], met)
            elif name == "f16":
                worst["f16_metric"] = max(worst["f16_metric"], met)
                worst["f16_cell"] = max(worst["f16_cell"], cell)
                worst["f16_range"] = max(worst["f16_range"], rng)
            else:
                worst[f"{name}_metric"] = max(worst[f"{name}_metric"], met)
                worst[f"{name}_range"] = max(worst[f"{name}_range"], rng)
                worst[f"{name}_cell"] = max(worst[f"{name}_cell"], cell)
        print(" | ".join(line))
    print("worst", worst)
    return worst


def test_many_droplet_window_error_series(window_series):
    """Regression bounds over the measured series, with margin."""
    worst = window_series
    assert worst["f32_cell"] < 2e-4 and worst["f32_range"] < 6e-5, worst
    assert worst["f32_metric"] < 1e-4, worst
    assert worst["f16_metric"] < 0.02, worst
    assert worst["f16c_metric"] < 0.02, worst
    assert worst["f16c_range"] < 2e-2, worst  # measured 1.3e-2 at step 5000
    assert worst["f16m_metric"] < 0.02, worst


@pytest.mark.xfail(strict=True, reason="the FP16 density bar (1e-3) is not met on this chaotic "
                   "2000-droplet window: FP16-shifted storage lets the droplets drift apart from "
                   "the FP64 run (order-one per-cell errors from step 2000), the per-cell shift "
                   "reaches 8.8e-3 of rho_max, and even the exact-moment form, whose rounding "
                   "never touches mass or momentum, keeps 6.5e-4 of rho_max but reaches "
                   "2.0e-3 per cell: coalescing droplets amplify its half-precision noise "
                   "(FP32 itself reaches 9.4e-5 per cell here)")
@pytest.mark.parametrize("form", ["f16", "f16c", "f16m"])
def test_many_droplet_window_fp16_density_bar(window_series, form):
    assert window_series[f"{form}_range"] <= 1e-3
    assert window_series[f"{form}_cell"] <= 1e-3
