"""Metric time series fused into the step (lbm_step_series).

Every record must be what lbm_interface_metrics reports for the same state:
the per-cell FP64 arithmetic is the same, so the count above the threshold,
G_max and the density extrema are equal, and the sums agree up to FP64
summation order.  The steps taken are bitwise those of lbm_step_n.
"""
import numpy as np
import pytest

from paper_2504_10539_amd import inputs
from tests.gpu_helpers import lbm, need_gpu, to_np

pytestmark = pytest.mark.gpu

EXACT = ("n_above", "Gmax", "rho_max", "rho_min", "finite", "step")
CLOSE = ("mass", "sum_grad", "E_int", "W", "W_eff", "drho")


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def _pair(nx, ny, G, tau, storage, drops, seed):
    L = lbm()
    rho0 = 1.0 if storage == L.LBM_F16_SHIFTED else 0.0
    return [L.Simulation(nx, ny, G, tau, storage, rho0).init_droplets(drops, seed=seed)
            for _ in range(2)]


@pytest.mark.parametrize("nx,ny,G,tau,storage,n,every", [
    (64, 64, -5.0, 1.0, 0, 100, 10),
    (300, 77, -5.2, 0.9, 0, 37, 5),
    (96, 40, -5.5, 1.0, 1, 30, 3),
    (130, 40, -5.5, 1.0, 2, 30, 4),
    (64, 64, -5.0, 1.0, 0, 600, 2),   # more records than the device keeps between copies
])
def test_series_matches_separate_metrics(nx, ny, G, tau, storage, n, every):
    drops = [(nx / 2, ny / 2, min(nx, ny) / 4)]
    a, b = _pair(nx, ny, G, tau, storage, drops, seed=5)
    a.step(3)
    b.step(3)
    series = a.step_series(n, every)
    assert len(series) == -(-n // every)
    done = 0
    for rec in series:
        assert rec["step"] == 3 + done
        ref = b.metrics()
        for k in EXACT:
            assert rec[k] == ref[k], (k, rec[k], ref[k])
        for k in CLOSE:
            assert rec[k] == pytest.approx(ref[k], rel=1e-12, abs=1e-300), k
        for k in ("mom_x", "mom_y"):
            assert abs(rec[k] - ref[k]) <= 1e-12 * ref["mass"], k
        s = min(every, n - done)
        b.step(s)
        done += s
    assert a.steps == b.steps == 3 + n
    assert np.array_equal(to_np(a.get_state()).view(np.uint32), to_np(b.get_state()).view(np.uint32))


def test_series_validation():
    L = lbm()
    a = L.Simulation(32, 32, -5.0, 1.0).init_droplets([(16, 16, 6)], seed=1)
    with pytest.raises(L.LbmError):
        a.step_series(10, 0)
    out = (L.lbm_metrics * 2)()
    cnt = L._i32()
    assert L.LIB.lbm_step_series(a.handle, 10, 3, out, 2, cnt) == L.LBM_EINVAL
    assert a.steps == 0
    assert a.step_series(0, 4) == []
