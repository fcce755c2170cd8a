"""lbm_interface_metrics_noalloc against lbm_interface_metrics.

The no-allocation variant runs the same kernels with its reduction partials in
a static device array and writes the lbm_metrics record to device memory; on
the same state it must report exactly what the allocating entry point
reports.  Two calls in a row, the second on a smaller grid, so that the
shared array's contents from the first call cannot leak into the second.
"""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2504_10539_amd import inputs
from tests.gpu_helpers import lbm, need_gpu, to_np, torch

pytestmark = pytest.mark.gpu

FIELDS = ("W", "Gmax", "drho", "W_eff", "E_int", "rho_max", "rho_min", "sum_grad", "mass",
          "mom_x", "mom_y", "n_above", "step", "finite")


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def _noalloc(L, sim):
    out = torch.zeros(ctypes.sizeof(L.lbm_metrics), dtype=torch.uint8, device=sim.device)
    code = L.LIB.lbm_interface_metrics_noalloc(sim.handle, out.data_ptr())
    assert code == L.LBM_OK, L.last_error()
    torch.cuda.synchronize()
    return L.lbm_metrics.from_buffer_copy(out.cpu().numpy().tobytes()).as_dict()


@pytest.mark.parametrize("storage", [0, 1, 2])
def test_noalloc_metrics_equal_the_allocating_entry_point(storage):
    L = lbm()
    # the second grid is smaller: fewer partial records than the first call left
    for n, m, steps in ((640, 520, 37), (96, 80, 12)):
        sim = L.Simulation(n, m, -5.0, 1.0, storage, 1.0 if storage == 1 else 0.0)
        sim.init_droplets([(n / 2, m / 2, min(n, m) / 5), (n / 5, m / 4, 9.0)], seed=7)
        sim.step(steps)
        got = _noalloc(L, sim)
        ref = sim.metrics()
        for k in FIELDS:
            assert got[k] == ref[k], (n, k, got[k], ref[k])
        # and the FP64 metrics agree with the oracle's on the same stored state
        rho = oracle.density(to_np(sim.get_state()))
        mo = oracle.metrics(rho)
        assert got["n_above"] == mo["n_above"]
        for k in ("Gmax", "drho", "W_eff", "E_int"):
            assert abs(got[k] - mo[k]) <= 1e-12 * max(1.0, abs(mo[k])), k
        sim.close()


def test_noalloc_rejects_bad_arguments():
    L = lbm()
    sim = L.Simulation(64, 64, -5.0, 1.0).init_droplets(inputs.single_droplet(64, 16), seed=1)
    out = torch.zeros(256, dtype=torch.uint8, device="cuda")
    assert L.LIB.lbm_interface_metrics_noalloc(sim.handle, None) == L.LBM_EINVAL
    assert L.LIB.lbm_interface_metrics_noalloc(None, out.data_ptr()) == L.LBM_EINVAL
    assert L.LIB.lbm_interface_metrics_noalloc(sim.handle, out.data_ptr() + 4) == L.LBM_EINVAL
    assert "aligned" in L.last_error()
