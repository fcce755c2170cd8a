"""The largest grid the library accepts (9 nx ny < 2^32 elements per buffer):
21844^2 cells, 17.2 GB per FP32 buffer, so row addresses pass 4 GiB.  Run in
the benchmark's launch configuration (autotuned tile), checked against the
FP64 oracle on sampled windows (including the far corner of the grid) and
for mass conservation; and the argument checks at and past the limit."""
import numpy as np
import pytest

import oracle
from paper_2504_10539_amd import inputs
from tests.gpu_helpers import lbm, need_gpu, to_np

pytestmark = pytest.mark.gpu

N = 21844
K, WIN = 8, 64
LO, HI = 2 * K, WIN - 2 * K


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def test_size_limit_is_enforced():
    L = lbm()
    ok = L.lbm_params(N, N, -5.0, 1.0, L.LBM_F32, 0.0)
    assert L.LIB.lbm_buffer_bytes(ok, None, None) == L.LBM_OK
    big = L.lbm_params(N + 2, N + 2, -5.0, 1.0, L.LBM_F32, 0.0)
    assert L.LIB.lbm_buffer_bytes(big, None, None) == L.LBM_EINVAL


def test_init_window_must_lie_inside_frame():
    L = lbm()
    s = L.Simulation(64, 64, -5.0, 1.0)
    with pytest.raises(L.LbmError):
        s.init_droplets([(10, 10, 5)], period=(100, 100), origin=(40, 0))
    s.init_droplets([(10, 10, 5)], period=(100, 100), origin=(36, 36))


def test_max_grid_fp32_windows_and_mass(nthreads):
    L = lbm()
    G, tau = -5.0, 1.0
    drops = inputs.many_droplets(N, 400, 8, 48, seed=7)
    sim = L.Simulation(N, N, G, tau).init_droplets(drops, seed=7)
    sim.autotune(reps=1)
    m0 = sim.metrics()
    sim.step(K)
    state = sim.get_state()
    rng = np.random.default_rng(3)
    origins = [tuple(int(v) for v in rng.integers(0, N - WIN, 2)) for _ in range(3)]
    origins.append((N - WIN, N - WIN))
    errs = []
    for ox, oy in origins:
        f0 = oracle.droplet_state(WIN, WIN, drops, seed=7, period=(N, N), origin=(ox, oy))
        ref = oracle.step(f0, G, tau, K, nthreads)[:, LO:HI, LO:HI]
        got = to_np(state[:, oy + LO:oy + HI, ox + LO:ox + HI])
        errs.append(float(np.max(np.abs(got - ref)) / np.max(np.abs(ref))))
    del state
    print("max grid window errors", errs)
    assert max(errs) < 5e-6
    sim.step(32 - K)
    m1 = sim.metrics()
    assert m1["finite"] == 1
    assert abs(m1["mass"] / m0["mass"] - 1) < 1e-6
    sim.close()
