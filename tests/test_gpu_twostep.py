"""Two-step tile shapes: one launch advances its strip by two time steps, the
intermediate post-collision populations kept on chip and rounded to the
storage type exactly as a store and a reload would round them.

Bar: every two-step shape reproduces the single-step path bitwise (every
storage type, ragged and degenerate grids, odd step counts split over calls),
and the FP64 oracle to FP32 rounding; the fused metric series and batches are
unchanged by a run's two-step tile.  Method: Li & Zhang, arXiv 2504.10539,
Sec. II-A Eq. (1).
"""
import numpy as np
import pytest

import oracle
from paper_2504_10539_amd import inputs
from tests.gpu_helpers import f32_state, lbm, need_gpu, set_state_from, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def _two_step(rows=None, storage=0):
    """Two-step shapes (moment storage: those whose strips keep four halo
    columns on each side)."""
    return [t for t in lbm().tiles() if t["steps"] == 2 and (rows is None or t["rows"] in rows)
            and (storage != 3 or t["width"] <= t["threads"] - 8)]


def _strip_tile():
    return next(t["id"] for t in lbm().tiles() if t["steps"] == 1 and not t["paired"]
                and t["threads"] == 256 and t["cells"] == 1 and t["prefetch"] == 2
                and t["rows"] == 8)


def _rho0(storage):
    return 1.0 if storage == lbm().LBM_F16_SHIFTED else 0.0


@pytest.mark.parametrize("storage", [0, 1, 2, 3])
@pytest.mark.parametrize("nx,ny", [(1, 1), (2, 5), (5, 3), (40, 9), (127, 6), (128, 4),
                                   (250, 2), (251, 13), (254, 3), (255, 6), (256, 7), (300, 77),
                                   (512, 3), (513, 5)])
def test_two_step_shapes_match_single_step(storage, nx, ny):
    """Strips narrower than the halo, one-row and short last bands, widths
    around the strip width and the workgroup width (grids up to the
    workgroup's width run as one periodic strip); 7 steps as 1 + 6 (one
    single-step launch, then three two-step launches)."""
    L = lbm()
    f0 = f32_state(inputs.random_positive_state(nx, ny, seed=nx * 7 + ny))
    ref = L.Simulation(nx, ny, -5.5, 0.8, storage, _rho0(storage))
    ref.set_tile(_strip_tile())
    set_state_from(ref, f0)
    ref.step(7)
    want = to_np(ref.get_state())
    for t in _two_step(rows=(2, 8, 128), storage=storage):
        s = L.Simulation(nx, ny, -5.5, 0.8, storage, _rho0(storage))
        s.set_tile(t["id"])
        set_state_from(s, f0)
        s.step(1)
        s.step(6)
        assert s.steps == 7
        got = to_np(s.get_state())
        assert np.array_equal(got, want), (t, nx, ny, storage)
        s.close()


def test_two_step_matches_oracle():
    nx, ny, G, tau = 96, 70, -5.5, 0.8
    f0 = f32_state(inputs.random_positive_state(nx, ny, seed=3))
    for t in _two_step(rows=(8,)):
        s = lbm().Simulation(nx, ny, G, tau)
        s.set_tile(t["id"])
        set_state_from(s, f0)
        s.step(4)
        got = to_np(s.get_state())
        ref = oracle.step(f0, G, tau, 4)
        assert float(np.max(np.abs(got - ref)) / np.max(np.abs(ref))) < 8e-6, t


def test_droplet_run_with_two_step_tile_meets_oracle_bar():
    """64^2 droplet, 1000 steps, density within 1e-5 of the oracle (Sec. III-A)."""
    N, G, tau = 64, -5.0, 1.0
    drops = inputs.single_droplet(N, 16)
    s = lbm().Simulation(N, N, G, tau).init_droplets(drops, seed=1)
    s.set_tile(_two_step(rows=(8,))[0]["id"])
    s.step(1000)
    rho = to_np(s.moments()[0])
    ref = oracle.density(oracle.step(oracle.droplet_state(N, N, drops, seed=1), G, tau, 1000, 8))
    assert float(np.max(np.abs(rho - ref) / ref)) < 1e-5


@pytest.mark.parametrize("storage", [0, 2, 3])
def test_series_with_two_step_tile_is_unchanged(storage):
    """step_series runs its recording steps with the series strip tile and the
    steps between them with the run's tile: records and final state equal
    those of a single-step run."""
    L = lbm()
    nx, ny = 200, 90
    drops = [(80.0, 45.0, 20.0), (170.0, 20.0, 9.0)]
    runs = []
    for tile in (_strip_tile(), _two_step(rows=(8,), storage=storage)[1]["id"]):
        s = L.Simulation(nx, ny, -5.5, 1.0, storage, _rho0(storage)).init_droplets(drops, seed=2)
        s.set_tile(tile)
        recs = s.step_series(25, 4)
        runs.append((recs, to_np(s.get_state()), s.steps))
    (ra, sa, na), (rb, sb, nb) = runs
    assert na == nb == 25
    assert np.array_equal(sa, sb)
    assert len(ra) == len(rb) == 7
    for a, b in zip(ra, rb):
        assert a == b


def test_batch_member_with_two_step_tile():
    """A batch whose widest member runs a two-step shape takes two steps per
    launch, plus a single-step tail launch for the odd last step of a tick:
    bitwise as alone."""
    L = lbm()
    mk = [lambda: L.Simulation(120, 64, -5.0, 1.0).init_droplets([(50, 30, 14)], seed=5),
          lambda: L.Simulation(96, 96, -5.5, 0.9, L.LBM_F16_CELL).init_droplets([(40, 40, 15)], seed=6)]
    two = _two_step(rows=(8,))[0]["id"]
    batch = [m() for m in mk]
    solo = [m() for m in mk]
    for s in batch + solo:
        s.set_tile(two)
    bt = L.Batch(batch, steps_per_graph=8)
    bt.step(13)
    for s in solo:
        s.step(13)
    for a, s in zip(batch, solo):
        assert a.steps == s.steps == 13
        assert np.array_equal(to_np(a.get_state()), to_np(s.get_state()))
    bt.close()


@pytest.mark.parametrize("K", [1, 2, 5, 8])
def test_two_step_batch_matches_single_step_runs(K):
    """Odd and even steps per graph, step counts split over calls (7 + 10),
    three storage types in one batch; every member bitwise equal to a
    single-step run of its own."""
    L = lbm()
    specs = [(130, 70, L.LBM_F32, 0.0), (64, 48, L.LBM_F16_SHIFTED, 1.0),
             (90, 90, L.LBM_F16_CELL, 0.0), (300, 40, L.LBM_F32, 0.0),
             (150, 60, L.LBM_F16_MOMENT, 0.0)]
    def make(i, nx, ny, st, r0):
        return L.Simulation(nx, ny, -5.5, 0.9, st, r0).init_droplets([(nx / 2, ny / 2, ny / 4)],
                                                                      seed=10 + i)
    batch = [make(i, *sp) for i, sp in enumerate(specs)]
    solo = [make(i, *sp) for i, sp in enumerate(specs)]
    two = next(t["id"] for t in L.tiles() if t["steps"] == 2 and t["threads"] == 128
               and t["rows"] == 4 and t["width"] == 112)
    for s in batch:
        s.set_tile(two)
    for s in solo:
        s.set_tile(_strip_tile())
    bt = L.Batch(batch, steps_per_graph=K)
    bt.step(7)
    bt.step(10)
    for s in solo:
        s.step(17)
    for a, s in zip(batch, solo):
        assert a.steps == 17
        assert np.array_equal(to_np(a.get_state()), to_np(s.get_state()))
    bt.close()
