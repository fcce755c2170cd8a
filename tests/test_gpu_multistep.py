"""Three-step tile shapes (FP32): one launch advances its strip by K = 3 time
steps, the intermediate post-collision states kept on chip.

Bar: every such shape reproduces the single-step path bitwise (ragged and
degenerate grids, step counts that are not multiples of K, split over calls)
and the FP64 oracle to FP32 rounding; a metric series and a batch are
unchanged by a run's K-step tile.  Method: Li & Zhang, arXiv 2504.10539,
Sec. II-A Eq. (1).
"""
import itertools

import numpy as np
import pytest

import oracle
from paper_2504_10539_amd import inputs
from tests.gpu_helpers import f32_state, lbm, need_gpu, set_state_from, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def _multi_step(rows=None, steps=(3,)):
    return [t for t in lbm().tiles() if t["steps"] in steps and (rows is None or t["rows"] in rows)]


def _strip_tile():
    return next(t["id"] for t in lbm().tiles() if t["steps"] == 1 and not t["paired"]
                and t["threads"] == 256 and t["cells"] == 1 and t["prefetch"] == 2
                and t["rows"] == 8)


@pytest.mark.parametrize("nx,ny", [(1, 1), (2, 5), (5, 3), (7, 4), (40, 9), (117, 6), (128, 4),
                                   (240, 2), (241, 13), (245, 3), (246, 6), (256, 7), (300, 77),
                                   (512, 3), (513, 5)])
def test_multi_step_shapes_match_single_step(nx, ny):
    """Strips narrower than the halo, short and one-row bands, widths around
    the strip and workgroup widths (grids up to the workgroup's width run as
    one periodic strip); 16 steps as 1 + 10 + 5 (a single step; three
    launches and a single step; one launch and the two steps left over in
    the two-step variant of the same strips)."""
    L = lbm()
    f0 = f32_state(inputs.random_positive_state(nx, ny, seed=nx * 11 + ny))
    ref = L.Simulation(nx, ny, -5.5, 0.8)
    ref.set_tile(_strip_tile())
    set_state_from(ref, f0)
    ref.step(16)
    want = to_np(ref.get_state())
    for t in _multi_step(rows=(2, 8, 128)):
        s = L.Simulation(nx, ny, -5.5, 0.8)
        s.set_tile(t["id"])
        set_state_from(s, f0)
        s.step(1)
        s.step(10)
        s.step(5)
        assert s.steps == 16
        got = to_np(s.get_state())
        assert np.array_equal(got, want), (t, nx, ny)
        s.close()


def test_multi_step_refused_by_fp16_storage():
    L = lbm()
    for t, st in itertools.product(_multi_step(rows=(8,)),
                                   (L.LBM_F16_SHIFTED, L.LBM_F16_CELL, L.LBM_F16_MOMENT)):
        s = L.Simulation(64, 64, -5.0, 1.0, st, 1.0 if st == L.LBM_F16_SHIFTED else 0.0)
        with pytest.raises(L.LbmError) as e:
            s.set_tile(t["id"])
        assert e.value.code == L.LBM_EINVAL


@pytest.mark.parametrize("k", [3])
def test_multi_step_droplet_meets_oracle(k):
    """A droplet run with the balanced K-step shape against the FP64 oracle."""
    L = lbm()
    N = 96
    drops = inputs.single_droplet(N, 20)
    bal = next(t for t in _multi_step(steps=(k,)) if t["threads"] == 256 and t["prefetch"] == 1
               and t["rows"] == 0)
    s = L.Simulation(N, N, -5.0, 1.0).init_droplets(drops, seed=1)
    s.set_tile(bal["id"])
    s.step(300)
    ref = oracle.step(oracle.droplet_state(N, N, drops, seed=1), -5.0, 1.0, 300, 8)
    rho = to_np(s.moments()[0])
    rho_ref = oracle.density(ref)
    assert float(np.max(np.abs(rho - rho_ref) / rho_ref)) < 1e-5


@pytest.mark.parametrize("k", [3])
def test_series_with_multi_step_tile_is_unchanged(k):
    L = lbm()
    nx, ny = 200, 90
    drops = [(80.0, 45.0, 20.0), (170.0, 20.0, 9.0)]
    runs = []
    for tile in (_strip_tile(), _multi_step(rows=(8,), steps=(k,))[1]["id"]):
        s = L.Simulation(nx, ny, -5.5, 1.0).init_droplets(drops, seed=2)
        s.set_tile(tile)
        recs = s.step_series(25, 4)
        runs.append((recs, to_np(s.get_state()), s.steps))
    (ra, sa, na), (rb, sb, nb) = runs
    assert na == nb == 25
    assert np.array_equal(sa, sb)
    assert ra == rb


@pytest.mark.parametrize("spg", [1, 2, 3, 4, 8])
def test_batch_with_three_step_tile(spg):
    """A batch whose FP32 members run a three-step tile: floor(K / 3) three-step
    launches per tick of K steps, then the two steps left over in the two-step
    variant of the same strips or the one left over in a single step.  13 and
    then 5 steps (ticks that leave 0, 1 and 2 steps over), bitwise as alone;
    an FP16 member beside them keeps its two-step launches."""
    L = lbm()
    mk = [lambda: L.Simulation(120, 64, -5.0, 1.0).init_droplets([(50, 30, 14)], seed=5),
          lambda: L.Simulation(300, 96, -5.5, 0.9).init_droplets([(140, 40, 15)], seed=6),
          lambda: L.Simulation(200, 80, -5.0, 1.0, L.LBM_F16_CELL).init_droplets([(90, 40, 12)],
                                                                                 seed=7)]
    multi = _multi_step(rows=(8,))[0]["id"]  # 128 threads, 112 columns
    batch = [m() for m in mk]
    solo = [m() for m in mk]
    for s in batch[:2]:
        s.set_tile(multi)
    bt = L.Batch(batch, steps_per_graph=spg)
    for n in (13, 5):
        bt.step(n)
        for s in solo:
            s.step(n)
        for a, s in zip(batch, solo):
            assert a.steps == s.steps
            assert np.array_equal(to_np(a.get_state()), to_np(s.get_state())), (spg, n)
    bt.close()
