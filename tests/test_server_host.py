"""Scheduling logic of the serving loop, on the host-only fake executor (no GPU).

The fake executor runs the same admission, budget, bypass, retirement and
polling code as the GPU path; a tick sleeps for the time its lattice updates
would take at `fake_mlups` instead of launching kernels.
"""
import threading
import time

import pytest

from paper_2504_10539_amd import lbm as _lbm_mod  # noqa: F401  (loads the library)


@pytest.fixture
def lbm():
    from paper_2504_10539_amd import lbm
    return lbm


def req_bytes(lbm, n):
    import ctypes
    p = lbm.make_params(n, n, -5.0, 1.0)
    pop, work = ctypes.c_size_t(), ctypes.c_size_t()
    lbm.LIB.lbm_buffer_bytes(ctypes.byref(p), ctypes.byref(pop), ctypes.byref(work))
    up = lambda v: (v + 255) // 256 * 256
    return 2 * up(pop.value) + up(work.value)


def test_poll_states_and_results(lbm):
    s = lbm.Server(1 << 30, fake=True, fake_mlups=20.0, steps_per_tick=50, max_slots=4)
    t = s.submit(64, 64, -5.0, 1.0, 500, [(32, 32, 16)])
    assert s.poll(t) is None  # 2M updates at 20 MLUPS: still running
    s.drain()
    code, m = s.poll(t)
    assert code == lbm.LBM_OK and m["step"] == 500 and m["finite"] == 1
    assert m["t_submit"] <= m["t_admit"] <= m["t_done"]
    with pytest.raises(lbm.LbmError):
        s.poll(t)
    with pytest.raises(lbm.LbmError):
        s.poll(12345)
    s.close()


def test_rejects_invalid_and_oversized(lbm):
    s = lbm.Server(8 << 20, fake=True, fake_mlups=1000.0)
    with pytest.raises(lbm.LbmError) as e:
        s.submit(64, 64, -5.0, 0.5, 10, [(32, 32, 8)])
    assert e.value.code == lbm.LBM_EINVAL
    with pytest.raises(lbm.LbmError) as e:
        s.submit(64, 64, -5.0, 1.0, -1, [(32, 32, 8)])
    assert e.value.code == lbm.LBM_EINVAL
    with pytest.raises(lbm.LbmError) as e:
        s.submit(2048, 2048, -5.0, 1.0, 10, [(32, 32, 8)])
    assert e.value.code == lbm.LBM_ENOMEM
    s.close()


def test_budget_is_never_exceeded(lbm):
    one = req_bytes(lbm, 256)
    pool = 2 * one + one // 2  # room for two at a time
    s = lbm.Server(pool, fake=True, fake_mlups=200.0, steps_per_tick=20, max_slots=64)
    tickets = [s.submit(256, 256, -5.0, 1.0, 200, [(128, 128, 30)], seed=k) for k in range(8)]
    s.drain()
    res = [s.poll(t)[1] for t in tickets]
    st = s.stats()
    assert st["completed"] == 8 and st["failed"] == 0
    assert st["pool_high_water"] <= pool and st["pool_high_water"] >= 2 * one
    # never more than two resident: at any admission time at most one other is running
    for r in res:
        overlapping = sum(1 for q in res if q["t_admit"] <= r["t_admit"] < q["t_done"])
        assert overlapping <= 2
    s.close()


def tables_bytes(lbm, pool, **kw):
    """Bytes the continuous policy keeps for its batch tables out of a pool."""
    s = lbm.Server(pool, fake=True, fake_mlups=1000.0, **kw)
    cap = s.stats()["pool_bytes"]
    s.close()
    return pool - cap


def test_small_requests_pass_a_large_one_that_does_not_fit(lbm):
    small, big = req_bytes(lbm, 128), req_bytes(lbm, 512)
    # the big one fits only when the requests' part of the pool is empty
    pool = big + small // 2 + tables_bytes(lbm, big + small, max_slots=64)
    s = lbm.Server(pool, fake=True, fake_mlups=100.0, steps_per_tick=20, max_slots=64)
    assert big <= s.stats()["pool_bytes"] < big + small
    t0 = s.submit(128, 128, -5.0, 1.0, 2000, [(64, 64, 20)])          # long small job
    t1 = s.submit(512, 512, -5.0, 1.0, 20, [(256, 256, 40)])           # big, must wait
    rest = [s.submit(128, 128, -5.0, 1.0, 20, [(64, 64, 20)]) for _ in range(3)]
    s.drain()
    r0, r1 = s.poll(t0)[1], s.poll(t1)[1]
    others = [s.poll(t)[1] for t in rest]
    assert r1["t_admit"] >= r0["t_done"] - 1e-3          # waited for the pool to free
    assert min(o["t_admit"] for o in others) < r1["t_admit"]  # later small ones went first
    s.close()


def test_fifo_policy_runs_one_at_a_time_in_order(lbm):
    s = lbm.Server(1 << 30, policy=lbm.LBM_POLICY_FIFO, fake=True, fake_mlups=100.0,
                   steps_per_tick=50, max_slots=16)
    tickets = [s.submit(96, 96, -5.0, 1.0, 100 * (k + 1), [(48, 48, 12)]) for k in range(5)]
    s.drain()
    res = [s.poll(t)[1] for t in tickets]
    for a, b in zip(res, res[1:]):
        assert b["t_admit"] >= a["t_done"] - 1e-3
    s.close()


def test_unstable_request_is_flagged_and_others_complete(lbm):
    s = lbm.Server(1 << 30, fake=True, fake_mlups=1000.0, steps_per_tick=10)
    good = s.submit(64, 64, -5.0, 1.0, 30, [(32, 32, 10)])
    bad = s.submit(64, 64, -5.0, 1.0, 30, [(32, 32, 10)], rho_g=-0.1)
    s.drain()
    code, rb = s.poll(bad)
    assert code == lbm.LBM_EUNSTABLE
    assert rb["step"] == 10 and rb["finite"] == 0  # retired after its first tick
    assert s.poll(good)[0] == lbm.LBM_OK
    st = s.stats()
    assert st["failed"] == 1 and st["unstable"] == 1 and st["retired_early"] == 1
    # throughput counts the stable request only; the unstable one's work apart
    assert st["lattice_updates"] == 64 * 64 * 30
    assert st["unstable_updates"] == 64 * 64 * 10
    s.close()


def test_diverging_request_retires_long_before_a_stable_one(lbm):
    """An unstable run leaves at its first tick instead of running its steps."""
    s = lbm.Server(1 << 30, fake=True, fake_mlups=50.0, steps_per_tick=50, max_slots=4)
    stable = s.submit(128, 128, -5.0, 1.0, 2000, [(64, 64, 20)])
    bad = s.submit(128, 128, -5.0, 1.0, 2000, [(64, 64, 20)], rho_g=-0.2)
    s.drain()
    _, rs = s.poll(stable)
    code, rb = s.poll(bad)
    assert code == lbm.LBM_EUNSTABLE and rb["step"] == 50
    assert rb["t_done"] - rb["t_admit"] < 0.1 * (rs["t_done"] - rs["t_admit"])
    s.close()


def test_capacity_excludes_the_batch_tables(lbm):
    """The continuous policy keeps its batch tables in the pool: a request larger
    than what is left is refused at submission instead of waiting forever."""
    one = req_bytes(lbm, 1024)
    pool = one + (64 << 10)
    s = lbm.Server(pool, fake=True, fake_mlups=1000.0, max_slots=4)
    cap = s.stats()["pool_bytes"]
    assert cap < one <= pool  # the tables take more than 64 KiB
    with pytest.raises(lbm.LbmError) as e:
        s.submit(1024, 1024, -5.0, 1.0, 10, [(512, 512, 100)])
    assert e.value.code == lbm.LBM_ENOMEM
    t = s.submit(512, 512, -5.0, 1.0, 10, [(256, 256, 60)])
    s.drain()
    assert s.poll(t)[0] == lbm.LBM_OK
    s.close()
    # the plain FIFO path keeps no tables: the whole pool is its budget
    f = lbm.Server(pool, policy=lbm.LBM_POLICY_FIFO, fake=True, fake_mlups=1000.0)
    assert f.stats()["pool_bytes"] == pool
    t = f.submit(1024, 1024, -5.0, 1.0, 10, [(512, 512, 100)])
    f.drain()
    assert f.poll(t)[0] == lbm.LBM_OK
    f.close()


def test_droplet_count_is_checked_before_the_array_is_read(lbm):
    """A huge n_drops with a one-droplet array is refused without reading past it."""
    import ctypes
    import numpy as np
    s = lbm.Server(1 << 30, fake=True, fake_mlups=1000.0)
    d = np.array([[32.0, 32.0, 8.0]])
    for n in (2**31 - 1, 10000):  # above the 4778 droplets a 64^2 FP32 grid holds
        req = lbm.lbm_request(lbm.make_params(64, 64, -5.0, 1.0), lbm.make_init(),
                              d.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n, 0, 10,
                              None, None)
        t = ctypes.c_uint64()
        code = lbm.LIB.lbm_submit(s.handle, ctypes.byref(req), ctypes.byref(t))
        assert code == lbm.LBM_EINVAL
        assert "droplets" in lbm.last_error()
    s.close()


def test_concurrent_submitters(lbm):
    s = lbm.Server(1 << 30, fake=True, fake_mlups=5000.0, steps_per_tick=10, max_slots=8)
    out, lock = [], threading.Lock()

    def worker(k):
        for j in range(10):
            t = s.submit(64, 64, -5.0, 1.0, 20, [(32, 32, 10)], seed=k * 100 + j)
            with lock:
                out.append(t)

    th = [threading.Thread(target=worker, args=(k,)) for k in range(4)]
    for x in th:
        x.start()
    for x in th:
        x.join()
    s.drain()
    assert len(set(out)) == 40
    assert all(s.poll(t)[0] == lbm.LBM_OK for t in out)
    assert s.stats()["completed"] == 40
    s.close()


def test_zero_step_request_completes(lbm):
    s = lbm.Server(1 << 30, fake=True, fake_mlups=1000.0)
    t = s.submit(32, 32, -5.0, 1.0, 0, [])
    s.drain()
    assert s.poll(t)[0] == lbm.LBM_OK
    s.close()
