"""Thin ctypes binding of libsclbm.so (declared in include/lbm.h).

Argument marshalling only: every step of the D2Q9 Shan-Chen path runs in the
library's gfx950 kernels.  PyTorch provides the device buffers (tensors on the
GPU) and the HIP stream.  The C functions keep their names (``lbm_create``,
``lbm_step_n``, ...); ``Simulation``, ``Batch`` and ``Server`` bundle them with
the tensors they borrow.  Importing this module fails loudly when the library
has not been built (``python -m paper_2504_10539_amd.build``).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# Always the in-tree build of this package (python -m paper_2504_10539_amd.build).
LIB_PATH = os.path.join(_HERE, "_lib", "libsclbm.so")

LBM_OK = 0
LBM_EINVAL = -1
LBM_ENOMEM = -2
LBM_EDEVICE = -3
LBM_PENDING = -4
LBM_EUNSTABLE = -5
LBM_ENOTFOUND = -6
LBM_EBUSY = -7

LBM_F32 = 0
LBM_F16_SHIFTED = 1
LBM_F16_CELL = 2
LBM_F16_MOMENT = 3
LBM_PINN_PARAMS = 33475
LBM_POLICY_CONTINUOUS = 0
LBM_POLICY_FIFO = 1

_NAMES = {0: "LBM_OK", -1: "LBM_EINVAL", -2: "LBM_ENOMEM", -3: "LBM_EDEVICE",
          -4: "LBM_PENDING", -5: "LBM_EUNSTABLE", -6: "LBM_ENOTFOUND", -7: "LBM_EBUSY"}


class LbmError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where}: {_NAMES.get(code, code)}: {msg}")
        self.code = code


class lbm_params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("G", ctypes.c_double),
                ("tau", ctypes.c_double), ("storage", ctypes.c_int32), ("rho0", ctypes.c_double)]


class lbm_init(ctypes.Structure):
    _fields_ = [("rho_l", ctypes.c_double), ("rho_g", ctypes.c_double),
                ("width", ctypes.c_double), ("noise_amp", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("period_x", ctypes.c_int64),
                ("period_y", ctypes.c_int64), ("origin_x", ctypes.c_int64),
                ("origin_y", ctypes.c_int64)]


class lbm_metrics(ctypes.Structure):
    _fields_ = [("W", ctypes.c_double), ("Gmax", ctypes.c_double), ("drho", ctypes.c_double),
                ("W_eff", ctypes.c_double), ("E_int", ctypes.c_double),
                ("rho_max", ctypes.c_double), ("rho_min", ctypes.c_double),
                ("sum_grad", ctypes.c_double), ("mass", ctypes.c_double),
                ("mom_x", ctypes.c_double), ("mom_y", ctypes.c_double),
                ("n_above", ctypes.c_int64), ("step", ctypes.c_int64),
                ("finite", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "reserved"}


class lbm_server_opts(ctypes.Structure):
    _fields_ = [("policy", ctypes.c_int32), ("steps_per_tick", ctypes.c_int32),
                ("max_slots", ctypes.c_int32), ("fake_executor", ctypes.c_int32),
                ("fake_mlups", ctypes.c_double)]


class lbm_request(ctypes.Structure):
    _fields_ = [("params", lbm_params), ("init", lbm_init),
                ("drops", ctypes.POINTER(ctypes.c_double)), ("n_drops", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("steps", ctypes.c_int64),
                ("rho_out", ctypes.c_void_p), ("f_out", ctypes.c_void_p)]


class lbm_result(ctypes.Structure):
    _fields_ = [("metrics", lbm_metrics), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double),
                ("ticket", ctypes.c_int64)]


class lbm_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("admitted", ctypes.c_int64),
                ("completed", ctypes.c_int64), ("failed", ctypes.c_int64),
                ("queued", ctypes.c_int64), ("resident", ctypes.c_int64),
                ("ticks", ctypes.c_int64), ("lattice_updates", ctypes.c_double),
                ("pool_bytes", ctypes.c_size_t), ("pool_in_use", ctypes.c_size_t),
                ("pool_high_water", ctypes.c_size_t), ("unstable", ctypes.c_int64),
                ("retired_early", ctypes.c_int64), ("unstable_updates", ctypes.c_double)]


_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_sz = ctypes.c_size_t
_P = ctypes.POINTER

_PROTOS = {
    "lbm_buffer_bytes": (_i32, [_P(lbm_params), _P(_sz), _P(_sz)]),
    "lbm_create": (_i32, [_P(lbm_params), _vp, _vp, _sz, _vp, _sz, _vp, _P(_vp)]),
    "lbm_destroy": (_i32, [_vp]),
    "lbm_init_droplets": (_i32, [_vp, _P(ctypes.c_double), _i32, _P(lbm_init)]),
    "lbm_step_n": (_i32, [_vp, _i64]),
    "lbm_step_series": (_i32, [_vp, _i64, _i32, _P(lbm_metrics), _i32, _P(_i32)]),
    "lbm_moments": (_i32, [_vp, _vp, _vp, _vp]),
    "lbm_interface_metrics": (_i32, [_vp, _P(lbm_metrics)]),
    "lbm_interface_metrics_noalloc": (_i32, [_vp, _vp]),
    "lbm_pinn_infer": (_i32, [_vp, _vp, _vp, _vp, _vp]),
    "lbm_pinn_correct": (_i32, [_vp, _vp, ctypes.c_double, _vp]),
    "lbm_get_state": (_i32, [_vp, _vp]),
    "lbm_set_state": (_i32, [_vp, _vp]),
    "lbm_step_count": (_i64, [_vp]),
    "lbm_tile_count": (_i32, []),
    "lbm_tile_describe": (_i32, [_i32, _P(_i32), _P(_i32), _P(_i32), _P(_i32), _P(_i32),
                                 _P(_i32), _P(_i32)]),
    "lbm_tile_layout": (_i32, [_P(lbm_params), _i32, _P(_i32), _P(_i32)]),
    "lbm_default_tile": (_i32, [_P(lbm_params), _P(_i32)]),
    "lbm_set_tile": (_i32, [_vp, _i32]),
    "lbm_get_tile": (_i32, [_vp]),
    "lbm_autotune": (_i32, [_vp, _i32, _P(_i32)]),
    "lbm_autotune_stepping": (_i32, [_vp, _i32, _vp, _sz, _P(_i32)]),
    "lbm_batch_work_bytes": (_i32, [_P(_vp), _i32, _P(_sz)]),
    "lbm_batch_create": (_i32, [_P(_vp), _i32, _vp, _sz, _i32, _P(_vp)]),
    "lbm_batch_step_n": (_i32, [_vp, _i64]),
    "lbm_batch_autotune": (_i32, [_vp, _i32, _P(_i32)]),
    "lbm_batch_destroy": (_i32, [_vp]),
    "lbm_server_create": (_i32, [_vp, _sz, _vp, _P(lbm_server_opts), _P(_vp)]),
    "lbm_submit": (_i32, [_vp, _P(lbm_request), _P(ctypes.c_uint64)]),
    "lbm_poll": (_i32, [_vp, ctypes.c_uint64, _P(lbm_result)]),
    "lbm_server_drain": (_i32, [_vp]),
    "lbm_server_get_stats": (_i32, [_vp, _P(lbm_server_stats)]),
    "lbm_server_clock": (ctypes.c_double, [_vp]),
    "lbm_server_destroy": (_i32, [_vp]),
    "lbm_stream_copy": (_i32, [_vp, _vp, _sz, _vp]),
    "lbm_last_error": (ctypes.c_char_p, []),
    "lbm_version": (ctypes.c_char_p, []),
}


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2504_10539_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _PROTOS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


LIB = _load()


def last_error() -> str:
    return (LIB.lbm_last_error() or b"").decode()


def _check(code: int, where: str) -> int:
    if code != LBM_OK:
        raise LbmError(code, where, last_error())
    return code


# The C functions under their own names.
for _name in _PROTOS:
    globals()[_name] = getattr(LIB, _name)


def _torch():
    import torch
    return torch


def _stream_handle(stream) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _dev_ptr(t) -> int:
    if t is None:
        return 0
    torch = _torch()
    assert isinstance(t, torch.Tensor) and t.is_cuda and t.is_contiguous()
    return int(t.data_ptr())


def _bytes_tensor(nbytes: int, device):
    torch = _torch()
    # 256-byte alignment: the caching allocator hands out 512-byte aligned blocks
    t = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
    assert t.data_ptr() % 256 == 0
    return t


def make_params(nx: int, ny: int, G: float, tau: float, storage: int = LBM_F32,
                rho0: float = 0.0) -> lbm_params:
    return lbm_params(int(nx), int(ny), float(G), float(tau), int(storage), float(rho0))


def make_init(rho_l=2.0, rho_g=0.15, width=2.0, noise_amp=1e-3, seed=1, period=(0, 0),
              origin=(0, 0)) -> lbm_init:
    return lbm_init(float(rho_l), float(rho_g), float(width), float(noise_amp),
                    int(seed) & (2**64 - 1), int(period[0]), int(period[1]), int(origin[0]),
                    int(origin[1]))


def _drops_array(drops):
    d = np.ascontiguousarray(np.asarray(drops, dtype=np.float64).reshape(-1, 3))
    return d, d.ctypes.data_as(_P(ctypes.c_double))


def buffer_bytes(nx: int, ny: int, storage: int = LBM_F32) -> tuple[int, int]:
    """(bytes of each population buffer, workspace bytes) of one run."""
    p = make_params(nx, ny, -5.0, 1.0, storage, 1.0)
    pop, work = _sz(), _sz()
    _check(LIB.lbm_buffer_bytes(ctypes.byref(p), ctypes.byref(pop), ctypes.byref(work)),
           "lbm_buffer_bytes")
    return pop.value, work.value


def carve(pool, sizes):
    """Consecutive 256-byte aligned byte views of one pool tensor, one per size."""
    out, off = [], 0
    for n in sizes:
        off = (off + 255) // 256 * 256
        if off + n > pool.numel():
            raise ValueError("pool too small")
        out.append(pool[off:off + n])
        off += n
    return out


def tiles() -> list[dict]:
    out = []
    for k in range(LIB.lbm_tile_count()):
        w, r, t, p, c, pa, st = _i32(), _i32(), _i32(), _i32(), _i32(), _i32(), _i32()
        _check(LIB.lbm_tile_describe(k, ctypes.byref(w), ctypes.byref(r), ctypes.byref(t),
                                     ctypes.byref(p), ctypes.byref(c), ctypes.byref(pa),
                                     ctypes.byref(st)),
               "lbm_tile_describe")
        out.append({"id": k, "width": w.value, "rows": r.value, "threads": t.value,
                    "prefetch": p.value, "cells": c.value, "paired": pa.value,
                    "steps": st.value})
    return out


def tile_layout(nx: int, ny: int, k: int, storage: int = LBM_F32) -> tuple[int, int]:
    """(band height, work items) of tile shape k on an nx x ny grid."""
    p = make_params(nx, ny, -5.0, 1.0, storage, 1.0 if storage == LBM_F16_SHIFTED else 0.0)
    rows, items = _i32(), _i32()
    _check(LIB.lbm_tile_layout(ctypes.byref(p), int(k), ctypes.byref(rows), ctypes.byref(items)),
           "lbm_tile_layout")
    return rows.value, items.value


def default_tile(nx: int, ny: int, storage: int = LBM_F32) -> int:
    """The built-in tile shape an nx x ny run starts with (no tuning-cache entry)."""
    p = make_params(nx, ny, -5.0, 1.0, storage, 1.0 if storage == LBM_F16_SHIFTED else 0.0)
    k = _i32()
    _check(LIB.lbm_default_tile(ctypes.byref(p), ctypes.byref(k)), "lbm_default_tile")
    return k.value


class Simulation:
    """One run: two population buffers and a workspace as torch tensors."""

    def __init__(self, nx: int, ny: int, G: float, tau: float, storage: int = LBM_F32,
                 rho0: float = 0.0, device="cuda", stream=None, buffers=None):
        """`buffers` = (popA, popB, work) device tensors to borrow (e.g. views of
        one pool, see `carve`); allocated here when omitted."""
        torch = _torch()
        self.params = make_params(nx, ny, G, tau, storage, rho0)
        pop, work = _sz(), _sz()
        _check(LIB.lbm_buffer_bytes(ctypes.byref(self.params), ctypes.byref(pop),
                                    ctypes.byref(work)), "lbm_buffer_bytes")
        self.device = torch.device(device)
        if buffers is None:
            self.popA = _bytes_tensor(pop.value, self.device)
            self.popB = _bytes_tensor(pop.value, self.device)
            self.work = _bytes_tensor(work.value, self.device)
        else:
            self.popA, self.popB, self.work = buffers
            self.device = self.popA.device
        for t in (self.popA, self.popB, self.work):
            assert t.is_cuda and t.is_contiguous() and t.data_ptr() % 256 == 0
        self.stream = stream
        h = _vp()
        _check(LIB.lbm_create(ctypes.byref(self.params), _dev_ptr(self.popA), _dev_ptr(self.popB),
                              pop.value, _dev_ptr(self.work), work.value,
                              _stream_handle(stream), ctypes.byref(h)), "lbm_create")
        self.handle = h

    @property
    def nx(self):
        return self.params.nx

    @property
    def ny(self):
        return self.params.ny

    def init_droplets(self, drops, rho_l=2.0, rho_g=0.15, width=2.0, noise_amp=1e-3, seed=1,
                      period=(0, 0), origin=(0, 0)):
        d, p = _drops_array(drops)
        ip = make_init(rho_l, rho_g, width, noise_amp, seed, period, origin)
        _check(LIB.lbm_init_droplets(self.handle, p if len(d) else None, len(d),
                                     ctypes.byref(ip)), "lbm_init_droplets")
        return self

    def step(self, n: int = 1):
        _check(LIB.lbm_step_n(self.handle, int(n)), "lbm_step_n")
        return self

    def moments(self):
        torch = _torch()
        rho = torch.empty((self.ny, self.nx), dtype=torch.float32, device=self.device)
        ux = torch.empty_like(rho)
        uy = torch.empty_like(rho)
        _check(LIB.lbm_moments(self.handle, _dev_ptr(rho), _dev_ptr(ux), _dev_ptr(uy)),
               "lbm_moments")
        return rho, ux, uy

    def metrics(self) -> dict:
        m = lbm_metrics()
        _check(LIB.lbm_interface_metrics(self.handle, ctypes.byref(m)), "lbm_interface_metrics")
        return m.as_dict()

    def step_series(self, n: int, every: int) -> list[dict]:
        """n steps; metrics of every `every`-th state on the way (ceil(n / every) records)."""
        cap = max(1, -(-int(n) // max(1, int(every))))
        out = (lbm_metrics * cap)()
        cnt = _i32()
        _check(LIB.lbm_step_series(self.handle, int(n), int(every), out, cap, ctypes.byref(cnt)),
               "lbm_step_series")
        return [out[k].as_dict() for k in range(cnt.value)]

    def pinn_infer(self, params):
        """The network's (rho, u_x, u_y) at every cell; `params` is a device
        tensor of LBM_PINN_PARAMS floats (see include/lbm.h)."""
        torch = _torch()
        assert params.dtype == torch.float32 and params.numel() == LBM_PINN_PARAMS
        out = [torch.empty((self.ny, self.nx), dtype=torch.float32, device=self.device)
               for _ in range(3)]
        _check(LIB.lbm_pinn_infer(self.handle, _dev_ptr(params), *[_dev_ptr(o) for o in out]),
               "lbm_pinn_infer")
        return tuple(out)

    def pinn_correct(self, params, beta: float, mask=None):
        """Sec. II-C correction of the state at its interface cells (in place)."""
        torch = _torch()
        assert params.dtype == torch.float32 and params.numel() == LBM_PINN_PARAMS
        if mask is not None:
            assert mask.dtype == torch.uint8 and mask.numel() == self.nx * self.ny
        _check(LIB.lbm_pinn_correct(self.handle, _dev_ptr(params), float(beta), _dev_ptr(mask)),
               "lbm_pinn_correct")
        return self

    def get_state(self):
        torch = _torch()
        f = torch.empty((9, self.ny, self.nx), dtype=torch.float32, device=self.device)
        _check(LIB.lbm_get_state(self.handle, _dev_ptr(f)), "lbm_get_state")
        return f

    def set_state(self, f):
        torch = _torch()
        f = f.to(device=self.device, dtype=torch.float32).contiguous()
        assert tuple(f.shape) == (9, self.ny, self.nx)
        _check(LIB.lbm_set_state(self.handle, _dev_ptr(f)), "lbm_set_state")
        self._keep = f
        return self

    @property
    def steps(self) -> int:
        return int(LIB.lbm_step_count(self.handle))

    def set_tile(self, k: int):
        _check(LIB.lbm_set_tile(self.handle, int(k)), "lbm_set_tile")
        return self

    @property
    def tile(self) -> int:
        return int(LIB.lbm_get_tile(self.handle))

    def autotune(self, reps: int = 5, stepping: bool = True) -> int:
        """Selects the fastest tile shape.  stepping=True times the shapes as
        the run steps (lbm_autotune_stepping, with a scratch copy of the state
        allocated here for the call; where the device has no room for it, the
        shapes are timed over the unchanged state instead); False times
        repeated launches over the unchanged state (lbm_autotune)."""
        best = _i32()
        pop = _sz()
        _check(LIB.lbm_buffer_bytes(ctypes.byref(self.params), ctypes.byref(pop), None),
               "lbm_buffer_bytes")
        scratch = None
        if stepping:
            try:
                scratch = _bytes_tensor(pop.value, self.device)
            except _torch().cuda.OutOfMemoryError:
                scratch = None
        if scratch is None:
            _check(LIB.lbm_autotune(self.handle, int(reps), ctypes.byref(best)), "lbm_autotune")
            return best.value
        _check(LIB.lbm_autotune_stepping(self.handle, int(reps), _dev_ptr(scratch), pop.value,
                                         ctypes.byref(best)), "lbm_autotune_stepping")
        del scratch
        return best.value

    def close(self):
        if getattr(self, "handle", None):
            _check(LIB.lbm_destroy(self.handle), "lbm_destroy")
            self.handle = None

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                LIB.lbm_destroy(self.handle)
                self.handle = None
        except Exception:
            pass


class Batch:
    """Several simulations advanced together by the batched graph."""

    def __init__(self, sims: Sequence[Simulation], steps_per_graph: int = 30):
        self.sims = list(sims)
        arr = (_vp * len(self.sims))(*[s.handle for s in self.sims])
        nbytes = _sz()
        _check(LIB.lbm_batch_work_bytes(arr, len(self.sims), ctypes.byref(nbytes)),
               "lbm_batch_work_bytes")
        self.work = _bytes_tensor(nbytes.value, self.sims[0].device)
        h = _vp()
        _check(LIB.lbm_batch_create(arr, len(self.sims), _dev_ptr(self.work), nbytes.value,
                                    int(steps_per_graph), ctypes.byref(h)), "lbm_batch_create")
        self.handle = h

    def step(self, n: int):
        _check(LIB.lbm_batch_step_n(self.handle, int(n)), "lbm_batch_step_n")
        return self

    def autotune(self, reps: int = 3) -> int:
        best = _i32()
        _check(LIB.lbm_batch_autotune(self.handle, int(reps), ctypes.byref(best)),
               "lbm_batch_autotune")
        return best.value

    def close(self):
        if getattr(self, "handle", None):
            _check(LIB.lbm_batch_destroy(self.handle), "lbm_batch_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching serving loop over one pool tensor."""

    def __init__(self, pool_bytes: int, policy: int = LBM_POLICY_CONTINUOUS,
                 steps_per_tick: int = 30, max_slots: int = 256, fake: bool = False,
                 fake_mlups: float = 1000.0, device="cuda", stream=None):
        self.pool = None if fake else _bytes_tensor(pool_bytes, _torch().device(device))
        opts = lbm_server_opts(int(policy), int(steps_per_tick), int(max_slots), int(bool(fake)),
                               float(fake_mlups))
        h = _vp()
        _check(LIB.lbm_server_create(_dev_ptr(self.pool) if self.pool is not None else None,
                                     int(pool_bytes), 0 if fake else _stream_handle(stream),
                                     ctypes.byref(opts), ctypes.byref(h)), "lbm_server_create")
        self.handle = h
        self._keep = {}

    def submit(self, nx, ny, G, tau, steps, drops, storage=LBM_F32, rho0=0.0, rho_l=2.0,
               rho_g=0.15, width=2.0, noise_amp=1e-3, seed=1, rho_out=None, f_out=None) -> int:
        d, p = _drops_array(drops)
        req = lbm_request(make_params(nx, ny, G, tau, storage, rho0),
                          make_init(rho_l, rho_g, width, noise_amp, seed), p if len(d) else None,
                          len(d), 0, int(steps), _dev_ptr(rho_out), _dev_ptr(f_out))
        t = ctypes.c_uint64()
        _check(LIB.lbm_submit(self.handle, ctypes.byref(req), ctypes.byref(t)), "lbm_submit")
        self._keep[t.value] = (rho_out, f_out)
        return t.value

    def poll(self, ticket: int):
        """None while pending; else (status, result dict)."""
        r = lbm_result()
        code = LIB.lbm_poll(self.handle, int(ticket), ctypes.byref(r))
        if code == LBM_PENDING:
            return None
        if code == LBM_ENOTFOUND:
            raise LbmError(code, "lbm_poll", last_error())
        self._keep.pop(int(ticket), None)
        out = r.metrics.as_dict()
        out.update(t_submit=r.t_submit, t_admit=r.t_admit, t_done=r.t_done, ticket=r.ticket)
        return code, out

    def drain(self):
        _check(LIB.lbm_server_drain(self.handle), "lbm_server_drain")

    def stats(self) -> dict:
        s = lbm_server_stats()
        _check(LIB.lbm_server_get_stats(self.handle, ctypes.byref(s)), "lbm_server_get_stats")
        return {name: getattr(s, name) for name, _ in s._fields_}

    def clock(self) -> float:
        return float(LIB.lbm_server_clock(self.handle))

    def close(self):
        if getattr(self, "handle", None):
            _check(LIB.lbm_server_destroy(self.handle), "lbm_server_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def stream_copy(dst, src, nbytes: Optional[int] = None, stream=None):
    n = int(nbytes if nbytes is not None else src.numel() * src.element_size())
    _check(LIB.lbm_stream_copy(_dev_ptr(dst), _dev_ptr(src), n, _stream_handle(stream)),
           "lbm_stream_copy")
