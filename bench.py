#!/usr/bin/env python3
"""Benchmark of the D2Q9 Shan-Chen step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

A bench "step" is one pass of the whole hot path over the many-droplet
workload: droplet initialisation, `--lbm-steps` (default 5000) fused
stream-collide-force time steps, FP64 conservation + interface metrics, and
the moments export, on a 4096 x 4096 periodic grid with 2000 droplets (centres
uniform, R uniform in [8, 48], max-merged, tanh width 2, noise 1e-3), G = -5.5
and tau = 1.0 (the paper's Sec. III-A values; with tau = 0.8 this field goes
non-finite within about 100 steps, in the FP64 oracle as on the GPU).
Populations are FP32; the arithmetic is FP32.

`value` is lattice updates per second (MLUPS) of the whole job with the inputs
resident; `roofline` prices the step kernel (the dominant kernel), with its
average launch time measured by HIP events on its stream over the timed
region.  A kernel that moves the populations once per one or two updates is
priced at 72 algorithmic bytes per launch and cell against the 8 TB/s HBM
peak; one that takes three updates per launch is bound by its vector ALU
work and is priced at 106 algorithmic FP32 operations per lattice update
against the vector issue peak (256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3
T lane operations per second without packed FP32), its HBM figures beside.  Extra objects report the FP16-shifted storage, a 1024^2
single-droplet run, the paper's own droplet protocol (Tables I-II layout), the
batched parameter sweep, the serving loop and the FP64 oracle's CPU rate.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

HBM_PEAK_GBS = 8000.0
# FP32 vector operations of one lattice update (density 8, psi 7, force 13,
# momentum 8, 1/rho 3, velocity 4, u^2 term 3, weights 4, the four
# equilibrium pairs 30, f_eq_0 8, relaxation 18); an FMA counts as one
ALU_OPS_PER_UPDATE = 106
ALU_PEAK_GOPS = 256 * 4 * 16 * 2.4  # lane operations per ns (one per lane per clock)
BYTES_F32 = 72   # 9 populations read + 9 written, 4 bytes each
BYTES_F16 = 36
BYTES_F16_CELL = 40  # 18 B read + 18 B written, plus the 2-byte reference density each way
BYTES_F16_MOMENT = 48  # 24 B record read + 24 B written (rho, jx, jy in FP32; six FP16 values)


def log(msg: str):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("sc_device.h", "sc_kernels.hip"):
        with open(os.path.join(HERE, "paper_2504_10539_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(lbm, kernel_hash: str, storage: str, n: int, tile: int):
    """HBM bytes per launch of the step kernel with this tile shape, from the
    committed rocprofv3 counter summary; None when the summary has no entry for
    it or was taken on other kernel sources."""
    path = os.path.join(HERE, "profiles", "step_counters.json")
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    t = lbm.tiles()[tile]
    code = {"f32": lbm.LBM_F32, "f16_shifted": lbm.LBM_F16_SHIFTED, "f16_cell": lbm.LBM_F16_CELL,
            "f16_moment": lbm.LBM_F16_MOMENT}[storage]
    rows = lbm.tile_layout(n, n, tile, code)[0]  # the band height this grid uses
    key = (storage, n, kernel_name(lbm, tile, code), t["width"], rows)
    for e in d.get("entries", []):
        if (e.get("storage"), e.get("n"), e.get("kernel"), e.get("width"), e.get("rows")) == key:
            return e.get("bytes_per_launch") if e.get("kernel_hash") == kernel_hash else None
    return None


def kernel_name(lbm, tile: int, storage: int) -> str:
    """Name of the step kernel instance that tile shape `tile` launches."""
    t = lbm.tiles()[tile]
    st = {lbm.LBM_F32: "StoreF32", lbm.LBM_F16_SHIFTED: "StoreF16S", lbm.LBM_F16_CELL: "StoreF16C",
          lbm.LBM_F16_MOMENT: "StoreF16M"}[storage]
    if t["steps"] >= 3:  # FP32 only
        return f"k_step{t['steps']}<{t['threads']}, {t['prefetch']}, {t['width']}>"
    if t["steps"] == 2:
        return f"k_step2<{st}, {t['threads']}, {t['prefetch']}, {t['width']}>"
    if t["paired"]:
        return f"k_step_pair<{st}, {t['threads'] // 64}, {t['prefetch']}>"
    return f"k_step<{st}, {t['threads']}, {t['cells']}, {t['prefetch']}>"


def launch_figures(lbm, tile: int, step_ms: float, bytes_per_update: int, cells: int) -> dict:
    """Per-launch roofline figures of the step kernel.  A launch reads and
    writes every population once, whether it advances one time step or two
    (two-step tile shapes), so its algorithmic bytes are bytes_per_update x
    cells either way; `step_ms` is the measured time per time step."""
    spl = lbm.tiles()[tile]["steps"]
    launch_ms = step_ms * spl
    gbs = bytes_per_update * cells / (launch_ms * 1e-3) / 1e9
    return {"steps_per_launch": spl, "launch_ms": launch_ms, "achieved_gbs": gbs}


def roofline_bound(r: dict) -> dict:
    """Bound, achieved rate, peak and fraction of the step kernel of leg r.
    Three updates per launch: the vector ALU (algorithmic operations per
    launch / launch time against the issue peak), with the per-launch HBM
    figures beside; otherwise HBM (72 algorithmic bytes per cell and launch)."""
    hbm = {"achieved": round(r["achieved_gbs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(r["achieved_gbs"] / HBM_PEAK_GBS, 4)}
    if r["steps_per_launch"] < 3:
        return dict(bound="hbm", **hbm)
    gops = ALU_OPS_PER_UPDATE * r["steps_per_launch"] * r["cells"] / (r["launch_ms"] * 1e6)
    return {"bound": "alu", "achieved": round(gops, 1), "peak": round(ALU_PEAK_GOPS, 1),
            "unit": "Gop/s", "frac": round(gops / ALU_PEAK_GOPS, 4),
            "ops_per_update": ALU_OPS_PER_UPDATE, "hbm": hbm}


def run_main(args, torch, lbm, inputs):
    N = args.n
    drops = inputs.many_droplets(N, args.drops, 8, 48, seed=3)
    stream = torch.cuda.current_stream()
    out = {}
    for storage, name in ((lbm.LBM_F32, "f32"), (lbm.LBM_F16_SHIFTED, "f16_shifted"),
                          (lbm.LBM_F16_CELL, "f16_cell"), (lbm.LBM_F16_MOMENT, "f16_moment")):
        if storage != lbm.LBM_F32 and args.no_fp16:
            continue
        if args.storages and name not in args.storages.split(","):
            continue
        rho0 = 1.0 if storage == lbm.LBM_F16_SHIFTED else 0.0
        sim = lbm.Simulation(N, N, args.G, args.tau, storage, rho0)
        sim.init_droplets(drops, seed=3)
        if args.tile >= 0:
            sim.set_tile(args.tile)
        elif not args.no_autotune:
            sim.autotune(reps=8)
        rho = torch.empty((N, N), dtype=torch.float32, device="cuda")
        ux = torch.empty_like(rho)
        uy = torch.empty_like(rho)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

        def job(timed_step_events=None):
            sim.init_droplets(drops, seed=3)
            if timed_step_events:
                timed_step_events[0].record(stream)
            sim.step(args.lbm_steps)
            if timed_step_events:
                timed_step_events[1].record(stream)
            m = sim.metrics()
            lbm.LIB.lbm_moments(sim.handle, rho.data_ptr(), ux.data_ptr(), uy.data_ptr())
            return m

        for _ in range(args.warmup):
            job()
        torch.cuda.synchronize()
        step_ms = []
        t0 = time.perf_counter()
        m = None
        for _ in range(args.steps):
            evs = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            m = job(evs)
            step_ms.append(evs[0].elapsed_time(evs[1]))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        lu = float(N) * N * args.lbm_steps * args.steps
        per_step_ms = sum(step_ms) / (args.lbm_steps * args.steps)
        bpu = {lbm.LBM_F32: BYTES_F32, lbm.LBM_F16_SHIFTED: BYTES_F16,
               lbm.LBM_F16_CELL: BYTES_F16_CELL, lbm.LBM_F16_MOMENT: BYTES_F16_MOMENT}[storage]
        lf = launch_figures(lbm, sim.tile, per_step_ms, bpu, N * N)
        out[name] = {
            "mlups": lu / wall / 1e6,
            "ms_per_job": wall * 1e3 / args.steps,
            "step_kernel_ms": per_step_ms,
            "step_kernel_mlups": N * N / (per_step_ms * 1e-3) / 1e6,
            "steps_per_launch": lf["steps_per_launch"],
            "launch_ms": lf["launch_ms"],
            "achieved_gbs": lf["achieved_gbs"],
            "bytes_per_update": bpu,
            "cells": N * N,
            # throughput over the HBM bound of a one-step-per-launch kernel
            "over_one_step_roofline": N * N / (per_step_ms * 1e-3) / (HBM_PEAK_GBS * 1e9 / bpu),
            "tile": sim.tile,
            "band_rows": lbm.tile_layout(N, N, sim.tile, storage)[0],
            "kernel": kernel_name(lbm, sim.tile, storage),
            "metrics": {k: m[k] for k in ("W", "Gmax", "drho", "W_eff", "E_int", "mass", "finite")},
        }
        log(f"[{name}] {out[name]['mlups']:.0f} MLUPS whole job, step kernel {per_step_ms:.4f} ms "
            f"per time step, {lf['steps_per_launch']} per launch: {lf['achieved_gbs']:.0f} GB/s "
            f"({lf['achieved_gbs'] / HBM_PEAK_GBS:.3f} of peak)")
        sim.close()
        del rho, ux, uy
        torch.cuda.empty_cache()
    return out


def run_single_droplet(args, torch, lbm, inputs):
    """One droplet, R = 200, on a 1024^2 grid (G -5.0, tau 1.0), FP32, 10000 steps.
    A+B are 75.5 MB, so this run is served largely from the Infinity Cache."""
    n, steps = 1024, args.c2_steps
    sim = lbm.Simulation(n, n, -5.0, 1.0, lbm.LBM_F32)
    sim.init_droplets(inputs.single_droplet(n, 200), seed=1)
    if not args.no_autotune:
        sim.autotune(reps=8)
    stream = torch.cuda.current_stream()
    sim.step(100)
    sim.init_droplets(inputs.single_droplet(n, 200), seed=1)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    m = sim.metrics()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / steps
    lf = launch_figures(lbm, sim.tile, ms, BYTES_F32, n * n)
    res = {"workload": "single_droplet_1024", "steps": steps, "mlups": n * n * steps / wall / 1e6,
           "step_kernel_ms": ms, "step_kernel_mlups": n * n / (ms * 1e-3) / 1e6,
           "steps_per_launch": lf["steps_per_launch"], "launch_ms": lf["launch_ms"],
           "achieved_gbs": lf["achieved_gbs"], "tile": sim.tile,
           "band_rows": lbm.tile_layout(n, n, sim.tile, lbm.LBM_F32)[0],
           "kernel": kernel_name(lbm, sim.tile, lbm.LBM_F32),
           "metrics": {k: m[k] for k in ("W", "Gmax", "drho", "W_eff", "E_int", "mass", "finite")}}
    log(f"[single droplet 1024^2] {res['step_kernel_mlups']:.0f} MLUPS per launch, "
        f"{res['mlups']:.0f} MLUPS whole run")
    sim.close()
    torch.cuda.empty_cache()
    return res


def run_series_cost(args, torch, lbm, inputs):
    """Cost of the fused metric time series on the bench workload: 500 FP32 steps with
    the interface metrics of every 10th state, against 500 plain steps and against
    50 separate diagnostics passes."""
    N = args.n
    drops = inputs.many_droplets(N, args.drops, 8, 48, seed=3)
    sim = lbm.Simulation(N, N, args.G, args.tau, lbm.LBM_F32)
    sim.init_droplets(drops, seed=3)
    sim.step(20)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(500)
    torch.cuda.synchronize()
    plain = time.perf_counter() - t0
    t0 = time.perf_counter()
    recs = sim.step_series(500, 10)
    series = time.perf_counter() - t0
    t0 = time.perf_counter()
    for _ in range(50):
        sim.step(10)
        sim.metrics()
    separate = time.perf_counter() - t0
    sim.close()
    torch.cuda.empty_cache()
    res = {"workload": f"many_droplets_{N}", "steps": 500, "every": 10, "records": len(recs),
           "plain_ms": plain * 1e3, "series_ms": series * 1e3, "separate_passes_ms": separate * 1e3,
           "series_overhead": series / plain - 1.0, "separate_overhead": separate / plain - 1.0}
    log(f"[metric series] plain {plain*1e3:.1f} ms, fused series {series*1e3:.1f} ms, "
        f"separate passes {separate*1e3:.1f} ms")
    return res


def run_paper_preset(args, torch, lbm):
    """The paper's pure-LBM protocol (R = nx/6, G -5.5, tau 1.0; 500 steps, then five
    segments) on a 256^2 grid, with the FP16-shifted fork from the common state."""
    from paper_2504_10539_amd import preset
    t0 = time.perf_counter()
    r = preset.run(nx=256, segment=500, every=50, fork_storage=lbm.LBM_F16_SHIFTED, pinn_beta=0.5)
    torch.cuda.synchronize()
    res = {"workload": "paper_droplet_256", "steps": 500 + 5 * 500, "wall_s": time.perf_counter() - t0,
           "table_I": r["table_I"], "table_II": r["table_II"],
           "fp16_fork": {"table_I": r["fork"]["table_I"], "table_II": r["fork"]["table_II"]},
           "pinn_lbm": {"beta": r["pinn"]["beta"], "table_I": r["pinn"]["table_I"],
                        "table_II": r["pinn"]["table_II"]}}
    log(f"[paper preset 256^2] pure LBM: table I {res['table_I']}, table II {res['table_II']}; "
        f"PINN-LBM: table I {res['pinn_lbm']['table_I']}, table II {res['pinn_lbm']['table_II']}")
    return res


def run_one_step_reference(args, torch, lbm, inputs):
    """The best single-step FP32 shape on the same workload (strips of 512
    threads, 2 rows in flight, 64-row bands), timed over 200 steps: the HBM
    roofline fraction a kernel that reads and writes every population once per
    step reaches, beside the two-step kernel's."""
    N = args.n
    sim = lbm.Simulation(N, N, args.G, args.tau, lbm.LBM_F32)
    sim.init_droplets(inputs.many_droplets(N, args.drops, 8, 48, seed=3), seed=3)
    tile = next(t["id"] for t in lbm.tiles() if t["steps"] == 1 and not t["paired"]
                and t["threads"] == 512 and t["cells"] == 1 and t["prefetch"] == 2
                and t["rows"] == 64)
    sim.set_tile(tile)
    sim.step(20)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    sim.step(200)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 200
    sim.close()
    gbs = BYTES_F32 * N * N / (ms * 1e-3) / 1e9
    return {"kernel": kernel_name(lbm, tile, lbm.LBM_F32), "tile": tile,
            "launch_ms": round(ms, 5), "achieved": round(gbs, 1),
            "frac": round(gbs / HBM_PEAK_GBS, 4)}


# Matrix-core flops per cell of the PINN inference: the dense layers 2-4
# (64 x 128, 128 x 128 and 128 x 64 multiply-adds).
PINN_MFMA_FLOPS = 2 * (64 * 128 + 128 * 128 + 128 * 64)
FP16_MFMA_PEAK_TFLOPS = 2500.0


def run_pinn(args, torch, lbm, inputs):
    """The PINN surrogate (Sec. II-B/III-B network) on a grid of the bench size:
    inference at every cell (lbm_pinn_infer) and the Sec. II-C correction
    (lbm_pinn_correct, interface cells only) of the paper's droplet (Sec. III-A:
    R = nx / 6, G -5.5, tau 1.0) after --pinn-steps FP32 steps, timed with HIP
    events.  The network is first trained on the state's own fields (Sec. III-B:
    300 epochs, learning rate 3e-4, PyTorch on the GPU; not part of the timed
    path).  A single droplet is the workload the surrogate is made for: a
    smooth network cannot represent the 2000-droplet field."""
    from paper_2504_10539_amd import pinn
    N = args.n
    sim = lbm.Simulation(N, N, -5.5, 1.0, lbm.LBM_F32)
    sim.init_droplets(inputs.single_droplet(N, N / 6.0), seed=1)
    sim.step(args.pinn_steps)
    net = pinn.make_net(seed=0, device="cuda")
    t0 = time.perf_counter()
    hist = pinn.train(net, pinn.state_fields(sim), args.G, args.tau, epochs=args.pinn_epochs, seed=0)
    train_s = time.perf_counter() - t0
    params = pinn.pack(net)
    out = [torch.empty((N, N), dtype=torch.float32, device="cuda") for _ in range(3)]
    stream = torch.cuda.current_stream()

    def infer():
        lbm.LIB.lbm_pinn_infer(sim.handle, params.data_ptr(), *[o.data_ptr() for o in out])

    infer()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 5
    e0.record(stream)
    for _ in range(reps):
        infer()
    e1.record(stream)
    torch.cuda.synchronize()
    infer_ms = e0.elapsed_time(e1) / reps
    mask = torch.zeros(N * N, dtype=torch.uint8, device="cuda")
    sim.pinn_correct(params, 0.5, mask)
    torch.cuda.synchronize()
    corrected = int(mask.sum().item())
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record(stream)
    for _ in range(reps):
        sim.pinn_correct(params, 0.5)
    c1.record(stream)
    torch.cuda.synchronize()
    correct_ms = c0.elapsed_time(c1) / reps
    finite = sim.metrics()["finite"]
    sim.close()
    del out, mask
    torch.cuda.empty_cache()
    tflops = PINN_MFMA_FLOPS * N * N / (infer_ms * 1e-3) / 1e12
    res = {"workload": f"paper_droplet_{N}", "cells": N * N, "steps_before": args.pinn_steps,
           "infer_ms": infer_ms, "infer_mcells_per_s": N * N / (infer_ms * 1e-3) / 1e6,
           "mfma_flops_per_cell": PINN_MFMA_FLOPS, "mfma_tflops": tflops,
           "mfma_peak_tflops": FP16_MFMA_PEAK_TFLOPS, "mfma_frac": tflops / FP16_MFMA_PEAK_TFLOPS,
           "correct_ms": correct_ms, "corrected_cells": corrected,
           "corrected_fraction": corrected / (N * N), "finite_after": finite,
           "train_epochs": args.pinn_epochs, "train_s": train_s,
           "train_loss": [hist[0], hist[-1]],
           "kernel": "k_pinn<StoreF32, true>"}
    log(f"[pinn] inference {infer_ms:.2f} ms for {N}^2 cells ({tflops:.0f} TFLOP/s on the matrix "
        f"cores, {tflops / FP16_MFMA_PEAK_TFLOPS:.3f} of FP16 peak); correction {correct_ms:.2f} ms, "
        f"{corrected} interface cells")
    return res


def run_copy_reference(torch, lbm):
    n = 2 << 30
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        lbm.stream_copy(b, a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        lbm.stream_copy(b, a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 10
    del a, b
    torch.cuda.empty_cache()
    return 2 * n / (ms * 1e-3) / 1e9


def run_sweep(args, torch, lbm, inputs):
    """512 instances of 256^2 in one batched persistent launch per step."""
    pairs = inputs.sweep_grid(32, 16)[: args.sweep_instances]
    res = {}
    for storage, name in ((lbm.LBM_F32, "f32"), (lbm.LBM_F16_SHIFTED, "f16_shifted")):
        sims = []
        for k, (G, tau) in enumerate(pairs):
            s = lbm.Simulation(256, 256, G, tau, storage, 1.0 if storage else 0.0)
            s.init_droplets(inputs.single_droplet(256, 40), seed=k)
            sims.append(s)
        batch = lbm.Batch(sims, steps_per_graph=args.graph_steps)
        tile = batch.autotune(reps=5) if not args.no_autotune else -1
        batch.step(args.graph_steps)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record()
        batch.step(args.sweep_steps)
        e1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = e0.elapsed_time(e1)
        batch.close()
        unstable = sum(1 for s in sims if not s.metrics()["finite"])
        lu = 256.0 * 256 * len(sims) * args.sweep_steps
        bpu = BYTES_F32 if storage == lbm.LBM_F32 else BYTES_F16
        spl = lbm.tiles()[tile]["steps"] if tile >= 0 else 1
        # algorithmic bytes: each launch reads and writes every population once
        res[name] = {"mlups": lu / wall / 1e6, "gpu_mlups": lu / (ms * 1e-3) / 1e6,
                     "achieved_gbs": lu * bpu / spl / (ms * 1e-3) / 1e9, "steps_per_launch": spl,
                     "instances": len(sims), "steps": args.sweep_steps,
                     "unstable_instances": unstable, "tile": tile}
        log(f"[sweep {name}] {res[name]['gpu_mlups']:.0f} MLUPS, {unstable} unstable")
        for s in sims:
            s.close()
        del sims
        torch.cuda.empty_cache()
    return res


def serving_capacity(args, torch, lbm, inputs):
    """Closed-loop capacity of the continuous path, in requests per second: a
    calibration batch of the trace's distribution (seed 40) submitted at once,
    counted until 80% of it has completed (before the tail of the last long
    requests leaves the GPU part-idle)."""
    cal = inputs.serving_trace(args.serve_calib, rate=0.0, seed=40, nmax=args.serve_nmax,
                               smax=args.serve_smax)
    srv = lbm.Server(args.serve_pool_gb << 30, policy=lbm.LBM_POLICY_CONTINUOUS,
                     steps_per_tick=args.graph_steps, max_slots=256)
    t0 = srv.clock()
    for r in cal:
        srv.submit(r.n, r.n, r.G, r.tau, r.steps, r.drops, seed=r.seed, storage=args.serve_storage,
                   rho0=1.0 if args.serve_storage == lbm.LBM_F16_SHIFTED else 0.0)
    target = int(0.8 * len(cal))
    while srv.stats()["completed"] < target:
        time.sleep(0.01)
    secs = srv.clock() - t0
    srv.drain()
    srv.close()
    torch.cuda.empty_cache()
    cap = target / secs
    log(f"[serving] closed-loop capacity {cap:.1f} requests/s ({target} of {len(cal)} in {secs:.1f} s)")
    return cap


def run_serving(args, torch, lbm, inputs):
    """Poisson trace, continuous batching vs the plain one-at-a-time path.  The
    arrival rate is --serve-rate, or (default) 1.1x the continuous path's
    measured closed-loop capacity, so that the trace saturates the GPU."""
    capacity = None
    rate = args.serve_rate
    if rate <= 0:
        capacity = serving_capacity(args, torch, lbm, inputs)
        rate = 1.1 * capacity
    trace = inputs.serving_trace(args.serve_requests, rate=rate, seed=4,
                                 nmax=args.serve_nmax, smax=args.serve_smax)
    res = {"rate_req_s": rate, "capacity_req_s": capacity, "arrival_span_s": trace[-1].arrival}
    policies = ((lbm.LBM_POLICY_CONTINUOUS, "continuous"), (lbm.LBM_POLICY_FIFO, "fifo"))
    for policy, name in policies:
        if args.serve_policy not in ("both", name):
            continue
        srv = lbm.Server(args.serve_pool_gb << 30, policy=policy, steps_per_tick=args.graph_steps,
                         max_slots=256)
        t0 = srv.clock()
        tickets = []
        for r in trace:
            while srv.clock() - t0 < r.arrival:
                time.sleep(min(0.001, max(0.0, r.arrival - (srv.clock() - t0))))
            tickets.append(srv.submit(r.n, r.n, r.G, r.tau, r.steps, r.drops, seed=r.seed,
                                      storage=args.serve_storage,
                                      rho0=1.0 if args.serve_storage == lbm.LBM_F16_SHIFTED else 0.0))
            if len(tickets) % 250 == 0:
                log(f"[serving {name}] {len(tickets)} submitted, {srv.stats()['completed']} done")
        last = time.perf_counter()
        while srv.stats()["completed"] < len(tickets):
            time.sleep(0.05)
            if time.perf_counter() - last > 15.0:
                last = time.perf_counter()
                log(f"[serving {name}] {srv.stats()['completed']} of {len(tickets)} done")
        srv.drain()
        lat, lat_ok, done, unstable = [], [], [], 0
        for t in tickets:
            code, m = srv.poll(t)
            lat.append(m["t_done"] - m["t_submit"])
            if code == lbm.LBM_OK:
                lat_ok.append(lat[-1])
            done.append(m["t_done"])
            unstable += code != lbm.LBM_OK
        st = srv.stats()
        srv.close()
        lat.sort()
        lat_ok.sort()

        def pct(v, q):
            return 1e3 * v[min(len(v) - 1, max(0, int(math.ceil(q * len(v))) - 1))]

        makespan = max(done) - t0
        # Throughput counts the lattice updates of requests that completed
        # LBM_OK; unstable requests are retired early and their work is listed
        # apart.
        res[name] = {"requests": len(trace),
                     "storage": ["f32", "f16_shifted", "f16_cell", "f16_moment"][args.serve_storage],
                     "aggregate_mlups": st["lattice_updates"] / makespan / 1e6,
                     "p50_ms": pct(lat, 0.5), "p99_ms": pct(lat, 0.99),
                     "ok_p50_ms": pct(lat_ok, 0.5), "ok_p99_ms": pct(lat_ok, 0.99),
                     "makespan_s": makespan, "unstable": unstable,
                     "retired_early": st["retired_early"],
                     "unstable_mlu": st["unstable_updates"] / 1e6,
                     "ok_mlu": st["lattice_updates"] / 1e6,
                     "pool_high_water_gb": st["pool_high_water"] / 2**30}
        log(f"[serving {name}] {res[name]}")
        torch.cuda.empty_cache()
    return res


def run_cpu_baseline(args, inputs):
    """The FP64 oracle on the host cores.  `value`: all host threads on a bounded
    sample of the bench workload (a 512^2 window of the 4096^2 field, about
    --cpu-seconds of work).  `legs`: one thread and all threads on that window,
    on config 1 in full (64^2 droplet, 1000 steps) and on the 1024^2 droplet
    truncated to 200 steps (its MLUPS stands for the 10000-step run, an
    extrapolation)."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    threads = max(1, min(threads, os.cpu_count() or 1))
    n = 512
    drops = inputs.many_droplets(args.n, args.drops, 8, 48, seed=3)
    window = oracle.droplet_state(n, n, drops, seed=3, period=(args.n, args.n))

    def timed(f, G, tau, steps, th):
        t0 = time.perf_counter()
        oracle.step(f, G, tau, steps, th)
        return time.perf_counter() - t0

    def window_rate(th, secs):
        probe = timed(window, args.G, args.tau, 10, th)
        steps = max(10, int(10 * secs / max(probe, 1e-3)))
        dt = timed(window, args.G, args.tau, steps, th)
        return steps, dt

    steps, dt = window_rate(threads, args.cpu_seconds)
    legs = [{"workload": f"many_droplets_{args.n} window {n}^2", "threads": threads, "steps": steps,
             "seconds": dt, "mlups": n * n * steps / dt / 1e6}]
    s1, d1 = window_rate(1, args.cpu_seconds / 2)
    legs.append({"workload": f"many_droplets_{args.n} window {n}^2", "threads": 1, "steps": s1,
                 "seconds": d1, "mlups": n * n * s1 / d1 / 1e6})
    c1 = oracle.droplet_state(64, 64, inputs.single_droplet(64, 16), seed=1)
    c2 = oracle.droplet_state(1024, 1024, inputs.single_droplet(1024, 200), seed=1)
    for th in (1, threads):
        d = timed(c1, -5.0, 1.0, 1000, th)
        legs.append({"workload": "config1 64^2, 1000 steps (full)", "threads": th, "steps": 1000,
                     "seconds": d, "mlups": 64 * 64 * 1000 / d / 1e6})
        d = timed(c2, -5.0, 1.0, 200, th)
        legs.append({"workload": "single_droplet_1024, 200 of 10000 steps (rate extrapolated)",
                     "threads": th, "steps": 200, "seconds": d, "mlups": 1024 * 1024 * 200 / d / 1e6})
    for leg in legs:
        log(f"[cpu baseline] {leg['workload']}, {leg['threads']} threads: {leg['mlups']:.1f} MLUPS")
    return {"value": legs[0]["mlups"], "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"FP64 oracle, {n}x{n} window of the 4096^2 2000-droplet field, {steps} steps, "
                      f"{dt:.1f} s on {threads} host threads",
            "legs": legs}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3, help="timed bench steps (whole jobs)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--drops", type=int, default=2000)
    ap.add_argument("--G", type=float, default=-5.5)
    ap.add_argument("--tau", type=float, default=1.0)
    ap.add_argument("--lbm-steps", type=int, default=5000)
    ap.add_argument("--tile", type=int, default=-1, help="fixed tile shape (default: autotune)")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-fp16", action="store_true")
    ap.add_argument("--storages", default="",
                    help="comma-separated storage legs of the main workload to run "
                         "(f32, f16_shifted, f16_cell, f16_moment; default: all)")
    ap.add_argument("--no-extras", action="store_true", help="skip sweep, serving and CPU baseline")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--c2-steps", type=int, default=10000)
    ap.add_argument("--pinn-steps", type=int, default=500)
    ap.add_argument("--pinn-epochs", type=int, default=300)
    ap.add_argument("--only", choices=["single_droplet_1024", "serving", "pinn", "sweep"],
                    default=None,
                    help="run one extra workload alone and print its result (for profiling)")
    ap.add_argument("--graph-steps", type=int, default=30)
    ap.add_argument("--sweep-instances", type=int, default=512)
    ap.add_argument("--sweep-steps", type=int, default=4000)
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-rate", type=float, default=0.0,
                    help="arrivals per second (default 0: 1.1x the measured closed-loop capacity)")
    ap.add_argument("--serve-calib", type=int, default=400,
                    help="requests of the closed-loop capacity calibration")
    ap.add_argument("--serve-nmax", type=int, default=2048)
    ap.add_argument("--serve-smax", type=int, default=20000)
    ap.add_argument("--serve-pool-gb", type=int, default=32)
    ap.add_argument("--serve-policy", choices=["both", "continuous", "fifo"], default="both")
    ap.add_argument("--serve-storage", type=int, default=0, choices=[0, 1, 2, 3],
                    help="storage form of every request (0 FP32, 1 FP16-shifted, 2 FP16 per cell, "
                         "3 FP16 with exact moments)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(independent runs would be placed whole on separate GPUs; one large grid "
              "would split into y-slabs exchanging halo rows)", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    from paper_2504_10539_amd import inputs, lbm

    if args.only == "single_droplet_1024":
        print(json.dumps(run_single_droplet(args, torch, lbm, inputs)), flush=True)
        return
    if args.only == "serving":
        print(json.dumps(run_serving(args, torch, lbm, inputs)), flush=True)
        return
    if args.only == "pinn":
        print(json.dumps(run_pinn(args, torch, lbm, inputs)), flush=True)
        return
    if args.only == "sweep":
        print(json.dumps(run_sweep(args, torch, lbm, inputs)), flush=True)
        return
    log(f"device {torch.cuda.get_device_name(0)}; workload {args.n}^2, {args.drops} droplets, "
        f"G {args.G}, tau {args.tau}, {args.lbm_steps} LBM steps per job")
    main_res = run_main(args, torch, lbm, inputs)
    if "f32" not in main_res:  # a subset of the storage legs (--storages): their figures only
        print(json.dumps(main_res), flush=True)
        return
    f32 = main_res["f32"]
    khash = kernel_source_hash()
    copy_gbs = run_copy_reference(torch, lbm)
    one_step = run_one_step_reference(args, torch, lbm, inputs)
    traffic = traffic_from_profiles(lbm, khash, "f32", args.n, f32["tile"])
    line = {
        "metric": "MLUPS & % HBM roofline (FP32 vs FP16-shifted); batched p50/p99 latency",
        "value": round(f32["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(f32["ms_per_job"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"many_droplets_{args.n}", "grid": [args.n, args.n],
                   "droplets": args.drops, "radius": [8, 48], "G": args.G, "tau": args.tau,
                   "lbm_steps_per_step": args.lbm_steps, "storage": "f32",
                   "parallelism": "single_gpu"},
        "roofline": dict(roofline_bound(f32), **{
                     "traffic": traffic, "kernel": f32["kernel"],
                     "bytes_per_launch_per_cell": BYTES_F32,
                     "steps_per_launch": f32["steps_per_launch"],
                     "launch_ms": round(f32["launch_ms"], 5),
                     # per update instead of per launch: MLUPS x 72 B / 8 TB/s (above 1
                     # because a multi-step launch moves each population once per K updates)
                     "over_one_step_roofline": round(f32["over_one_step_roofline"], 4),
                     "frac_per_update": round(f32["over_one_step_roofline"], 4),
                     "one_step_kernel": one_step,
                     "copy_reference_gbs": round(copy_gbs, 1), "kernel_hash": khash}),
        "f32": f32,
    }
    for key in ("f16_shifted", "f16_cell", "f16_moment"):
        if key in main_res:
            r = main_res[key]
            line[key] = dict(r, roofline_frac=round(r["achieved_gbs"] / HBM_PEAK_GBS, 4),
                             traffic=traffic_from_profiles(lbm, khash, key, args.n, r["tile"]))
    if not args.no_extras:
        line["single_droplet_1024"] = run_single_droplet(args, torch, lbm, inputs)
        line["paper_preset"] = run_paper_preset(args, torch, lbm)
        line["metric_series"] = run_series_cost(args, torch, lbm, inputs)
        line["sweep_512x256"] = run_sweep(args, torch, lbm, inputs)
        line["pinn"] = run_pinn(args, torch, lbm, inputs)
        line["serving"] = run_serving(args, torch, lbm, inputs)
        if not args.no_cpu:
            line["cpu_baseline"] = run_cpu_baseline(args, inputs)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
