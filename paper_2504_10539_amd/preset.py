"""The paper's pure-LBM droplet protocol on the GPU path.

Set-up (Sec. III-A): a square periodic nx x nx lattice, tau = 1.0,
G = -5.5, one droplet of radius nx / 6 at the centre.  The stated density
ratio "2.0" is read as rho_l = 2.0 inside and rho_g = 0.15 outside (the
pseudopotential coexistence pair at G = -5.5 is 2.31 / 0.105, so a
literal 2:1 ratio would not be a stable droplet); tanh width 2 and noise
1e-3 as in every other workload here.

Protocol (Sec. III-C), pure-LBM branch:

1. initialisation: 500 steps, the interface metrics recorded every `every`
   steps (the series of the initialisation figure: W, G_max, drho);
2. evolution: five segments of `segment` steps each (the paper does not give
   their length), the metrics recorded every `every` steps within them and
   at the end of each;
3. evaluation: the final metrics laid out as Tables I (W, G_max, drho) and
   II (W_eff, E_int).

`fork_storage` additionally forks the state after initialisation into a
second run with another storage form (lbm_get_state / lbm_set_state) and
takes it through the same evolution, the paper's compare-from-a-common-state
pattern applied to precision.

`pinn_beta` adds the PINN-LBM branch of the protocol, forked from the same
initialised state: before each evolution segment the network of Sec. III-B
is trained (PyTorch, learning rate 3e-4) on the branch's current state for
300, 240, 180, 120 and 60 epochs (the "decreasing training epochs" of
Sec. III-C), and the state is corrected at its interface cells on the GPU
(lbm_pinn_correct, blending factor pinn_beta); its final metrics fill the
second column of Tables I and II.

    python -m paper_2504_10539_amd.preset --nx 256 --segment 500
"""
from __future__ import annotations

import argparse
import json

from . import inputs, lbm

G_PAPER = -5.5
TAU_PAPER = 1.0
INIT_STEPS = 500
SEGMENTS = 5

TABLE_I = ("W", "Gmax", "drho")
TABLE_II = ("W_eff", "E_int")


def _brief(m: dict) -> dict:
    return {k: m[k] for k in ("step", "W", "Gmax", "drho", "W_eff", "E_int", "mass", "finite")}


def _evolve(sim, segment: int, every: int) -> tuple[list, list]:
    series, ends = [], []
    for _ in range(SEGMENTS):
        series += [_brief(m) for m in sim.step_series(segment, every)]
        ends.append(_brief(sim.metrics()))
    return series, ends


PINN_EPOCHS = (300, 240, 180, 120, 60)


def _evolve_pinn(sim, segment: int, every: int, beta: float, seed: int) -> tuple[list, list]:
    from . import pinn
    net = pinn.make_net(seed=seed, device=sim.device)
    series, ends = [], []
    for ep in PINN_EPOCHS:
        pinn.train(net, pinn.state_fields(sim), G_PAPER, TAU_PAPER, epochs=ep, seed=seed)
        sim.pinn_correct(pinn.pack(net), beta)
        series += [_brief(m) for m in sim.step_series(segment, every)]
        ends.append(_brief(sim.metrics()))
    return series, ends


def run(nx: int = 256, segment: int = 500, every: int = 10, storage: int = None,
        rho0: float = 1.0, seed: int = 1, fork_storage: int | None = None,
        pinn_beta: float | None = None) -> dict:
    """Runs the protocol; returns the series, the segment ends and the tables."""
    storage = lbm.LBM_F32 if storage is None else storage
    drops = inputs.single_droplet(nx, nx / 6.0)
    sim = lbm.Simulation(nx, nx, G_PAPER, TAU_PAPER, storage, rho0)
    sim.init_droplets(drops, seed=seed)
    out = {"nx": nx, "G": G_PAPER, "tau": TAU_PAPER, "radius": nx / 6.0, "segment": segment,
           "every": every, "storage": storage, "seed": seed}
    out["init_series"] = [_brief(m) for m in sim.step_series(INIT_STEPS, every)]
    out["after_init"] = _brief(sim.metrics())
    fork = None
    if fork_storage is not None:
        fork = lbm.Simulation(nx, nx, G_PAPER, TAU_PAPER, fork_storage, rho0)
        fork.set_state(sim.get_state())
    coupled = None
    if pinn_beta is not None:
        coupled = lbm.Simulation(nx, nx, G_PAPER, TAU_PAPER, storage, rho0)
        coupled.set_state(sim.get_state())
    out["evolution_series"], out["segment_ends"] = _evolve(sim, segment, every)
    final = out["segment_ends"][-1]
    out["table_I"] = {k: final[k] for k in TABLE_I}
    out["table_II"] = {k: final[k] for k in TABLE_II}
    if fork is not None:
        series, ends = _evolve(fork, segment, every)
        out["fork"] = {"storage": fork_storage, "segment_ends": ends,
                       "table_I": {k: ends[-1][k] for k in TABLE_I},
                       "table_II": {k: ends[-1][k] for k in TABLE_II}}
        fork.close()
    if coupled is not None:
        series, ends = _evolve_pinn(coupled, segment, every, pinn_beta, seed)
        out["pinn"] = {"beta": pinn_beta, "epochs": list(PINN_EPOCHS), "segment_ends": ends,
                       "table_I": {k: ends[-1][k] for k in TABLE_I},
                       "table_II": {k: ends[-1][k] for k in TABLE_II}}
        coupled.close()
    sim.close()
    return out


def main() -> None:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--nx", type=int, default=256)
    ap.add_argument("--segment", type=int, default=500)
    ap.add_argument("--every", type=int, default=10)
    ap.add_argument("--fp16", action="store_true", help="run with FP16-shifted storage")
    ap.add_argument("--fork-fp16", action="store_true",
                    help="also fork the initialised state into FP16-shifted storage")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--pinn-beta", type=float, default=None,
                    help="also run the PINN-LBM branch with this blending factor")
    a = ap.parse_args()
    r = run(a.nx, a.segment, a.every, lbm.LBM_F16_SHIFTED if a.fp16 else lbm.LBM_F32, seed=a.seed,
            fork_storage=lbm.LBM_F16_SHIFTED if a.fork_fp16 else None, pinn_beta=a.pinn_beta)
    print(json.dumps(r))


if __name__ == "__main__":
    main()
