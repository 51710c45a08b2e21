"""Constant-temperature dynamics, gradient descent and flocking, as a command.

    python -m paper_1912_04232_amd.simulate [--method langevin|langevin_fused|nose_hoover|brownian|gradient_descent|all|
                                             flocking]
                                            [--steps 1000] [--n-cells 40] [--boids 65536]

The integrators run on 3D Lennard-Jones, 4 n^3 particles on an FCC lattice at density 0.84 (N = 256000 for
n = 40), Maxwell velocities at T = 1, cutoff 2.5, skin 0.3.  Flocking (Sec. 4.3, App. B) runs the boid model with
its default parameters: boids uniform in a square box at density 0.25 with 16 disk obstacles, skin 0.5, and
optionally predators (App. B's two-player extension).  Each run
takes 100 steps (graph capture and warm-up), then `steps` timed steps replayed from HIP graphs of 20 steps (the
fused Langevin run, like NVE, is one launch per step with the list rebuilt inside the run); one JSON line per run.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import inputs, md

METHODS = {
    "langevin": ("BAOAB, gamma 1, kT 1, dt 0.005", lambda s, c: md.nvt_langevin(s, c["dt"], 1.0, 1.0, 1)),
    "langevin_fused": ("BAOAB fused into the step kernel, gamma 1, kT 1, dt 0.005",
                       lambda s, c: md.nvt_langevin(s, c["dt"], 1.0, 1.0, 1, fused=True)),
    "nose_hoover": ("chain Q = (100, 10), kT 1, dt 0.005",
                    lambda s, c: md.nvt_nose_hoover(s, c["dt"], 1.0, (100.0, 10.0))[:2]),
    "brownian": ("gamma 1, kT 1, dt 1e-4", lambda s, c: md.brownian(s, 1e-4, 1.0, 1.0, 1)),
    "gradient_descent": ("dt 1e-4", lambda s, c: md.gradient_descent(s, 1e-4)),
}


def run(ctx, method: str, steps: int = 1000, n_cells: int = 40) -> dict:
    c = inputs.lj_large(n_cells=n_cells)
    box = md.Box(tuple(c["L"]), 3)
    pot = md.Potential("lj", [[1.0]], [[1.0]], r_cut=c["r_cut"])
    what, make = METHODS[method]
    s = md.System(box, pot, c["u"], c["v"], skin=c["skin"], ctx=ctx)
    init, update = make(s, c)
    init()
    update(100, graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    update(steps, graph=True)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    inertial = method in ("langevin", "langevin_fused", "nose_hoover")
    return {"method": method, "scheme": what, "N": s.N, "steps": steps, "steps_per_s": steps / t,
            "us_per_step": 1e6 * t / steps,
            "kinetic_T": float((s.vel.double() ** 2).sum()) / (3 * s.N) if inertial else None}


def run_flocking(ctx, steps: int = 1000, N: int = 65536, n_obstacles: int = 16, seed: int = 29, skin: float = 0.5,
                 lanes: int = 4, predators: int = 0) -> dict:
    L = float(np.float32(np.sqrt(N / 0.25)))
    u, theta, obs = inputs.boids(N, L, seed, n_obstacles)
    pred = inputs.boids(predators, L, seed + 100, 0)[:2] if predators else None
    f = md.Flock(md.Box((L, L), 2), u, theta, None, obs, skin=skin, ctx=ctx, lanes=lanes, predators=pred)
    init, update = md.flocking(f)
    init()
    update(100, graph=True)
    torch.cuda.synchronize()
    f.nl.clear_flags()
    t0 = time.perf_counter()
    update(steps, graph=True)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    return {"method": "flocking", "N": f.N, "L": L, "obstacles": n_obstacles, "predators": predators, "skin": skin,
            "lanes": lanes,
            "steps": steps, "steps_per_s": steps / t, "boid_steps_per_s": f.N * steps / t,
            "us_per_step": 1e6 * t / steps, "mean_row": float(f.nl.lengths().mean()),
            "rebuilds_in_last_20_steps": int(f.last_flags[md.FLAG_REBUILDS])}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--method", choices=tuple(METHODS) + ("all", "flocking"), default="all")
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--n-cells", type=int, default=40)
    ap.add_argument("--boids", type=int, default=65536)
    ap.add_argument("--skin", type=float, default=0.5, help="flocking list skin")
    ap.add_argument("--lanes", type=int, default=4, help="GPU lanes per boid")
    ap.add_argument("--predators", type=int, default=0, help="flocking predators")
    a = ap.parse_args(argv)
    md.load()
    if not torch.cuda.is_available():
        sys.exit("no GPU visible")
    ctx = md.Context()
    if a.method == "flocking":
        print(json.dumps(run_flocking(ctx, a.steps, a.boids, skin=a.skin, lanes=a.lanes,
                                                 predators=a.predators)), flush=True)
        return
    for m in (METHODS if a.method == "all" else (a.method,)):
        print(json.dumps(run(ctx, m, a.steps, a.n_cells)), flush=True)


if __name__ == "__main__":
    main()
