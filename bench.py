"""Benchmark: Lennard-Jones NVE steps/s and pair evaluations/s at N = 256000 on one MI355X.

Workload (lj_large): 3D LJ, FCC 4*40^3 = 256000 particles at reduced density 0.84, Maxwell velocities at
T = 1 (net momentum zero), cutoff 2.5 sigma (energy shifted), skin 0.3, velocity Verlet with dt = 0.005.
One step = one fused launch: neighbor-list rebuild on the device when a particle has moved more than skin/2
(cell binning + list build), then forces over the list, kick and drift.  The timed region holds exactly
--steps steps, rebuilds included, with all data resident in HBM.

    python bench.py [--steps 10000] [--warmup 100] [--gpus 1] [--no-cpu-baseline]

Prints one JSON line (see the keys below).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KERNEL_SRC = os.path.join(ROOT, "paper_1912_04232_amd", "csrc", "md_core.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "verlet_step_lj256k_traffic.json")


def kernel_sha() -> str:
    h = hashlib.sha256()
    for f in (KERNEL_SRC, os.path.join(ROOT, "paper_1912_04232_amd", "csrc", "md_device.h")):
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per k_verlet_step launch from the committed rocprofv3 counter runs, if they match this kernel."""
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha") != kernel_sha():
        return None
    return float(t["fetch_bytes_per_launch"]) + float(t["write_bytes_per_launch"])


def cpu_baseline(cfg, seconds: float):
    """The FP64 oracle on the host's cores: one brute-force force evaluation (the cost of one oracle step) timed
    on a sample of rows, scaled to steps/s of the full system."""
    import numpy as np

    import oracle
    threads = oracle.default_threads()
    x = oracle.decode(cfg["u"], cfg["L"])
    pot = oracle.Potential("lj", np.ones((1, 1)), np.ones((1, 1)), r_cut=cfg["r_cut"])
    N = cfg["N"]
    rng = np.random.default_rng(0)
    m = 256
    t = 0.0
    while True:
        rows = rng.choice(N, m, replace=False)
        t0 = time.perf_counter()
        oracle.pair_rows(x, cfg["L"], pot, rows=rows, nthreads=threads)
        t = time.perf_counter() - t0
        if t > seconds / 4 or m >= N:
            break
        m = min(N, int(m * max(2.0, seconds / max(t, 1e-3) / 2)))
    sec_per_step = t * N / m
    return {"value": 1.0 / sec_per_step, "unit": "steps/s", "cores": threads, "kind": "oracle",
            "sample": f"brute-force FP64 forces of {m} of {N} particles (each against all N) in {t:.1f} s, "
                      f"scaled by N/{m} to one step"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--n-cells", type=int, default=40, help="FCC cells per edge (N = 4 n^3)")
    ap.add_argument("--lanes", type=int, default=None, help="GPU lanes per particle (default: chosen from the list size)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    def progress(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    progress("importing torch")
    import numpy as np
    import torch

    from paper_1912_04232_amd import inputs, md

    torch.cuda.set_device(0)
    progress("generating the FCC workload")
    cfg = inputs.lj_large(n_cells=args.n_cells)
    N = cfg["N"]
    box = md.Box(tuple(cfg["L"]), 3)
    pot = md.Potential("lj", [[1.0]], [[1.0]], r_cut=cfg["r_cut"])
    s = md.System(box, pot, cfg["u"], cfg["v"], skin=cfg["skin"], lanes=args.lanes)
    init, update = md.nve(s, cfg["dt"])
    init()
    E_init = s.potential_energy() + s.kinetic_energy()
    progress(f"initial list built (capacity {s.nl.capacity}, bins of {s.nl.max_per_cell}); warming up")
    if args.warmup:
        update(args.warmup)
    progress(f"timing {args.steps} steps")
    E0 = s.potential_energy() + s.kinetic_energy()
    s.nl.clear_flags()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    md.verlet_step(s.ctx, s.box, s.pot, s.pos, s.vel, s.force, s.species, s.nl, cfg["dt"], args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    flags = s.nl.read_flags()
    if (flags[md.FLAG_OVERFLOW] or flags[md.FLAG_CELL_OVERFLOW] or flags[md.FLAG_STALE]
            or flags[md.FLAG_NONFINITE] or flags[md.FLAG_STEPS] != args.steps):
        raise SystemExit(f"timed run invalid: flags {flags.tolist()}")
    E1 = s.potential_energy() + s.kinetic_energy()
    counts = s.nl.lengths().astype(np.int64)
    mean_n = float(counts.mean())
    sec = wall
    steps_per_s = args.steps / sec
    pair_evals = mean_n * N * steps_per_s
    # dominant kernel: one k_verlet_step launch per step; its algorithmic bytes with the implemented layout:
    # own position read 12 B, velocity read+write 24 B, new position write 12 B, reference position read 12 B,
    # row length 4 B, and 4 B per list entry; neighbor positions are gathers served by cache.
    bytes_per_launch = N * (12 + 24 + 12 + 12 + 4) + 4.0 * float(counts.sum())
    kernel_s = gpu_ms * 1e-3 / args.steps
    achieved = bytes_per_launch / kernel_s / 1e9
    traffic = measured_traffic()
    out = {
        "metric": "LJ MD steps/s & pair-evals/s at N=256k; surrogate vs plain at stated force RMSE",
        "value": round(steps_per_s, 2),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1000.0 * sec / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"lj_large: 3D Lennard-Jones FCC N={N} rho=0.84 T=1 rc=2.5 skin=0.3 dt=0.005 NVE",
                   "N": N, "dt": cfg["dt"], "r_cut": cfg["r_cut"], "skin": cfg["skin"],
                   "positions": "uint32 torus coordinates", "lanes_per_particle": s.nl.lanes,
                   "parallelism": "single GPU"},
        "extra": {
            "pair_evals_per_s": pair_evals,
            "mean_list_entries": mean_n,
            "rebuilds_in_timed_region": int(flags[md.FLAG_REBUILDS]),
            "energy_drift_per_particle": (E1 - E0) / N,
            "energy_drift_from_start_per_particle": (E1 - E_init) / N,
            "gpu_event_ms": gpu_ms,
            "wall_s": wall,
        },
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": "k_verlet_step<3,0,false>",
                     "bytes_per_launch": bytes_per_launch, "avg_launch_us": kernel_s * 1e6},
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        progress("timing the oracle on the host")
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
