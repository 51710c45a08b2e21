"""The small-disk-diameter sweep of Sec. 4.2 / App. A on one GPU, as a command.

    python -m paper_1912_04232_amd.sweep [--method unrolled|envelope] [--K 300] [--phi 1.0] [--starts 100]
                                         [--launches 3] [--breakdown]

128 disks, half of diameter D and half of diameter 1, box rescaled with D at packing fraction phi, `starts` random
starts per D for D = 0.50, 0.55, ..., 1.20.  `unrolled` runs K FIRE steps from every start and differentiates the
final energy through the steps (every (D, start) pair one replica of a single launch); `envelope` minimizes every
replica to max |F| < 1e-7 and takes dE*/dD at the minima.  Prints one JSON line: timings and, per D, the mean and
spread of E and of dE/dD (mean, standard error, median, 10 %-trimmed mean).  `--breakdown` (unrolled) also
compares the samples far from their D's median with typical ones, from the trajectory the launch recorded: the
largest FIRE mixing factor alpha |v| / |F|, the smallest and the final |F|, the P <= 0 restarts, and the pairs that
cross contact (r = sigma) between consecutive recorded states.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import adjoint, inputs, md

DIAMETERS = np.round(np.arange(0.5, 1.2001, 0.05), 2)


def _stats(E, G, Ds):
    q = np.sort(G, axis=1)
    cut = max(1, int(round(0.1 * q.shape[1])))
    mE = E.mean(axis=1)
    mG = G.mean(axis=1)
    med = np.median(G, axis=1)
    trim = q[:, cut:-cut].mean(axis=1) if q.shape[1] > 2 * cut else mG
    k_max = int(np.argmax(mE))

    def crossing(v):
        k = next((k for k in range(1, len(Ds)) if v[k - 1] > 0 >= v[k]), None)
        return None if k is None else float(Ds[k])

    se = G.std(axis=1) / np.sqrt(G.shape[1])
    k1 = int(np.argmin(np.abs(Ds - 1.0)))
    return {"D": Ds.tolist(), "mean_E": mE.tolist(), "std_E": E.std(axis=1).tolist(), "mean_dEdD": mG.tolist(),
            "stderr_dEdD": se.tolist(), "median_dEdD": med.tolist(),
            "trimmed_mean_dEdD": trim.tolist(), "D_energy_max": float(Ds[k_max]),
            "D_zero_crossing_mean": crossing(mG), "D_zero_crossing_median": crossing(med),
            "D_zero_crossing_trimmed": crossing(trim),
            "dEdD_positive_below_energy_max": bool((mG[:k_max] > 0).all()),
            "median_dEdD_positive_below_energy_max": bool((med[:k_max] > 0).all()),
            "dEdD_at_D1_within_2_stderr": bool(abs(mG[k1]) <= 2 * se[k1])}


def run_unrolled(ctx, K: int = 300, phi: float = 1.0, n_starts: int = 100, launches: int = 3, Ds=DIAMETERS,
                 with_breakdown: bool = False):
    """One launch over every (D, start), then `launches` more timed with HIP events on the launch stream."""
    starts = inputs.rescaled_box_starts(count=n_starts)
    bt, pot, sig = adjoint.unrolled_box_batch(Ds, starts, phi)
    u0 = bt.pos.clone()
    res = md.fire_unrolled_grad(ctx, bt, pot, md.FireParams(), K, sigma=sig)
    G = adjoint.unrolled_box_grad(ctx, bt, pot, sig, Ds, n_starts, res)
    E = res["energy"].cpu().numpy().reshape(len(Ds), n_starts)
    done = int((res["status"].cpu().numpy() == 1).sum())
    t = None
    if launches > 0:
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(launches):
            bt.pos.copy_(u0)
            md.fire_unrolled_grad(ctx, bt, pot, md.FireParams(), K, sigma=sig, workspace=res["workspace"])
        ev1.record()
        torch.cuda.synchronize()
        t = ev0.elapsed_time(ev1) / 1e3 / launches
    n = np.asarray(bt.sizes, dtype=np.float64)
    pairs = float((n * (n - 1)).sum()) * (2 * K + 3)   # K+1 force passes forward; energy and K+1 adjoint passes
    out = {"method": "unrolled", "N": int(n.max()), "K": K, "packing_fraction": phi, "starts_per_D": n_starts,
           "replicas_in_one_launch": int(bt.B), "done": done, "workspace_bytes": int(res["workspace"].numel())}
    if t is not None:
        out.update({"seconds_per_launch": t, "replica_steps_per_s": bt.B * K / t, "pair_evals_per_s": pairs / t})
    out.update(_stats(E, G, np.asarray(Ds)))
    if with_breakdown:
        # every launch from u0 records the same trajectory (the kernel is deterministic): the workspace holds it
        out["breakdown"] = breakdown(bt, sig, res, G, K)
    return out


def _rank_corr(a, b) -> float:
    ra, rb = np.argsort(np.argsort(a)), np.argsort(np.argsort(b))
    return float(np.corrcoef(ra, rb)[0, 1])


def breakdown(bt, sig, res, G, K: int, per_kind: int = 12, far: float = 20.0, seed: int = 0) -> dict:
    """Samples of dE_K/dD [len(D)][starts] more than `far` median absolute deviations from their D's median against
    the rest, from the trajectory fire_unrolled_grad recorded: per replica the step records (dt, alpha, |v|, |F'|,
    P > 0) of every step, and for `per_kind` replicas of each kind the states, to count pairs crossing r = sigma."""
    B, n = bt.B, np.asarray(bt.sizes)
    ws = res["workspace"]
    rec = ws[: B * K * 5 * 8].view(torch.float64).reshape(B, K, 5).cpu().numpy()
    al, vn, fn, mix = rec[..., 1], rec[..., 2], rec[..., 3], rec[..., 4]
    cf = np.where(mix > 0, al * vn / np.maximum(fn, 1e-300), 0.0)   # v' = (1 - alpha) v + cf F after step k
    g = G.ravel()
    med = np.repeat(np.median(G, axis=1), G.shape[1])
    dev = np.abs(g - med)
    mad = np.repeat(np.median(np.abs(G - np.median(G, axis=1, keepdims=True)), axis=1), G.shape[1])
    far_mask = dev > far * np.maximum(mad, 1e-3)
    part_base = (B * K * 5 * 8 + 255) // 256 * 256
    off = np.concatenate([[0], np.cumsum(n)])
    boxes = np.asarray(bt.boxes, dtype=np.float64)

    def contact_changes(b):
        # state k of replica b: positions uint32 [nb][2], then forces and velocities (24 nb bytes per state)
        nb, base = int(n[b]), part_base + 24 * (K + 1) * int(off[b])
        L = boxes[b][:2]
        sp = np.array([0] * (nb // 2) + [1] * (nb - nb // 2))
        S = np.asarray(sig[b])[sp[:, None], sp[None, :]]
        iu = np.triu_indices(nb, 1)
        u = ws[base: base + 24 * nb * (K + 1)].view(torch.int32).cpu().numpy().view(np.uint32)
        prev, changes = None, np.zeros(K, dtype=np.int64)
        for k in range(K + 1):
            x = u[6 * nb * k: 6 * nb * k + 2 * nb].reshape(nb, 2).astype(np.float64) * (L / 2.0 ** 32)
            d = x[:, None, :] - x[None, :, :]
            d -= L * np.round(d / L)
            c = (np.sqrt((d ** 2).sum(-1)) < S)[iu]
            if prev is not None:
                changes[k - 1] = int((c != prev).sum())
            prev = c
        return changes

    rng = np.random.default_rng(seed)
    picks = {"far": [int(b) for b in np.argsort(-dev)[:per_kind]],
             "typical": [int(b) for b in rng.choice(np.where(~far_mask)[0], per_kind, replace=False)]}
    kinds = {}
    for kind, lst in picks.items():
        ch = [contact_changes(b) for b in lst]
        kinds[kind] = {"replicas": len(lst), "median_abs_dEdD": float(np.median(np.abs(g[lst]))),
                       "median_max_mixing_factor": float(np.median(cf[lst].max(1))),
                       "median_min_F": float(np.median(fn[lst].min(1))),
                       "median_final_F": float(np.median(fn[lst, -1])),
                       "median_restarts": float(np.median((mix[lst] == 0).sum(1))),
                       "median_contact_changes": float(np.median([c.sum() for c in ch])),
                       "median_contact_changes_last100": float(np.median([c[-100:].sum() for c in ch]))}
    return {"far_samples": int(far_mask.sum()), "samples": int(g.size), "far_threshold_mad": far,
            "far_per_D": far_mask.reshape(G.shape[0], -1).sum(1).tolist(), "kinds": kinds,
            "rank_corr_with_deviation": {"max_mixing_factor": _rank_corr(dev, cf.max(1)),
                                         "final_F": _rank_corr(dev, fn[:, -1]), "min_F": _rank_corr(dev, fn.min(1)),
                                         "restarts": _rank_corr(dev, (mix == 0).sum(1))}}


def run_envelope(ctx, phi: float = 1.0, n_starts: int = 100, f_tol: float = 1e-7, Ds=DIAMETERS):
    starts = inputs.rescaled_box_starts(count=n_starts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res, _ = adjoint.rescaled_box_sweep(ctx, Ds, starts, phi, f_tol=f_tol)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    out = {"method": "envelope", "N": 128, "packing_fraction": phi, "starts_per_D": n_starts,
           "converged": int((res["status"] == 1).sum()), "replicas": int(res["status"].size), "seconds": t,
           "particle_steps_per_s": float(res["steps"].sum()) * 128 / t}
    out.update(_stats(res["energy"], res["dEdD"], np.asarray(Ds)))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--method", choices=("unrolled", "envelope"), default="unrolled")
    ap.add_argument("--K", type=int, default=300)
    ap.add_argument("--phi", type=float, default=1.0)
    ap.add_argument("--starts", type=int, default=100)
    ap.add_argument("--launches", type=int, default=3)
    ap.add_argument("--breakdown", action="store_true", help="unrolled: where the far-off dE/dD samples come from")
    a = ap.parse_args(argv)
    md.load()
    if not torch.cuda.is_available():
        sys.exit("no GPU visible")
    ctx = md.Context()
    if a.method == "unrolled":
        out = run_unrolled(ctx, a.K, a.phi, a.starts, a.launches, with_breakdown=a.breakdown)
    else:
        out = run_envelope(ctx, a.phi, a.starts)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
