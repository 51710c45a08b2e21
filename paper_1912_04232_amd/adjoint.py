"""Minimized energies as a differentiable function of the pair parameters (paper Sec. 4.2, App. A).

The paper differentiates ``minimize_energy(diameter, key)`` by running reverse-mode autodiff through the
FIRE steps.  Here the forward pass minimizes every replica with one batched FIRE launch (``fire_batched``)
and the backward pass calls the hand-written parameter-gradient kernel (``envelope_grad``) at the minima
R*: at a converged minimum F(R*) = 0, so by the envelope theorem

    dE*/dtheta = dU/dtheta (R*; theta)        (positions held fixed),

which is the derivative the unrolled reverse pass converges to as max |F| -> 0.  Soft-sphere diameters
enter through sigma_ab = (d_a + d_b) / 2 (App. A), so dE*/dd_s = 1/2 sum_b (G_sb + G_bs) with
G_ab = dU/dsigma_ab per ordered species pair.  The box is held fixed while the diameters change.  Every step of
this arithmetic (the chain rule, and the product with the upstream gradient in backward) runs in the library
(envelope_grad_wrt, md_diameter_grad); this module only sequences the calls.

``rescaled_box_sweep`` is the experiment of Sec. 4.2 with the box of App. A: half the disks have diameter D and
half diameter 1, and the box edge follows the packing fraction, L(D) ~ sqrt(D^2 + 1), so positions are fractional
and every distance scales with L.  At a minimum s* in fractional coordinates the envelope theorem gives

    dE*/dD = dU/dD (s*; D) = G_AA + (G_AB + G_BA)/2 - D/(D^2 + 1) * W,

where the last term is the box's: W = sum over pairs of -r du/dr.  The harmonic soft sphere depends on r/sigma
only, so W = sum_ab sigma_ab G_ab and the GPU's parameter-gradient sums give it with no further pass.

``unrolled_box_sweep`` is the same experiment the way App. A computes it: a fixed number of FIRE steps (300) from
each start, and the derivative of the final energy E_K through those steps (``fire_unrolled_grad``, reverse mode
through the loop).  Every diameter and every start is one replica of a single launch (the paper's two nested
vmaps), each with its own sigma matrix and box, and

    dE_K/dD = G_AA + (G_AB + G_BA)/2 + D/(D^2 + 1) * dE_K/dln c

with dE_K/dln c the derivative for the box scaled at fixed fractional start.  Unlike E*, E_K is not at a minimum
when K is too short to converge, so the two sweeps agree only where FIRE has converged.
"""
from __future__ import annotations

import numpy as np
import torch

from . import md


def sigma_from_diameters(d: np.ndarray) -> np.ndarray:
    d = np.asarray(d, dtype=np.float64)
    return 0.5 * (d[:, None] + d[None, :])


class FireMinimizedEnergy(torch.autograd.Function):
    """E*_b(d, eps) for every replica b of a batch: forward = batched FIRE, backward = envelope_grad."""

    @staticmethod
    def forward(ctx, diameters, epsilon, batch_u, batch, fp, f_tol, max_steps, md_ctx, alpha):
        d = diameters.detach().cpu().numpy().astype(np.float64)
        eps = float(epsilon.detach().cpu())
        S = d.shape[0]
        pot = md.Potential("soft_sphere", sigma_from_diameters(d), np.full((S, S), eps), alpha=alpha)
        batch.pos.copy_(batch_u)   # every evaluation starts from the same initial positions
        e, fmax, steps, status = md.fire_batched(md_ctx, batch, pot, fp, max_steps, f_tol)
        ctx.md = (md_ctx, batch, pot, S)
        ctx.pos_star = batch.pos.clone()
        ctx.info = dict(fmax=fmax.cpu().numpy(), steps=steps.cpu().numpy(), status=status.cpu().numpy())
        FireMinimizedEnergy.last_info = ctx.info
        return e.to(diameters.device)

    @staticmethod
    def backward(ctx, g_e):
        md_ctx, batch, pot, S = ctx.md
        batch.pos.copy_(ctx.pos_star)
        # the library forms sum_b g_b dE_b/dd_s and sum_b g_b dE_b/deps (chain rule and weighted sum on the device)
        w = g_e.to(batch.pos.device, torch.float64)
        grad_d = md.envelope_grad_wrt(md_ctx, batch, pot, md.WRT_DIAMETER, md.BOX_FIXED, weights=w)
        grad_e = md.envelope_grad_wrt(md_ctx, batch, pot, md.WRT_EPSILON_COMMON, md.BOX_FIXED, weights=w)
        return grad_d.cpu(), grad_e[0].cpu(), None, None, None, None, None, None, None


def minimized_energy(diameters: torch.Tensor, epsilon: torch.Tensor, batch: "md.Batch", batch_u: torch.Tensor,
                     fp: "md.FireParams | None" = None, f_tol: float = 1e-6, max_steps: int = 200000,
                     md_ctx: "md.Context | None" = None, alpha: float = 2.0) -> torch.Tensor:
    """E*_b for every replica, differentiable w.r.t. the species diameters and epsilon (box fixed)."""
    return FireMinimizedEnergy.apply(diameters, epsilon, batch_u, batch, fp or md.FireParams(), f_tol, max_steps,
                                     md_ctx or md.Context(), alpha)


def rescaled_box_sweep(md_ctx: "md.Context", diameters, starts, phi: float, fp: "md.FireParams | None" = None,
                       f_tol: float = 1e-6, max_steps: int = 200000, epsilon: float = 1.0, alpha: float = 2.0):
    """For every small-disk diameter D and every start (uint32 fractional positions [N][2], N even; the first N/2
    disks are the small ones): minimize with batched FIRE in the box of packing fraction phi, then return per D the
    minimized energies E*, dE*/dD with the box rescaled with D (see the module docstring), max |F|, the FIRE step
    counts and the status words, as numpy arrays [len(D)][len(starts)]; also the batches (minimized positions)."""
    from . import inputs
    fp = fp or md.FireParams()
    out = {k: [] for k in ("energy", "dEdD", "fmax", "steps", "status")}
    batches = []
    for D in diameters:
        D = float(D)
        reps = []
        for u in starts:
            N = int(u.shape[0])
            L = inputs.box_for_packing([D, 1.0], [N // 2, N - N // 2], phi, 2)
            reps.append(dict(N=N, L=[L, L, 0.0], u=u, species=inputs.bidisperse_species(N)))
        bt = md.Batch(reps)
        d = np.array([D, 1.0])
        sig = sigma_from_diameters(d)
        pot = md.Potential("soft_sphere", sig, np.full((2, 2), float(epsilon)), alpha=alpha)
        e, fmax, steps, status = md.fire_batched(md_ctx, bt, pot, fp, max_steps, f_tol)
        g = md.envelope_grad_wrt(md_ctx, bt, pot, md.WRT_DIAMETER, md.BOX_PACKING)   # [B][2]: species 0 has D
        out["energy"].append(e.cpu().numpy())
        out["dEdD"].append(g[:, 0].cpu().numpy())
        out["fmax"].append(fmax.cpu().numpy())
        out["steps"].append(steps.cpu().numpy())
        out["status"].append(status.cpu().numpy())
        batches.append(bt)
    return {k: np.array(v) for k, v in out.items()}, batches



def unrolled_box_batch(diameters, starts, phi: float, epsilon: float = 1.0, alpha: float = 2.0):
    """(Batch, Potential, sigma [B][2][2]) for the rescaled-box sweep: replica (D, start) in D-major order, box of
    packing fraction phi at diameters (D, 1), species 0 = the first N/2 disks (diameter D)."""
    from . import inputs
    reps, sig = [], []
    for D in diameters:
        D = float(D)
        for u in starts:
            N = int(u.shape[0])
            L = inputs.box_for_packing([D, 1.0], [N // 2, N - N // 2], phi, 2)
            reps.append(dict(N=N, L=[L, L, 0.0], u=u, species=inputs.bidisperse_species(N)))
            sig.append(sigma_from_diameters([D, 1.0]))
    pot = md.Potential("soft_sphere", sigma_from_diameters([1.0, 1.0]), np.full((2, 2), float(epsilon)), alpha=alpha)
    return md.Batch(reps), pot, np.array(sig)


def unrolled_box_grad(md_ctx: "md.Context", bt: "md.Batch", pot: "md.Potential", sig, diameters, n_starts: int, res):
    """dE_K/dD [len(D)][n_starts] from a fire_unrolled_grad result on an unrolled_box_batch: the library's chain rule
    (md_diameter_grad) with each replica's sigma and its box derivative g_lnc; D is species 0's diameter."""
    g = md.diameter_grad(md_ctx, bt, pot, res["g_sigma"], dln=res["g_lnc"], box=md.BOX_PACKING, sigma=sig)
    return g[:, 0].cpu().numpy().reshape(len(diameters), n_starts)


def unrolled_box_sweep(md_ctx: "md.Context", diameters, starts, phi: float, K: int = 300,
                       fp: "md.FireParams | None" = None, epsilon: float = 1.0, alpha: float = 2.0, workspace=None):
    """E_K and dE_K/dD after K FIRE steps for every small-disk diameter D and every start (uint32 fractional
    positions [N][2], N even, the first N/2 disks small), box at packing fraction phi rescaled with D, all in one
    launch.  Returns (dict of numpy arrays [len(D)][len(starts)]: energy, dEdD, g_lnc, status; the raw result
    of fire_unrolled_grad, whose "workspace" can be passed back in to reuse the trajectory buffer)."""
    bt, pot, sig = unrolled_box_batch(diameters, starts, phi, epsilon, alpha)
    res = md.fire_unrolled_grad(md_ctx, bt, pot, fp or md.FireParams(), K, workspace=workspace, sigma=sig)
    nD, ns = len(diameters), len(starts)
    out = {"energy": res["energy"].cpu().numpy().reshape(nD, ns),
           "dEdD": unrolled_box_grad(md_ctx, bt, pot, sig, diameters, ns, res),
           "g_lnc": res["g_lnc"].cpu().numpy().reshape(nD, ns),
           "status": res["status"].cpu().numpy().reshape(nD, ns)}
    return out, res
