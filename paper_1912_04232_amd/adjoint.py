"""Minimized energies as a differentiable function of the pair parameters (paper Sec. 4.2, App. A).

The paper differentiates ``minimize_energy(diameter, key)`` by running reverse-mode autodiff through the
FIRE steps.  Here the forward pass minimizes every replica with one batched FIRE launch (``fire_batched``)
and the backward pass calls the hand-written parameter-gradient kernel (``envelope_grad``) at the minima
R*: at a converged minimum F(R*) = 0, so by the envelope theorem

    dE*/dtheta = dU/dtheta (R*; theta)        (positions held fixed),

which is the derivative the unrolled reverse pass converges to as max |F| -> 0.  Soft-sphere diameters
enter through sigma_ab = (d_a + d_b) / 2 (App. A), so dE*/dd_s = 1/2 sum_b (G_sb + G_bs) with
G_ab = dU/dsigma_ab per ordered species pair.  The box is held fixed while the diameters change.
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
        gs, ge, _ = md.envelope_grad(md_ctx, batch, pot)
        g = g_e.to(gs.device, torch.float64)
        # dE_b/dd_s = 1/2 sum_c (G_sc + G_cs)
        dEdd = 0.5 * (gs.sum(dim=2) + gs.sum(dim=1))          # [B][S]
        dEde = ge.sum(dim=(1, 2))                              # [B]
        grad_d = (g[:, None] * dEdd).sum(dim=0)
        grad_e = (g * dEde).sum()
        return grad_d.cpu(), grad_e.cpu(), None, None, None, None, None, None, None


def minimized_energy(diameters: torch.Tensor, epsilon: torch.Tensor, batch: "md.Batch", batch_u: torch.Tensor,
                     fp: "md.FireParams | None" = None, f_tol: float = 1e-6, max_steps: int = 200000,
                     md_ctx: "md.Context | None" = None, alpha: float = 2.0) -> torch.Tensor:
    """E*_b for every replica, differentiable w.r.t. the species diameters and epsilon (box fixed)."""
    return FireMinimizedEnergy.apply(diameters, epsilon, batch_u, batch, fp or md.FireParams(), f_tol, max_steps,
                                     md_ctx or md.Context(), alpha)
