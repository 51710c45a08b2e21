"""The flocking energy model of App. B (Sec. 4.3), in float64, by brute force over all pairs.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, never by the product package.  It shares no code with the HIP
path.

Boids have positions R_i in a periodic 2D box and headings theta_i, N_i = (cos theta_i, sin theta_i).  With the
cutoff function of App. B, rho(r; Rc) = (1/alpha)(1 - r/Rc)^alpha for r < Rc (else 0), the energy is
    E = E_align + E_avoid + E_cohesion + E_obstacle
    E_align    = 1/2 sum_{i != j} J_align rho(r_ij; R_align) (1 - N_i . N_j)^2     (position gradient stopped)
    E_avoid    = 1/2 sum_{i != j} J_avoid rho(r_ij; R_avoid)
    E_cohesion = sum_i 1/2 J_coh (1 - hat(dR_i) . N_i)^2,  dR_i = mean over j with r_ij < R_coh of (R_j - R_i)
    E_obstacle = sum_i sum_o J_obs rho(|R_i - C_o|; D_o) (1 - N_i . hat(R_i - C_o))^2
and one step of the dynamics is forward Euler,
    R_i' = R_i + dt (v N_i - dE/dR_i),   theta_i' = theta_i - dt dE/dtheta_i.
Readings (the printed forms disagree with the behavior the text describes): dR_i points from the boid to its
neighbors' center of mass, and the obstacle term vanishes when the boid faces away from the obstacle; the
obstacle's range is its radius D_o.  Displacements are nearest images.
Predators (the two-player extension of App. B) follow at the end of the file.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class FlockParams:
    J_align: float = 1.0
    R_align: float = 3.0
    J_avoid: float = 25.0
    R_avoid: float = 1.0
    J_coh: float = 0.05
    R_coh: float = 3.0
    J_obs: float = 10.0
    alpha: float = 3.0
    v: float = 1.0
    dt: float = 0.05


def rho(r, Rc, alpha):
    t = np.clip(1.0 - r / Rc, 0.0, None)
    return np.where(r < Rc, t ** alpha / alpha, 0.0)


def drho(r, Rc, alpha):
    t = np.clip(1.0 - r / Rc, 0.0, None)
    return np.where(r < Rc, -(t ** (alpha - 1.0)) / Rc, 0.0)


def _disp(R, L):
    d = R[:, None, :] - R[None, :, :]          # d[i, j] = R_i - R_j
    d -= L * np.round(d / L)
    r = np.sqrt((d * d).sum(-1))
    np.fill_diagonal(r, np.inf)
    return d, r


def energy_terms(R, theta, L, p: FlockParams, centers=None, radii=None):
    """(E_align, E_avoid, E_cohesion, E_obstacle)."""
    L = np.asarray(L, dtype=np.float64)
    d, r = _disp(R, L)
    N = np.stack([np.cos(theta), np.sin(theta)], 1)
    c = N @ N.T
    e_al = 0.5 * (p.J_align * rho(r, p.R_align, p.alpha) * (1.0 - c) ** 2).sum()
    e_av = 0.5 * (p.J_avoid * rho(r, p.R_avoid, p.alpha)).sum()
    m = r < p.R_coh
    n = m.sum(1)
    dR = -(d * m[..., None]).sum(1) / np.maximum(n, 1)[:, None]
    dn = np.sqrt((dR * dR).sum(1))
    ok = (n > 0) & (dn > 0)
    ch = np.where(ok, (dR * N).sum(1) / np.where(ok, dn, 1.0), 1.0)
    e_co = (0.5 * p.J_coh * (1.0 - ch) ** 2 * ok).sum()
    e_ob = 0.0
    if centers is not None:
        for C, D in zip(np.asarray(centers, np.float64), np.asarray(radii, np.float64)):
            x = R - C
            x -= L * np.round(x / L)
            ro = np.sqrt((x * x).sum(1))
            xh = x / np.where(ro > 0, ro, 1.0)[:, None]
            e_ob += (p.J_obs * rho(ro, D, p.alpha) * (1.0 - (N * xh).sum(1)) ** 2).sum()
    return e_al, e_av, e_co, e_ob


def gradients(R, theta, L, p: FlockParams, centers=None, radii=None):
    """(dE/dR [N,2] without the alignment term's position part, dE/dtheta [N])."""
    L = np.asarray(L, dtype=np.float64)
    d, r = _disp(R, L)
    rr = np.where(np.isfinite(r), r, 1.0)
    rh = d / rr[..., None]
    N = np.stack([np.cos(theta), np.sin(theta)], 1)
    Np = np.stack([-np.sin(theta), np.cos(theta)], 1)
    gR = (p.J_avoid * drho(r, p.R_avoid, p.alpha))[..., None] * rh
    gR = gR.sum(1)
    dth = theta[:, None] - theta[None, :]
    c = np.cos(dth)
    gT = (p.J_align * rho(r, p.R_align, p.alpha) * 2.0 * (1.0 - c) * np.sin(dth)).sum(1)
    # cohesion: e_i(dR_i), dR_i = (1/n_i) sum_j (R_j - R_i); dE/dR_k = -g_k + sum_{i: k in N_i} g_i / n_i
    m = r < p.R_coh
    n = m.sum(1)
    dR = -(d * m[..., None]).sum(1) / np.maximum(n, 1)[:, None]
    dn = np.sqrt((dR * dR).sum(1))
    ok = (n > 0) & (dn > 0)
    dh = dR / np.where(ok, dn, 1.0)[:, None]
    ci = (dh * N).sum(1)
    g = np.where(ok[:, None], -p.J_coh * (1.0 - ci)[:, None] * (N - ci[:, None] * dh) / np.where(ok, dn, 1.0)[:, None],
                 0.0)
    gT += np.where(ok, -p.J_coh * (1.0 - ci) * (dh * Np).sum(1), 0.0)
    gn = g / np.maximum(n, 1)[:, None]
    gR += -g + (m[..., None] * gn[None, :, :]).sum(1)
    if centers is not None:
        for C, D in zip(np.asarray(centers, np.float64), np.asarray(radii, np.float64)):
            x = R - C
            x -= L * np.round(x / L)
            ro = np.sqrt((x * x).sum(1))
            xh = x / np.where(ro > 0, ro, 1.0)[:, None]
            a = (N * xh).sum(1)
            w = rho(ro, D, p.alpha)
            dw = drho(ro, D, p.alpha)
            dadR = (N - a[:, None] * xh) / np.where(ro > 0, ro, 1.0)[:, None]
            gR += p.J_obs * (dw[:, None] * xh * ((1.0 - a) ** 2)[:, None] - (w * 2.0 * (1.0 - a))[:, None] * dadR)
            gT += p.J_obs * w * 2.0 * (1.0 - a) * (-(Np * xh).sum(1))
    return gR, gT


def step(R, theta, L, p: FlockParams, centers=None, radii=None, n_steps: int = 1):
    """n_steps of the forward-Euler dynamics.  Returns (R, theta)."""
    L = np.asarray(L, dtype=np.float64)
    R = np.array(R, dtype=np.float64)
    theta = np.array(theta, dtype=np.float64)
    for _ in range(n_steps):
        gR, gT = gradients(R, theta, L, p, centers, radii)
        N = np.stack([np.cos(theta), np.sin(theta)], 1)
        R = R + p.dt * (p.v * N - gR)
        R -= L * np.floor(R / L)
        theta = theta - p.dt * gT
    return R, theta


# ----------------------------------------------------------------------------------------------- predators
# App. B adds predators, each with a position and a heading, and makes the simulation a two-player game: boids
# minimize E_boid = (the four terms above) + E_boid-predator, predators minimize E_predator = E_predator-boid +
# E_obstacle.  The boid-predator term is the obstacle term with the predator in the obstacle's place (range
# R_flee, strength J_flee); the predator-boid term is the cohesion term of a predator over the boids within
# R_chase (strength J_chase).  Each side takes the forward-Euler step of its own energy in its own variables
# (predators at speed v_pred); both steps start from the same state.  The predators' occasional sprint is not
# modeled (the text gives no rule for it).

@dataclass
class PredatorParams:
    J_flee: float = 10.0
    R_flee: float = 4.0
    J_chase: float = 1.0
    R_chase: float = 8.0
    v: float = 1.2


def _wrap(x, L):
    return x - L * np.round(x / L)


def _facing_term(X, N, C, D, J, alpha, L):
    """sum_i J rho(|X_i - C|; D)(1 - N_i . hat(X_i - C))^2 and its gradients in X_i and in the heading angle."""
    x = _wrap(X - C, L)
    ro = np.sqrt((x * x).sum(1))
    xh = x / np.where(ro > 0, ro, 1.0)[:, None]
    a = (N * xh).sum(1)
    w = rho(ro, D, alpha)
    dw = drho(ro, D, alpha)
    Np = np.stack([-N[:, 1], N[:, 0]], 1)
    e = (J * w * (1.0 - a) ** 2).sum()
    dadX = (N - a[:, None] * xh) / np.where(ro > 0, ro, 1.0)[:, None]
    gX = J * (dw[:, None] * xh * ((1.0 - a) ** 2)[:, None] - (w * 2.0 * (1.0 - a))[:, None] * dadX)
    gT = J * w * 2.0 * (1.0 - a) * (-(Np * xh).sum(1))
    return e, gX, gT


def predator_terms(R, theta, Rp, thp, L, p: FlockParams, q: PredatorParams, centers=None, radii=None):
    """(E_boid-predator, E_predator-boid, E_obstacle of the predators)."""
    L = np.asarray(L, dtype=np.float64)
    N = np.stack([np.cos(theta), np.sin(theta)], 1)
    Np_ = np.stack([np.cos(thp), np.sin(thp)], 1)
    e_flee = sum(_facing_term(R, N, c, q.R_flee, q.J_flee, p.alpha, L)[0] for c in Rp)
    e_chase = 0.0
    for k in range(len(Rp)):
        d = _wrap(R - Rp[k], L)                       # R_j - R_p
        m = (d * d).sum(1) < q.R_chase ** 2
        if m.any():
            dR = d[m].mean(0)
            dn = math.sqrt((dR * dR).sum())
            if dn > 0:
                e_chase += 0.5 * q.J_chase * (1.0 - (dR / dn) @ Np_[k]) ** 2
    e_obs = 0.0
    if centers is not None:
        for C, D in zip(np.asarray(centers, np.float64), np.asarray(radii, np.float64)):
            e_obs += _facing_term(Rp, Np_, C, D, p.J_obs, p.alpha, L)[0]
    return e_flee, e_chase, e_obs


def predator_gradients(R, theta, Rp, thp, L, p: FlockParams, q: PredatorParams, centers=None, radii=None):
    """Gradients of each side's own energy in its own variables: (dE_boid-predator/dR [N,2], d/dtheta [N],
    dE_predator/dR_p [P,2], d/dtheta_p [P])."""
    L = np.asarray(L, dtype=np.float64)
    N = np.stack([np.cos(theta), np.sin(theta)], 1)
    gR, gT = np.zeros_like(R), np.zeros_like(theta)
    for c in Rp:
        _, a, b = _facing_term(R, N, c, q.R_flee, q.J_flee, p.alpha, L)
        gR += a
        gT += b
    Np_ = np.stack([np.cos(thp), np.sin(thp)], 1)
    gRp, gTp = np.zeros_like(Rp), np.zeros_like(thp)
    for k in range(len(Rp)):
        d = _wrap(R - Rp[k], L)
        m = (d * d).sum(1) < q.R_chase ** 2
        if not m.any():
            continue
        dR = d[m].mean(0)
        dn = math.sqrt((dR * dR).sum())
        if dn == 0:
            continue
        h = dR / dn
        c = h @ Np_[k]
        g = -q.J_chase * (1.0 - c) * (Np_[k] - c * h) / dn      # dE/d(dR)
        gRp[k] += -g                                           # dR moves by -dR_p
        gTp[k] += -q.J_chase * (1.0 - c) * (h @ np.array([-Np_[k, 1], Np_[k, 0]]))
    if centers is not None:
        for C, D in zip(np.asarray(centers, np.float64), np.asarray(radii, np.float64)):
            _, a, b = _facing_term(Rp, Np_, C, D, p.J_obs, p.alpha, L)
            gRp += a
            gTp += b
    return gR, gT, gRp, gTp


def step_with_predators(R, theta, Rp, thp, L, p: FlockParams, q: PredatorParams, centers=None, radii=None,
                        n_steps: int = 1):
    """n_steps of the two-player forward-Euler dynamics.  Returns (R, theta, Rp, thp)."""
    L = np.asarray(L, dtype=np.float64)
    R, theta = np.array(R, dtype=np.float64), np.array(theta, dtype=np.float64)
    Rp, thp = np.array(Rp, dtype=np.float64), np.array(thp, dtype=np.float64)
    for _ in range(n_steps):
        gR, gT = gradients(R, theta, L, p, centers, radii)
        fR, fT, gRp, gTp = predator_gradients(R, theta, Rp, thp, L, p, q, centers, radii)
        N = np.stack([np.cos(theta), np.sin(theta)], 1)
        Np_ = np.stack([np.cos(thp), np.sin(thp)], 1)
        R = R + p.dt * (p.v * N - gR - fR)
        theta = theta - p.dt * (gT + fT)
        Rp = Rp + p.dt * (q.v * Np_ - gRp)
        thp = thp - p.dt * gTp
        R -= L * np.floor(R / L)
        Rp -= L * np.floor(Rp / L)
    return R, theta, Rp, thp
