"""Constant-temperature dynamics and gradient descent, in float64 (paper Sec. 3.3.1: the Nose-Hoover, Langevin
and Brownian simulations and the gradient-descent minimizer that sit beside NVE and FIRE).

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and ``bench.py``'s ``cpu_baseline`` leg, never by the
product package.  It shares no code with the HIP path.

The paper names these integrators without giving their discretizations; the ones written out here are
published schemes (unit masses, positions x, velocities v, forces F = -grad U from md_oracle.c):

* Langevin: BAOAB (Leimkuhler and Matthews, Appl. Math. Res. Express 2013):
      v += dt/2 F;  x += dt/2 v;  v = c1 v + c2 xi;  x += dt/2 v;  F = F(x);  v += dt/2 F
  with c1 = exp(-gamma dt), c2 = sqrt((1 - c1^2) kT).
* Brownian (overdamped Langevin, Euler-Maruyama):  x += (dt / gamma) F + sqrt(2 kT dt / gamma) xi.
* Gradient descent:  x += dt F.
* Nose-Hoover chain (Martyna, Klein and Tuckerman 1992, the reference the paper cites), integrated with the
  half-step chain update of Martyna, Tuckerman, Tobias and Klein (Mol. Phys. 1996) around velocity Verlet:
      chain(dt/2);  v += dt/2 F;  x += dt v;  F = F(x);  v += dt/2 F;  chain(dt/2)
  for M thermostats with masses Q_k, momenta p_k = Q_k xi_k and positions eta_k; the conserved quantity is
      H' = K + U + sum_k p_k^2 / (2 Q_k) + n_f kT eta_1 + kT sum_{k>1} eta_k.

Noise: xi for particle i at step s comes from the counter-based generator Philox4x64-10 (Salmon, Moraes, Dror
and Shaw, SC'11) with counter (i, s, 0, 0) and key (seed, 0).  Its four 64-bit words give four uniforms
u_k = (floor(w_k / 2^40) + 1/2) / 2^24 (24-bit, exact in float32), and Box-Muller turns (u0, u1) and (u2, u3)
into four standard normals, of which the first `dim` are used.
"""
from __future__ import annotations

import math

import numpy as np

from . import Potential, pair_rows

_M0, _M1 = 0xD2E7470EE14C6C93, 0xCA5A826395121157     # Philox4x64 multipliers
_W0, _W1 = 0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B     # key increments (golden ratio, sqrt(3) - 1)
_MASK = (1 << 64) - 1


def philox4x64(counter, key, rounds: int = 10):
    """Philox4x64 of one 4-word counter and 2-word key (Python integers): the published round function."""
    c = [int(x) & _MASK for x in counter]
    k = [int(x) & _MASK for x in key]
    for _ in range(rounds):
        p0 = _M0 * c[0]
        p1 = _M1 * c[2]
        c = [(p1 >> 64) ^ c[1] ^ k[0], p1 & _MASK, (p0 >> 64) ^ c[3] ^ k[1], p0 & _MASK]
        k = [(k[0] + _W0) & _MASK, (k[1] + _W1) & _MASK]
    return c


def normals(N: int, dim: int, seed: int, step: int) -> np.ndarray:
    """xi [N][dim]: standard normals of every particle at one step (see the module docstring)."""
    out = np.zeros((N, dim))
    for i in range(N):
        w = philox4x64((i, step, 0, 0), (seed, 0))
        u = [((x >> 40) + 0.5) / 16777216.0 for x in w]
        r0 = math.sqrt(-2.0 * math.log(u[0]))
        r1 = math.sqrt(-2.0 * math.log(u[2]))
        z = (r0 * math.cos(2.0 * math.pi * u[1]), r0 * math.sin(2.0 * math.pi * u[1]),
             r1 * math.cos(2.0 * math.pi * u[3]), r1 * math.sin(2.0 * math.pi * u[3]))
        out[i] = z[:dim]
    return out


def _wrap(x, L):
    return x - L * np.floor(x / L)


def _forces(x, L, pot, species):
    F, e, _ = pair_rows(x, L, pot, species)
    return F, math.fsum(e.tolist())


def langevin_baoab(x, v, F, L, pot: Potential, species, dt: float, gamma: float, kT: float, seed: int, step0: int,
                   n_steps: int):
    """n_steps of BAOAB from (x, v, F = F(x)); noise of step s = step0, step0 + 1, ...  Returns (x, v, F)."""
    Lv = np.asarray(L, dtype=np.float64)[: x.shape[1]]
    x, v, F = (np.array(a, dtype=np.float64) for a in (x, v, F))
    c1 = math.exp(-gamma * dt)
    c2 = math.sqrt((1.0 - c1 * c1) * kT)
    for s in range(step0, step0 + n_steps):
        v = v + 0.5 * dt * F
        x = x + 0.5 * dt * v
        v = c1 * v + c2 * normals(x.shape[0], x.shape[1], seed, s)
        x = _wrap(x + 0.5 * dt * v, Lv)
        F, _ = _forces(x, Lv, pot, species)
        v = v + 0.5 * dt * F
    return x, v, F


def brownian(x, F, L, pot: Potential, species, dt: float, gamma: float, kT: float, seed: int, step0: int,
             n_steps: int):
    """n_steps of overdamped Langevin (Euler-Maruyama) from (x, F = F(x)).  Returns (x, F)."""
    Lv = np.asarray(L, dtype=np.float64)[: x.shape[1]]
    x, F = np.array(x, dtype=np.float64), np.array(F, dtype=np.float64)
    a = math.sqrt(2.0 * kT * dt / gamma)
    for s in range(step0, step0 + n_steps):
        xi = normals(x.shape[0], x.shape[1], seed, s) if kT > 0.0 else 0.0
        x = _wrap(x + (dt / gamma) * F + a * xi, Lv)
        F, _ = _forces(x, Lv, pot, species)
    return x, F


def gradient_descent(x, F, L, pot: Potential, species, dt: float, n_steps: int):
    """n_steps of x += dt F from (x, F = F(x)).  Returns (x, F, U)."""
    Lv = np.asarray(L, dtype=np.float64)[: x.shape[1]]
    x, F = np.array(x, dtype=np.float64), np.array(F, dtype=np.float64)
    U = None
    for _ in range(n_steps):
        x = _wrap(x + dt * F, Lv)
        F, U = _forces(x, Lv, pot, species)
    return x, F, U


def nhc_half(v, p, eta, Q, kT: float, n_f: int, h: float):
    """The chain's update over time h (= dt/2), Martyna-Tuckerman-Tobias-Klein 1996, one Suzuki-Yoshida stage:
    thermostat forces G_1 = (2K - n_f kT), G_k = p_{k-1}^2 / Q_{k-1} - kT; momenta from the last thermostat down
    (each scaled by exp(-h/4 p_{k+1}/Q_{k+1}) on both sides of its h/2 kick), positions eta += h p / Q, the
    particle velocities scaled by exp(-h p_1 / Q_1), then momenta back up the chain.  Returns (v, p, eta)."""
    v = np.array(v, dtype=np.float64)
    p = np.array(p, dtype=np.float64)
    eta = np.array(eta, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    M = p.shape[0]
    K2 = float((v * v).sum())                     # 2K

    def G(k, K2):
        return (K2 - n_f * kT) if k == 0 else (p[k - 1] ** 2 / Q[k - 1] - kT)

    p[M - 1] += 0.5 * h * G(M - 1, K2)
    for k in range(M - 2, -1, -1):
        f = math.exp(-0.25 * h * p[k + 1] / Q[k + 1])
        p[k] = (p[k] * f + 0.5 * h * G(k, K2)) * f
    eta += h * p / Q
    s = math.exp(-h * p[0] / Q[0])
    v *= s
    K2 *= s * s
    for k in range(M - 1):
        f = math.exp(-0.25 * h * p[k + 1] / Q[k + 1])
        p[k] = (p[k] * f + 0.5 * h * G(k, K2)) * f
    p[M - 1] += 0.5 * h * G(M - 1, K2)
    return v, p, eta


def nose_hoover(x, v, F, L, pot: Potential, species, dt: float, kT: float, Q, n_steps: int, p=None, eta=None):
    """n_steps of the Nose-Hoover chain from (x, v, F = F(x)); n_f = N dim.  Returns (x, v, F, p, eta, H')
    with H' the conserved quantity after the last step."""
    Lv = np.asarray(L, dtype=np.float64)[: x.shape[1]]
    x, v, F = (np.array(a, dtype=np.float64) for a in (x, v, F))
    Q = np.asarray(Q, dtype=np.float64)
    M = Q.shape[0]
    p = np.zeros(M) if p is None else np.array(p, dtype=np.float64)
    eta = np.zeros(M) if eta is None else np.array(eta, dtype=np.float64)
    n_f = x.size
    U = None
    for _ in range(n_steps):
        v, p, eta = nhc_half(v, p, eta, Q, kT, n_f, 0.5 * dt)
        v = v + 0.5 * dt * F
        x = _wrap(x + dt * v, Lv)
        F, U = _forces(x, Lv, pot, species)
        v = v + 0.5 * dt * F
        v, p, eta = nhc_half(v, p, eta, Q, kT, n_f, 0.5 * dt)
    if U is None:
        _, U = _forces(x, Lv, pot, species)
    H = 0.5 * float((v * v).sum()) + U + float((p * p / (2.0 * Q)).sum()) + n_f * kT * eta[0] + kT * eta[1:].sum()
    return x, v, F, p, eta, H
