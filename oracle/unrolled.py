"""Reverse mode through a fixed number of FIRE steps, in float64 (paper Sec. 4.2 and App. A).

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and ``bench.py``'s ``cpu_baseline`` leg, never by the
product package.  It shares no code with the HIP path.

App. A minimizes a bidisperse soft-disk packing by running FIRE for a fixed number of steps on positions
stored as fractional coordinates R in the unit square (the box maps them to x = L R, so the box size is a
parameter of the energy), and differentiates the final energy with respect to the small-disk diameter by
reverse-mode automatic differentiation through the loop of steps.  This module writes that derivative out by
hand:

* ``fire_fixed_steps`` records the forward recurrence: the FIRE step of ``md_oracle.c`` (velocity and force in
  real units, real time step), with the drift applied to R as (dt V + dt^2/2 F) / L;
* ``fire_unrolled_grad`` transposes each step in reverse order (chain rule).  The only pair sums it needs
  are the Jacobian of the force applied to a vector (``force_jvp``, minus a Hessian-vector product) and the
  derivative of the force with respect to the pair parameters and the box scale, contracted with a vector
  (``force_param_vjp``).

Parameters: sigma_ab and eps_ab as independent entries of the ordered species matrices (the derivative with
respect to a symmetric entry is the (a,b) plus the (b,a) value), and ln c for a box scaled as L -> c L at fixed
fractional initial positions and fixed time parameters (the rescaled box of App. A).  Branch decisions of FIRE
(P > 0, the dt / alpha schedule) are piecewise constant in the parameters and are held fixed, as automatic
differentiation of the loop does.

All pair sums are brute force over every ordered pair (i, j), i != j, with the nearest-image displacement
d_ij = x_i - x_j - L round((x_i - x_j) / L); r = |d|, rhat = d / r.  For a pair potential u(r):
    F_i         = -sum_j u'(r) rhat_ij
    dF_i/dx_i   = -sum_j K_ij,   dF_i/dx_j = K_ij,   K = u'' rhat rhat^T + (u'/r)(I - rhat rhat^T)
    dF_i/dln c  = -sum_j u''(r) r rhat_ij        (every distance scales with the box at fixed R)
"""
from __future__ import annotations

import math

import numpy as np

from . import FireParams, Potential, decode, pair_rows, param_grad


def _pairs(R, L):
    """Real nearest-image displacements d[i, j] = x_i - x_j and distances for all ordered pairs (diagonal r=inf)."""
    Lv = np.asarray(L, dtype=np.float64)[: R.shape[1]]
    x = R * Lv
    d = x[:, None, :] - x[None, :, :]
    d -= Lv * np.round(d / Lv)
    r = np.sqrt((d * d).sum(-1))
    np.fill_diagonal(r, np.inf)
    return d, r


def _pair_table(pot: Potential, species, N):
    sp = np.zeros(N, dtype=np.int64) if species is None else np.asarray(species, dtype=np.int64)
    sig = np.atleast_2d(np.asarray(pot.sigma, dtype=np.float64))
    eps = np.atleast_2d(np.asarray(pot.epsilon, dtype=np.float64))
    return sp, sig[sp[:, None], sp[None, :]], eps[sp[:, None], sp[None, :]]


def pair_derivatives(pot: Potential, r, sig, eps):
    """u, u' = du/dr, u'' = d2u/dr2, du/dsigma, du'/dsigma for arrays of distances (0 outside the cutoff).

    Soft sphere (Sec. 3.3.2): u = eps/alpha t^alpha with t = 1 - r/sigma for r < sigma.
        u'  = -(eps/sigma) t^(alpha-1)            u'' = (eps/sigma^2)(alpha-1) t^(alpha-2)
        du/dsigma  = eps t^(alpha-1) r / sigma^2  du'/dsigma = (eps/sigma^2) t^(alpha-2) (t - (alpha-1) r/sigma)
    Lennard-Jones: u = 4 eps (q^2 - q) - u(r_c) with q = (sigma/r)^6 for r < r_c.
        u'  = -(4 eps / r)(12 q^2 - 6 q)          u'' = (4 eps / r^2)(156 q^2 - 42 q)
        du/dsigma  = (4 eps / sigma)(12 q^2 - 6 q) minus the same at r_c when shifted
        du'/dsigma = -(4 eps / (r sigma))(144 q^2 - 36 q)
    Derivatives in eps are u / eps and u' / eps.  The force discontinuity at the cutoff is not differentiated.
    """
    z = np.zeros_like(r)
    if pot.kind == "soft_sphere":
        a = float(pot.alpha)
        inside = r < sig
        t = np.where(inside, 1.0 - np.where(inside, r, 0.0) / sig, 0.0)
        u = np.where(inside, eps / a * t ** a, 0.0)
        u1 = np.where(inside, -(eps / sig) * t ** (a - 1.0), 0.0)
        with np.errstate(divide="ignore", invalid="ignore"):
            ta2 = np.where(inside, t ** (a - 2.0), 0.0)
        u2 = np.where(inside, eps / sig ** 2 * (a - 1.0) * ta2, 0.0)
        us = np.where(inside, eps * t ** (a - 1.0) * np.where(inside, r, 0.0) / sig ** 2, 0.0)
        u1s = np.where(inside, eps / sig ** 2 * ta2 * (t - (a - 1.0) * np.where(inside, r, 0.0) / sig), 0.0)
        return u, u1, u2, us, u1s
    rc = float(pot.r_cut)
    inside = r < rc
    rr = np.where(inside, r, 1.0)
    q = (sig / rr) ** 6
    u = 4.0 * eps * (q * q - q)
    us = 4.0 * eps / sig * (12.0 * q * q - 6.0 * q)
    if pot.shift:
        qc = (sig / rc) ** 6
        u = u - 4.0 * eps * (qc * qc - qc)
        us = us - 4.0 * eps / sig * (12.0 * qc * qc - 6.0 * qc)
    u1 = -(4.0 * eps / rr) * (12.0 * q * q - 6.0 * q)
    u2 = 4.0 * eps / rr ** 2 * (156.0 * q * q - 42.0 * q)
    u1s = -(4.0 * eps / (rr * sig)) * (144.0 * q * q - 36.0 * q)
    return tuple(np.where(inside, a_, z) for a_ in (u, u1, u2, us, u1s))


def forces(R, L, pot: Potential, species=None):
    """F(x) at x = L R, from the brute-force pair sum of md_oracle.c."""
    Lv = np.asarray(L, dtype=np.float64)[: R.shape[1]]
    F, _, _ = pair_rows(R * Lv, Lv, pot, species)
    return F


def _pair_state(R, L, pot, species):
    N = R.shape[0]
    sp, sig, eps = _pair_table(pot, species, N)
    d, r = _pairs(R, L)
    u, u1, u2, us, u1s = pair_derivatives(pot, r, sig, eps)
    with np.errstate(invalid="ignore", divide="ignore"):
        rhat = np.where(np.isfinite(r)[..., None], d / r[..., None], 0.0)
    rr = np.where(np.isfinite(r), r, 0.0)
    return sp, eps, rr, rhat, u1, u2, u1s


def force_jvp(R, L, pot: Potential, species, z):
    """(dF/dx) z at x = L R: (dF/dx z)_i = -sum_j K_ij (z_i - z_j), minus the Hessian of U applied to z."""
    _, _, rr, rhat, u1, u2, _ = _pair_state(R, L, pot, species)
    dz = z[:, None, :] - z[None, :, :]
    with np.errstate(invalid="ignore", divide="ignore"):
        a = np.where(rr > 0, u1 / np.where(rr > 0, rr, 1.0), 0.0)
    s = (rhat * dz).sum(-1)
    Kdz = a[..., None] * dz + ((u2 - a) * s)[..., None] * rhat
    return -Kdz.sum(1)


def force_param_vjp(R, L, pot: Potential, species, z):
    """z . dF/dtheta at x = L R for theta = every sigma_ab, every eps_ab (ordered entries) and ln c.

    With ordered entries, a pair (i, j) of species (a, b) feels the mean of the (a,b) and (b,a) entries, so it
    contributes -1/2 du'/dsigma rhat_ij . (z_i - z_j) to entry (a, b) (and likewise u'/eps for eps); the box
    scale contributes -1/2 u'' r rhat_ij . (z_i - z_j).
    """
    sp, eps, rr, rhat, u1, u2, u1s = _pair_state(R, L, pot, species)
    dz = z[:, None, :] - z[None, :, :]
    s = (rhat * dz).sum(-1)
    S = np.atleast_2d(pot.sigma).shape[0]
    gs = np.zeros((S, S))
    ge = np.zeros((S, S))
    for a_ in range(S):
        for b_ in range(S):
            m = (sp[:, None] == a_) & (sp[None, :] == b_)
            gs[a_, b_] = -0.5 * (u1s * s)[m].sum()
            ge[a_, b_] = -0.5 * (u1 / eps * s)[m].sum()
    return gs, ge, -0.5 * (u2 * rr * s).sum()


def energy_grads(R, L, pot: Potential, species=None):
    """(U, dU/dsigma_ab, dU/deps_ab, dU/dln c) at fixed fractional positions.

    dU/dln c = sum over pairs of r u'(r) = -W with W = sum_i w_i the pair virial of md_oracle.c.
    """
    Lv = np.asarray(L, dtype=np.float64)[: R.shape[1]]
    x = R * Lv
    _, e, w = pair_rows(x, Lv, pot, species)
    gs, ge = param_grad(x, Lv, pot, species)
    return math.fsum(e.tolist()), gs, ge, -math.fsum(w.tolist())


def fire_fixed_steps(R0, L, pot: Potential, species=None, K: int = 300, params: FireParams | None = None):
    """K FIRE steps (App. A) on positions kept as fractional coordinates, recording what the reverse pass needs.

    One step, unit masses, F = F(L R) (the rules of md_oracle.c's orc_fire with no convergence test):
        R'   = wrap(R + (dt V + dt^2/2 F) / L)
        F'   = F(L R')
        w    = V + dt/2 (F + F')
        P = F' . w,  vn = |w|,  fn = |F'|
        P > 0: V' = (1 - a) w + a vn F'/fn; n_pos += 1; n_pos > n_min: dt = min(f_inc dt, dt_max), a *= f_alpha
        else : V' = 0; dt *= f_dec; a = alpha_start; n_pos = 0
    Returns dict with R [K+1,N,dim], F [K+1,N,dim], w [K,N,dim], drift [K,N,dim] (the increment of R before
    wrapping), dt [K], alpha [K], mixed [K] (P > 0), vn [K], fn [K], and the final velocity V.
    """
    p = params or FireParams()
    R = np.array(R0, dtype=np.float64) % 1.0
    N, dim = R.shape
    Lv = np.asarray(L, dtype=np.float64)[:dim]
    F = forces(R, L, pot, species)
    V = np.zeros_like(R)
    dt, a, n_pos = float(p.dt_start), float(p.alpha_start), 0
    rec = {k: [] for k in ("R", "F", "w", "drift", "dt", "alpha", "mixed", "vn", "fn")}
    rec["R"].append(R.copy())
    rec["F"].append(F.copy())
    for _ in range(K):
        drift = (dt * V + 0.5 * dt * dt * F) / Lv
        Rn = (R + drift) % 1.0
        Fn = forces(Rn, L, pot, species)
        w = V + 0.5 * dt * (F + Fn)
        P = float((Fn * w).sum())
        vn = math.sqrt(float((w * w).sum()))
        fn = math.sqrt(float((Fn * Fn).sum()))
        for k, v in (("w", w.copy()), ("drift", drift), ("dt", dt), ("alpha", a), ("mixed", P > 0.0),
                     ("vn", vn), ("fn", fn)):
            rec[k].append(v)
        if P > 0.0:
            V = (1.0 - a) * w + a * vn * Fn / fn
            n_pos += 1
            if n_pos > p.n_min:
                dt = min(dt * p.f_inc, p.dt_max)
                a *= p.f_alpha
        else:
            V = np.zeros_like(w)
            dt *= p.f_dec
            a = p.alpha_start
            n_pos = 0
        R, F = Rn, Fn
        rec["R"].append(R.copy())
        rec["F"].append(F.copy())
    out = {k: np.array(v) for k, v in rec.items()}
    out["V"] = V
    return out


def fire_unrolled_grad(R0, L, pot: Potential, species=None, K: int = 300, params: FireParams | None = None):
    """E_K = U(L R_K) after K FIRE steps from R0 and its derivatives by reverse mode through the steps.

    Cotangents: Rb (of R), Vb (of V), Fb (of the force of the state being processed), and the parameter
    cotangents.  Start at step K: Rb = dU/dR = -L F(R_K), Vb = 0, Fb = 0, parameters = the energy's own
    derivatives at R_K.  Step k, (R_k, V_k) -> (R_k+1, V_k+1), is transposed for k = K-1 .. 0 as
        mixing (P > 0 only):  c = Fhat . Vb with Fhat = F_k+1 / fn
                              wb = (1 - a) Vb + a c w / vn;   Fb += a vn (Vb - c Fhat) / fn
                              (P <= 0: V_k+1 = 0, so wb = 0)
        w = V + dt/2 (F + F'): Fb += dt/2 wb
        F' = F(L R_k+1):     Rb += L (dF/dx) Fb  (dF/dx is symmetric);  theta-bar += Fb . dF/dtheta
        R' = R + drift / c:  ln c-bar -= Rb . drift  (the drift is divided by the scaled box)
                             Vb = wb + dt Rb / L;  Fb = dt/2 wb + dt^2/2 Rb / L  (now the cotangent of F_k)
    and after the loop the force of R_0 is transposed once more (R_0 itself does not depend on the parameters at
    a fixed fractional start).  Returns dict E, g_sigma, g_eps, g_lnc, Rbar0 (dE_K/dR_0) and the trajectory.
    """
    tr = fire_fixed_steps(R0, L, pot, species, K, params)
    Lv = np.asarray(L, dtype=np.float64)[: tr["R"].shape[2]]
    RK = tr["R"][K]
    E, gs, ge, gl = energy_grads(RK, L, pot, species)
    Rb = -tr["F"][K] * Lv
    Vb = np.zeros_like(Rb)
    Fb = np.zeros_like(Rb)
    for k in range(K - 1, -1, -1):
        dt, a = tr["dt"][k], tr["alpha"][k]
        w, Fn = tr["w"][k], tr["F"][k + 1]
        if tr["mixed"][k]:
            vn, fn = tr["vn"][k], tr["fn"][k]
            Fhat = Fn / fn
            c = float((Fhat * Vb).sum())
            wb = (1.0 - a) * Vb + a * c * w / vn
            Fb = Fb + a * vn * (Vb - c * Fhat) / fn
        else:
            wb = np.zeros_like(Vb)
        Fb = Fb + 0.5 * dt * wb
        Rk1 = tr["R"][k + 1]
        Rb = Rb + Lv * force_jvp(Rk1, L, pot, species, Fb)
        dgs, dge, dgl = force_param_vjp(Rk1, L, pot, species, Fb)
        gs, ge, gl = gs + dgs, ge + dge, gl + dgl
        gl -= float((Rb * tr["drift"][k]).sum())
        Vb = wb + dt * Rb / Lv
        Fb = 0.5 * dt * wb + 0.5 * dt * dt * Rb / Lv
    Rb = Rb + Lv * force_jvp(tr["R"][0], L, pot, species, Fb)
    dgs, dge, dgl = force_param_vjp(tr["R"][0], L, pot, species, Fb)
    return {"E": E, "g_sigma": gs + dgs, "g_eps": ge + dge, "g_lnc": gl + dgl, "Rbar0": Rb, "traj": tr}


def final_energy(R0, L, pot: Potential, species=None, K: int = 300, params: FireParams | None = None):
    """E_K alone (the function whose derivatives fire_unrolled_grad returns) and the branch record."""
    tr = fire_fixed_steps(R0, L, pot, species, K, params)
    Lv = np.asarray(L, dtype=np.float64)[: tr["R"].shape[2]]
    _, e, _ = pair_rows(tr["R"][K] * Lv, Lv, pot, species)
    return math.fsum(e.tolist()), tr["mixed"]


def torus_to_frac(u):
    """uint32 torus coordinates -> fractional coordinates u / 2^32 in float64 (exact)."""
    return decode(u, np.ones(np.asarray(u).shape[1]))
