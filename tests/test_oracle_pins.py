"""Pins of the FP64 oracle against closed forms, invariants, brute force and library routines.

Each test checks the oracle against something other than itself, chosen so
that a dropped term, a wrong sign, a wrong index or a transposed operand in
oracle/md_oracle.c fails at least one of them.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from paper_1912_04232_amd import inputs

LJ = dict(kind="lj", r_cut=2.5)


def lj_pot(orc, shift=True, sigma=1.0, eps=1.0, rc=2.5):
    return orc.Potential("lj", np.array([[sigma]]), np.array([[eps]]), r_cut=rc, shift=shift)


def ss_pot(orc, d=(1.0, 1.4), eps=1.0, alpha=2.0):
    d = np.asarray(d, dtype=np.float64)
    return orc.Potential("soft_sphere", 0.5 * (d[:, None] + d[None, :]), np.full((len(d), len(d)), eps),
                         alpha=alpha)


def dimer(r, L=20.0, dim=3, across=False):
    x = np.full((2, dim), L / 2)
    if across:
        x[0, 0] = 0.3
        x[1, 0] = 0.3 - r + L
    else:
        x[1, 0] += r
    return x, [L] * dim


# ------------------------------------------------------------------ potentials

def test_lj_minimum_closed_form(orc):
    """Unshifted LJ: u(2^(1/6) sigma) = -eps, F = 0 there; u(sigma) = 0; |F(sigma)| = 24 eps/sigma."""
    for sigma, eps in [(1.0, 1.0), (1.3, 0.7)]:
        p = lj_pot(orc, shift=False, sigma=sigma, eps=eps, rc=2.5 * sigma)
        x, L = dimer(2 ** (1 / 6) * sigma)
        F, e, _ = orc.pair_rows(x, L, p)
        assert math.isclose(e.sum(), -eps, rel_tol=1e-14)
        assert np.abs(F).max() < 1e-12 * eps / sigma
        x, L = dimer(sigma)
        F, e, _ = orc.pair_rows(x, L, p)
        assert abs(e.sum()) < 1e-14
        # particle 0 sits at smaller x, it is pushed to -x
        assert math.isclose(F[0, 0], -24 * eps / sigma, rel_tol=1e-13)
        assert math.isclose(F[1, 0], 24 * eps / sigma, rel_tol=1e-13)


def test_lj_shift_and_cutoff(orc):
    """Shifted LJ: u(r) - u(r_c) with u(r_c) = 4(2.5^-12 - 2.5^-6) = -0.0163169...; zero at r >= r_c."""
    uc = 4 * (2.5 ** -12 - 2.5 ** -6)
    assert math.isclose(uc, -0.01631689, rel_tol=1e-6)
    p = lj_pot(orc, shift=True)
    x, L = dimer(1.5)
    _, e, _ = orc.pair_rows(x, L, p)
    assert math.isclose(e.sum(), 4 * (1.5 ** -12 - 1.5 ** -6) - uc, rel_tol=1e-14)
    for r in (2.5, 2.6):
        x, L = dimer(r)
        F, e, w = orc.pair_rows(x, L, p)
        assert e.sum() == 0 and np.all(F == 0) and w.sum() == 0


def test_lj_curvature_at_minimum(orc):
    """u''(r_min) = 72 * 2^(-1/3) = 57.146: the force derivative checked by central differences of F."""
    p = lj_pot(orc, shift=False)
    r0, h = 2 ** (1 / 6), 1e-5
    f = []
    for r in (r0 - h, r0 + h):
        x, L = dimer(r)
        F, _, _ = orc.pair_rows(x, L, p)
        f.append(F[1, 0])
    k = -(f[1] - f[0]) / (2 * h)
    assert math.isclose(k, 72 * 2 ** (-1 / 3), rel_tol=1e-7)


def test_soft_sphere_closed_forms(orc):
    """u(0+) -> eps/alpha, u(sigma) = 0, force continuous (-> 0) at contact for alpha = 2, alpha = 2.5 form."""
    p = ss_pot(orc, d=(1.0,))
    x, L = dimer(1e-9, dim=2)
    _, e, _ = orc.pair_rows(x, L, p)
    assert math.isclose(e.sum(), 0.5, rel_tol=1e-8)
    x, L = dimer(1.0, dim=2)
    F, e, _ = orc.pair_rows(x, L, p)
    assert e.sum() == 0 and np.all(F == 0)
    x, L = dimer(1.0 - 1e-9, dim=2)
    F, e, _ = orc.pair_rows(x, L, p)
    assert abs(F[0, 0]) < 2e-9
    # general alpha at r = 0.6 sigma with sigma_ab = (1.0 + 1.4)/2 = 1.2
    p = ss_pot(orc, d=(1.0, 1.4), eps=2.0, alpha=2.5)
    x, L = dimer(0.72, dim=2)
    F, e, _ = orc.pair_rows(x, L, p, species=[0, 1])
    assert math.isclose(e.sum(), 2.0 / 2.5 * 0.4 ** 2.5, rel_tol=1e-14)
    assert math.isclose(F[1, 0], 2.0 / 1.2 * 0.4 ** 1.5, rel_tol=1e-14)


def test_nearest_image_across_face(orc):
    """A pair straddling the x face interacts exactly like the same pair in the middle of the box."""
    p = lj_pot(orc)
    for r in (0.95, 1.2, 2.3):
        x, L = dimer(r)
        F0, e0, w0 = orc.pair_rows(x, L, p)
        x, L = dimer(r, across=True)
        F1, e1, w1 = orc.pair_rows(x, L, p)
        assert math.isclose(e0.sum(), e1.sum(), rel_tol=1e-12)
        # across the face particle 0 is to the right of particle 1
        assert math.isclose(F1[0, 0], -F0[0, 0], rel_tol=1e-10)


# -------------------------------------------------------- energy / forces / virial

def small_lj_system(N=64, rho=0.6, seed=7):
    L = inputs.box_for_density(N, rho)
    u = inputs.random_insertion_torus(N, L, 3, 0.85, seed)
    return u, [L, L, L]


def small_ss_system(N=60, phi=0.9, seed=5):
    L = inputs.box_for_packing([1.0, 1.4], [N // 2, N // 2], phi, 2)
    u = inputs.uniform_torus(N, 2, seed)
    return u, [L, L], inputs.bidisperse_species(N)


def test_newton_third_law(orc):
    u, L = small_lj_system()
    F, _, _ = orc.pair_rows(orc.decode(u, L), L, lj_pot(orc))
    assert np.abs(F.sum(axis=0)).max() < 1e-11 * np.abs(F).max()
    u, L, sp = small_ss_system()
    F, _, _ = orc.pair_rows(orc.decode(u, L), L, ss_pot(orc), species=sp)
    assert np.abs(F.sum(axis=0)).max() < 1e-12 * np.abs(F).max()


@pytest.mark.parametrize("which", ["lj", "ss"])
def test_forces_are_minus_gradient(orc, which):
    """Central finite differences of U (h = 1e-6) reproduce the analytic forces."""
    if which == "lj":
        u, L = small_lj_system()
        p, sp = lj_pot(orc), None
    else:
        u, L, sp = small_ss_system()
        p = ss_pot(orc)
    x = orc.decode(u, L)
    F, _, _ = orc.pair_rows(x, L, p, species=sp)
    rng = np.random.default_rng(0)
    h = 1e-6
    for i in rng.choice(len(x), 6, replace=False):
        for k in range(x.shape[1]):
            xp = x.copy()
            xp[i, k] += h
            xm = x.copy()
            xm[i, k] -= h
            fd = -(orc.energy(xp, L, p, sp) - orc.energy(xm, L, p, sp)) / (2 * h)
            assert abs(fd - F[i, k]) <= 1e-6 * max(1.0, abs(F[i, k])), (i, k, fd, F[i, k])


@pytest.mark.parametrize("which", ["lj", "ss"])
def test_virial_is_minus_dU_dlnlambda(orc, which):
    """W = sum_{i<j} r f(r) = -dU/dlambda at lambda = 1 for r -> lambda r (box scaled too)."""
    if which == "lj":
        u, L = small_lj_system()
        p, sp = lj_pot(orc), None
    else:
        u, L, sp = small_ss_system()
        p = ss_pot(orc)
    x = orc.decode(u, L)
    _, _, w = orc.pair_rows(x, L, p, species=sp)
    W = math.fsum(w)
    h = 1e-6
    Up = orc.energy(x * (1 + h), [l * (1 + h) for l in L], p, sp)
    Um = orc.energy(x * (1 - h), [l * (1 - h) for l in L], p, sp)
    assert math.isclose(W, -(Up - Um) / (2 * h), rel_tol=1e-6, abs_tol=1e-8)


def test_fcc_lattice_symmetry(orc):
    """Perfect FCC: every force vanishes by symmetry and every e_i is equal."""
    n = 4
    L = inputs.box_for_density(4 * n ** 3, 0.84)
    u = inputs.fcc_torus(n, L)
    F, e, _ = orc.pair_rows(orc.decode(u, [L] * 3), [L] * 3, lj_pot(orc))
    assert np.abs(F).max() < 1e-10
    assert e.max() - e.min() < 1e-12
    assert e.mean() < -3.0


def test_triangular_lattice_closed_form(orc):
    """Triangular disks of diameter 1 at spacing a < 1: 6 contacts each, E/N = 3/2 (1 - a)^2, F = 0."""
    a = 0.98
    u, Lx, Ly = inputs.triangular_torus(8, 8, a)
    p = ss_pot(orc, d=(1.0,))
    x = orc.decode(u, [Lx, Ly])
    F, e, _ = orc.pair_rows(x, [Lx, Ly], p)
    assert np.abs(F).max() < 1e-6
    assert math.isclose(e.sum() / len(e), 1.5 * (1 - a) ** 2, rel_tol=1e-5)


def test_translation_invariance(orc):
    u, L = small_lj_system()
    p = lj_pot(orc)
    U0 = orc.energy(orc.decode(u, L), L, p)
    shift = np.array([123456789, 3000000000, 77], dtype=np.uint64)
    u2 = ((u.astype(np.uint64) + shift) % 2 ** 32).astype(np.uint32)
    U1 = orc.energy(orc.decode(u2, L), L, p)
    assert math.isclose(U0, U1, rel_tol=1e-12)


# ------------------------------------------------------------------ neighbor set

def exact_neighbors(u, L, r_list):
    """Exact rational brute force: (i, j) with sum_k (wrap32(u_ik - u_jk) L_k / 2^32)^2 < r_list^2."""
    N, dim = u.shape
    Lq = [Fraction(float(np.float32(l))) for l in L[:dim]]
    rl2 = Fraction(float(np.float32(r_list))) ** 2
    out = []
    for i in range(N):
        row = []
        for j in range(N):
            if i == j:
                continue
            r2 = Fraction(0)
            for k in range(dim):
                d = (int(u[i, k]) - int(u[j, k])) % 2 ** 32
                if d >= 2 ** 31:
                    d -= 2 ** 32
                r2 += (Fraction(d) * Lq[k] / 2 ** 32) ** 2
            if r2 < rl2:
                row.append(j)
        out.append(row)
    return out


def test_neighbors_match_exact_rational(orc):
    for dim in (2, 3):
        N = 60
        L = [inputs.f32(5.3), inputs.f32(6.1), inputs.f32(4.9)][:dim]
        u = inputs.uniform_torus(N, dim, 11 + dim)
        got = orc.neighbors(u, L + [0.0] * (3 - dim), 2.2)
        want = exact_neighbors(u, L, 2.2)
        assert [list(r) for r in got] == want


def test_neighbors_boundary_is_strict(orc):
    """Hand-built pairs at the list radius: r^2 == r_list^2 is out, one unit closer is in."""
    L = 16.0  # 2^32 units per 16 -> exact scale 2^-28
    r_list = 2.5
    s = L / 2 ** 32
    d_exact = int(round(r_list / s))  # 2.5 * 2^28, exactly representable: r == r_list
    assert d_exact * s == r_list
    u = np.zeros((4, 3), dtype=np.uint32)
    u[1, 0] = d_exact                 # exactly at r_list: excluded
    u[2, 1] = d_exact - 1             # one unit inside: included
    u[3, 2] = (2 ** 32 - (d_exact - 1)) % 2 ** 32  # one unit inside, across the z face
    rows = orc.neighbors(u, [L, L, L], r_list)
    assert list(rows[0]) == [2, 3]
    assert list(rows[1]) == []        # 0 sits exactly at r_list; 2 and 3 are 2.5*sqrt(2) away
    assert list(rows[2]) == [0] and list(rows[3]) == [0]


def test_neighbor_symmetry_and_density(orc):
    N = 2000
    L = inputs.box_for_density(N, 0.84)
    u = inputs.uniform_torus(N, 3, 3)
    rows = orc.neighbors(u, [L] * 3, 2.8)
    pairs = {(i, int(j)) for i, r in enumerate(rows) for j in r}
    assert all((j, i) in pairs for (i, j) in pairs)
    mean = len(pairs) / N
    expect = 0.84 * 4 / 3 * math.pi * 2.8 ** 3
    assert abs(mean - expect) < 0.05 * expect


# -------------------------------------------------------------- velocity Verlet

def test_verlet_dimer_period(orc):
    """Small oscillation of an LJ dimer: period 2 pi / sqrt(2 u''(r_min)) = 0.58772."""
    p = lj_pot(orc, shift=False)
    r0 = 2 ** (1 / 6)
    x, L = dimer(r0 + 1e-4)
    F, _, _ = orc.pair_rows(x, L, p)
    v = np.zeros_like(x)
    dt, n = 1e-4, 15000
    rs = []
    for _ in range(n // 50):
        x, v, F = orc.verlet(x, v, F, L, p, dt, 50, nthreads=1)
        rs.append(x[1, 0] - x[0, 0] - r0)
    rs = np.array(rs)
    t = (np.arange(len(rs)) + 1) * 50 * dt
    up = np.where((rs[:-1] < 0) & (rs[1:] >= 0))[0]
    tc = t[up] - rs[up] * (t[up + 1] - t[up]) / (rs[up + 1] - rs[up])
    period = np.diff(tc).mean()
    assert math.isclose(period, 2 * math.pi / math.sqrt(2 * 72 * 2 ** (-1 / 3)), rel_tol=2e-3)
    assert math.isclose(period, 0.58772, rel_tol=2e-3)


def lj108():
    n = 3
    L = inputs.box_for_density(4 * n ** 3, 0.84)
    u = inputs.fcc_torus(n, L)
    v = inputs.maxwell_velocities(4 * n ** 3, 3, 1.0, 9).astype(np.float64)
    return u, [L] * 3, v


def total_energy(orc, x, v, L, p):
    return orc.energy(x, L, p) + 0.5 * float(np.sum(v * v))


def test_verlet_energy_error_scales_dt2(orc):
    u, L, v0 = lj108()
    p = lj_pot(orc, rc=2.5)
    x0 = orc.decode(u, L)
    F0, _, _ = orc.pair_rows(x0, L, p)
    E0 = total_energy(orc, x0, v0, L, p)
    err = []
    for dt in (0.004, 0.002):
        x, v, F = x0, v0, F0
        worst = 0.0
        for _ in range(int(round(0.2 / dt / 10))):
            x, v, F = orc.verlet(x, v, F, L, p, dt, 10)
            worst = max(worst, abs(total_energy(orc, x, v, L, p) - E0))
        err.append(worst)
    ratio = err[0] / err[1]
    assert 3.0 < ratio < 5.5, err
    assert err[1] / len(x0) < 1e-4


def test_verlet_reversible_and_momentum(orc):
    u, L, v0 = lj108()
    p = lj_pot(orc)
    x0 = orc.decode(u, L)
    F0, _, _ = orc.pair_rows(x0, L, p)
    x, v, F = orc.verlet(x0, v0, F0, L, p, 0.005, 40)
    assert np.abs(v.sum(axis=0) - v0.sum(axis=0)).max() < 1e-10
    xb, vb, _ = orc.verlet(x, -v, F, L, p, 0.005, 40)
    d = xb - x0
    d -= np.array(L) * np.rint(d / np.array(L))
    assert np.abs(d).max() < 1e-8
    assert np.abs(-vb - v0).max() < 1e-8


# ------------------------------------------------------------------------ FIRE

def test_fire_two_disks_separate_to_contact(orc):
    p = ss_pot(orc, d=(1.0, 1.4))
    x, L = dimer(0.7, dim=2)
    res = orc.fire(x, L, p, species=[0, 1], f_tol=1e-10, max_steps=20000)
    assert res["converged"]
    d = res["x"][1] - res["x"][0]
    d -= np.array(L) * np.rint(d / np.array(L))
    assert np.linalg.norm(d) >= 1.2 - 1e-9
    assert orc.energy(res["x"], L, p, [0, 1]) < 1e-18


def test_fire_perturbed_triangular_lattice(orc):
    """FIRE brings a jittered compressed triangular lattice back to E/N = 3/2 (1 - a)^2."""
    a = 0.98
    u, Lx, Ly = inputs.triangular_torus(8, 8, a)
    L = [Lx, Ly]
    x = orc.decode(u, L)
    x += np.random.default_rng(2).normal(0, 0.01, x.shape)
    p = ss_pot(orc, d=(1.0,))
    res = orc.fire(x, L, p, f_tol=1e-10, max_steps=50000)
    assert res["converged"]
    assert math.isclose(orc.energy(res["x"], L, p) / len(x), 1.5 * (1 - a) ** 2, rel_tol=1e-6)


def test_fire_matches_scipy_minimum(orc):
    """On a small jammed system FIRE and scipy's L-BFGS reach a minimum of the same energy from a shared start."""
    from scipy.optimize import minimize
    a = 0.97
    u, Lx, Ly = inputs.triangular_torus(6, 6, a)
    L = [Lx, Ly]
    x0 = orc.decode(u, L) + np.random.default_rng(4).normal(0, 0.02, (36, 2))
    p = ss_pot(orc, d=(1.0,))
    res = orc.fire(x0, L, p, f_tol=1e-11, max_steps=50000)

    def fun(z):
        xx = z.reshape(-1, 2)
        F, e, _ = orc.pair_rows(xx, L, p)
        return math.fsum(e), -F.ravel()

    sp = minimize(fun, x0.ravel(), jac=True, method="L-BFGS-B", options=dict(ftol=1e-16, gtol=1e-12,
                                                                               maxiter=10000))
    assert math.isclose(orc.energy(res["x"], L, p), sp.fun, rel_tol=1e-8)


def test_fire_step_rules(orc):
    """After one step from rest the state follows the FIRE rules: P > 0 on the first step, dt unchanged
    (n_pos = 1 <= n_min), v = (1 - a) v + a |v| F/|F| applied to the velocity-Verlet velocity."""
    u, L, sp = small_ss_system()
    p = ss_pot(orc)
    x0 = orc.decode(u, L)
    fp = orc.FireParams()
    res = orc.fire(x0, L, p, sp, fp, max_steps=1, f_tol=0.0)
    F0, _, _ = orc.pair_rows(x0, L, p, sp)
    x1 = x0 + 0.5 * fp.dt_start ** 2 * F0
    x1 -= np.array(L) * np.floor(x1 / np.array(L))
    F1, _, _ = orc.pair_rows(x1, L, p, sp)
    v = 0.5 * fp.dt_start * (F0 + F1)
    assert float(np.sum(F1 * v)) > 0
    a = fp.alpha_start
    v = (1 - a) * v + a * np.linalg.norm(v) * F1 / np.linalg.norm(F1)
    assert np.allclose(res["v"], v, rtol=1e-12, atol=1e-14)
    assert res["dt"] == fp.dt_start and res["n_pos"] == 1 and res["steps"] == 1


# --------------------------------------------------------- parameter gradients

def test_param_grad_matches_fd(orc):
    u, L, sp = small_ss_system()
    x = orc.decode(u, L)
    d = np.array([1.0, 1.4])
    g = orc.diameter_grad(x, L, d, 1.0, sp)
    h = 1e-6
    for s in range(2):
        dp = d.copy()
        dp[s] += h
        dm = d.copy()
        dm[s] -= h
        Up = orc.energy(x, L, ss_pot(orc, d=dp), sp)
        Um = orc.energy(x, L, ss_pot(orc, d=dm), sp)
        assert math.isclose(g[s], (Up - Um) / (2 * h), rel_tol=1e-6)
    # LJ sigma / epsilon entries by FD on a two-species LJ system
    u, L = small_lj_system()
    x = orc.decode(u, L)
    spl = inputs.bidisperse_species(len(x))
    sig = np.array([[1.0, 1.1], [1.1, 1.2]])
    eps = np.array([[1.0, 0.8], [0.8, 0.6]])
    gs, ge = orc.param_grad(x, L, orc.Potential("lj", sig, eps, r_cut=2.5), spl)
    for (a, b) in [(0, 0), (0, 1), (1, 1)]:
        for which, G in (("s", gs), ("e", ge)):
            vals = []
            for sgn in (1, -1):
                s2, e2 = sig.copy(), eps.copy()
                M = s2 if which == "s" else e2
                M[a, b] += sgn * h
                if a != b:
                    M[b, a] += sgn * h
                vals.append(orc.energy(x, L, orc.Potential("lj", s2, e2, r_cut=2.5), spl))
            fd = (vals[0] - vals[1]) / (2 * h)
            an = G[a, b] + (G[b, a] if a != b else 0.0)
            assert math.isclose(an, fd, rel_tol=1e-6, abs_tol=1e-9), (which, a, b, an, fd)


def test_param_grad_identities(orc):
    """dU/deps = U/eps; soft spheres: sum_s d_s dU/dd_s = W (u depends on r/sigma only)."""
    u, L, sp = small_ss_system()
    x = orc.decode(u, L)
    p = ss_pot(orc, eps=1.7)
    _, ge = orc.param_grad(x, L, p, sp)
    assert math.isclose(ge.sum() * 1.7, orc.energy(x, L, p, sp), rel_tol=1e-12)
    d = np.array([1.0, 1.4])
    g = orc.diameter_grad(x, L, d, 1.0, sp)
    _, _, w = orc.pair_rows(x, L, ss_pot(orc, d=d), sp)
    assert math.isclose(float(g @ d), math.fsum(w), rel_tol=1e-12)


def test_rescaled_box_grad_matches_fd(orc):
    """dU/dD at fixed fractional positions for the bidisperse disks whose box follows the packing-fraction law
    (App. A): central differences of U with the box edge and sigma both recomputed at D +- h."""
    rng = np.random.default_rng(12)
    N, phi = 64, 0.9
    u = rng.integers(0, 2 ** 32, size=(N, 2), dtype=np.uint64).astype(np.uint32)
    sp = inputs.bidisperse_species(N)

    def box(D):  # the packing-fraction law in float64: N/2 disks of each diameter
        return math.sqrt((N // 2) * math.pi * (D * D + 1.0) / 4.0 / phi)

    for D in (0.6, 0.8, 1.0, 1.3):
        U, g = orc.rescaled_box_grad(u, box(D), D, sp)
        h = 1e-6
        Up, _ = orc.rescaled_box_grad(u, box(D + h), D + h, sp)
        Um, _ = orc.rescaled_box_grad(u, box(D - h), D - h, sp)
        assert U > 0
        assert math.isclose(g, (Up - Um) / (2 * h), rel_tol=1e-6, abs_tol=1e-9), (D, g, (Up - Um) / (2 * h))


def test_rescaled_box_envelope_matches_fd_through_minimization(orc):
    """At an FP64 FIRE minimum s* of the rescaled-box disks, dU/dD(s*) equals the central difference of the
    minimized energy E*(D +- h), each minimized from s* in the box of D +- h (envelope theorem, Sec. 4.2)."""
    N, phi, D, h = 32, 0.9, 0.8, 1e-5
    u0 = np.random.default_rng(21).integers(0, 2 ** 32, size=(N, 2), dtype=np.uint64).astype(np.uint32)
    sp = inputs.bidisperse_species(N)

    def box(Dx):
        return math.sqrt((N // 2) * math.pi * (Dx * Dx + 1.0) / 4.0 / phi)

    def pot(Dx):
        d = np.array([Dx, 1.0])
        return orc.Potential("soft_sphere", 0.5 * (d[:, None] + d[None, :]), np.ones((2, 2)), alpha=2.0)

    def minimize(s, Dx):
        L = box(Dx)
        r = orc.fire(s * L, [L, L], pot(Dx), sp, f_tol=1e-11, max_steps=400000)
        assert r["converged"]
        return r["x"] / L, orc.energy(r["x"], [L, L], pot(Dx), sp)

    s_star, E = minimize(u0.astype(np.float64) / 2.0 ** 32, D)
    u_star = inputs.to_torus(s_star, [1.0, 1.0])
    _, g = orc.rescaled_box_grad(u_star, box(D), D, sp)
    fd = (minimize(s_star, D + h)[1] - minimize(s_star, D - h)[1]) / (2 * h)
    assert E > 0
    assert math.isclose(g, fd, rel_tol=1e-4, abs_tol=1e-7), (g, fd)


# ----------------------------------------------------------------------- inputs

def test_workload_boxes():
    """Float32 box edges of the workloads (density / packing fraction definitions)."""
    assert math.isclose(inputs.box_for_density(1000, 0.8), 10.772173, rel_tol=1e-6)
    assert math.isclose(inputs.box_for_density(256000, 0.84), 67.29563, rel_tol=1e-6)
    assert math.isclose(inputs.box_for_packing([1.0, 1.4], [32768, 32768], 0.9, 2), 290.93402, rel_tol=1e-6)
    u = inputs.fcc_torus(3, 5.0)
    assert u.shape == (108, 3) and len({tuple(r) for r in u.tolist()}) == 108
    v = inputs.maxwell_velocities(500, 3, 1.5, 1)
    assert np.abs(v.astype(np.float64).sum(0)).max() < 1e-4
    assert math.isclose(float(np.sum(v.astype(np.float64) ** 2)) / (3 * 499), 1.5, rel_tol=1e-5)


def test_envelope_theorem_through_fire(orc):
    """dE*/dd_s of the FIRE-minimized energy (box fixed, same start) by central differences (h = 1e-4) equals
    dU/dd_s at the minimum: the oracle's parameter gradient is the adjoint of the minimizer."""
    N = 40
    L = inputs.box_for_packing([1.0, 1.4], [N // 2, N // 2], 0.9, 2)
    x0 = orc.decode(inputs.uniform_torus(N, 2, 77), [L, L])
    sp = inputs.bidisperse_species(N)
    d = np.array([1.0, 1.4])
    res = orc.fire(x0, [L, L], ss_pot(orc, d=d), sp, f_tol=1e-11, max_steps=200000)
    assert res["converged"]
    g = orc.diameter_grad(res["x"], [L, L], d, 1.0, sp)
    h = 1e-4
    for s in range(2):
        E = []
        for sgn in (1, -1):
            dd = d.copy()
            dd[s] += sgn * h
            r = orc.fire(x0, [L, L], ss_pot(orc, d=dd), sp, f_tol=1e-11, max_steps=200000)
            assert r["converged"]
            E.append(orc.energy(r["x"], [L, L], ss_pot(orc, d=dd), sp))
        fd = (E[0] - E[1]) / (2 * h)
        assert math.isclose(g[s], fd, rel_tol=1e-5, abs_tol=1e-10), (s, g[s], fd)


# ------------------------------------------------------------------------ Morse

def morse_pot(orc, shift=True):
    return orc.Potential("morse", np.array([[1.1, 1.2], [1.2, 1.3]]), np.array([[1.0, 0.7], [0.7, 1.4]]), alpha=3.0,
                         r_cut=2.8, shift=shift)


def test_morse_dimer_closed_form(orc):
    """Two particles of species (0, 1): u(r) = eps [(1 - exp(-a (r - s)))^2 - 1], minimum -eps at r = s, zero force
    there, and the energy shift is u(r_c)."""
    L = [30.0, 30.0, 30.0]
    for r, shift in ((1.2, False), (1.0, False), (2.0, True), (2.79, True)):
        x = np.array([[5.0, 5.0, 5.0], [5.0 + r, 5.0, 5.0]])
        F, e, _ = orc.pair_rows(x, L, morse_pot(orc, shift), [0, 1])
        t = math.exp(-3.0 * (r - 1.2))
        u = 0.7 * ((1 - t) ** 2 - 1)
        if shift:
            tc = math.exp(-3.0 * (2.8 - 1.2))
            u -= 0.7 * ((1 - tc) ** 2 - 1)
        fr = -2.0 * 3.0 * 0.7 * t * (1 - t)          # force on particle 1 along +x
        assert math.isclose(e.sum(), u, rel_tol=1e-13, abs_tol=1e-15)
        assert math.isclose(F[1, 0], fr, rel_tol=1e-13, abs_tol=1e-13) and F[0, 0] == pytest.approx(-fr, abs=1e-13)
    x = np.array([[5.0, 5.0, 5.0], [6.2, 5.0, 5.0]])
    F, e, _ = orc.pair_rows(x, L, morse_pot(orc, False), [0, 1])
    assert math.isclose(e.sum(), -0.7, rel_tol=1e-14) and abs(F).max() < 1e-13
    x = np.array([[5.0, 5.0, 5.0], [7.85, 5.0, 5.0]])       # beyond the cutoff
    F, e, _ = orc.pair_rows(x, L, morse_pot(orc), [0, 1])
    assert e.sum() == 0.0 and abs(F).max() == 0.0


def test_morse_forces_are_minus_energy_gradient(orc):
    N = 60
    L = [5.5, 5.0, 4.8]
    x = inputs.uniform_torus(N, 3, 19).astype(np.float64) * (np.array(L) / 2.0 ** 32)
    sp = np.arange(N) % 2
    pot = morse_pot(orc)
    F, _, _ = orc.pair_rows(x, L, pot, sp)
    rng = np.random.default_rng(2)
    z = rng.standard_normal(x.shape)
    h = 1e-6
    fd = -(orc.energy(x + h * z, L, pot, sp) - orc.energy(x - h * z, L, pot, sp)) / (2 * h)
    assert (F * z).sum() == pytest.approx(fd, rel=1e-7, abs=1e-9)


# ------------------------------------------------------------------- Buckingham

def buck_pot(orc, A=((2.6e5, 2.0e5), (2.0e5, 1.6e5)), rho=((0.08, 0.085), (0.085, 0.09)),
             C=((1.0, 1.2), (1.2, 1.4)), shift=True, r_cut=2.8):
    return orc.Potential("buckingham", np.array(rho), np.array(A), r_cut=r_cut, shift=shift, coef=np.array(C))


def dimer_energy_force(orc, pot, r, sp=(0, 1)):
    L = [30.0, 30.0, 30.0]
    x = np.array([[5.0, 5.0, 5.0], [5.0 + r, 5.0, 5.0]])
    F, e, _ = orc.pair_rows(x, L, pot, list(sp))
    return float(e.sum()), float(F[1, 0])     # energy and the force on the second particle along +x


def test_buckingham_exponential_and_dispersion_laws(orc):
    """The two parts of the (0, 1) pair separately, unshifted: with the dispersion off, the energy falls by e over
    one range rho_01 = 0.085 and the force is u / rho; with the repulsion off, doubling r divides u by 64 and
    r f = 6 u (an attraction: u < 0, f < 0).  Both parts use the (0, 1) entries of their matrices."""
    rep = buck_pot(orc, C=((0.0, 0.0), (0.0, 0.0)), shift=False)
    for r in (0.9, 1.3):
        u1, f1 = dimer_energy_force(orc, rep, r)
        u2, _ = dimer_energy_force(orc, rep, r + 0.085)
        assert math.isclose(u2 / u1, math.exp(-1.0), rel_tol=1e-13)
        assert math.isclose(f1, u1 / 0.085, rel_tol=1e-13)
    disp = buck_pot(orc, A=((0.0, 0.0), (0.0, 0.0)), shift=False)
    for r in (0.9, 1.2):
        u1, f1 = dimer_energy_force(orc, disp, r)
        u2, _ = dimer_energy_force(orc, disp, 2 * r)
        assert math.isclose(u2 / u1, 1.0 / 64.0, rel_tol=1e-13) and u1 < 0
        assert math.isclose(r * f1, 6.0 * u1, rel_tol=1e-13) and f1 < 0
    # beyond the cutoff nothing; with the shift the energy is continuous at the cutoff, without it is not
    assert dimer_energy_force(orc, buck_pot(orc), 2.8001) == (0.0, 0.0)
    assert abs(dimer_energy_force(orc, buck_pot(orc), 2.8 - 1e-9)[0]) < 1e-9
    assert abs(dimer_energy_force(orc, buck_pot(orc, shift=False), 2.8 - 1e-9)[0]) > 1e-3


def test_buckingham_force_vanishes_at_the_energy_minimum(orc):
    """The (0, 0) dimer's energy minimum located from energies alone (bounded scalar minimization) is where the
    oracle's force vanishes."""
    from scipy.optimize import minimize_scalar
    pot = buck_pot(orc, shift=False)
    res = minimize_scalar(lambda r: dimer_energy_force(orc, pot, r, (0, 0))[0], bounds=(0.8, 2.5), method="bounded",
                          options={"xatol": 1e-10})
    r0 = res.x
    u0, f0 = dimer_energy_force(orc, pot, r0, (0, 0))
    assert u0 < 0 and 0.9 < r0 < 2.0
    _, f_near = dimer_energy_force(orc, pot, r0 - 0.05, (0, 0))
    assert abs(f0) < 1e-6 * abs(f_near)


def test_buckingham_forces_are_minus_energy_gradient(orc):
    N = 60
    L = [5.5, 5.0, 4.8]
    x = inputs.random_insertion_torus(N, 5.0, 3, 0.85, 23).astype(np.float64) * (5.0 / 2.0 ** 32)
    L = [5.0, 5.0, 5.0]
    sp = np.arange(N) % 2
    pot = buck_pot(orc, r_cut=2.4)
    F, _, _ = orc.pair_rows(x, L, pot, sp)
    assert abs(F.sum(0)).max() < 1e-10 * abs(F).max()
    rng = np.random.default_rng(3)
    z = rng.standard_normal(x.shape)
    h = 1e-6
    fd = -(orc.energy(x + h * z, L, pot, sp) - orc.energy(x - h * z, L, pot, sp)) / (2 * h)
    assert (F * z).sum() == pytest.approx(fd, rel=1e-7, abs=1e-9)
