"""Pins of the FP64 reverse pass through fixed-K FIRE (oracle/unrolled.py) against finite differences of the
brute-force C pair sum and of the forward recurrence, the C FIRE of md_oracle.c, and the envelope theorem."""
import math

import numpy as np
import pytest

from paper_1912_04232_amd import inputs


@pytest.fixture(scope="module")
def un():
    from oracle import unrolled
    return unrolled


def ss(d=(1.0, 1.4), eps=(1.0, 1.0, 1.0), alpha=2.0):
    from oracle import Potential
    d = np.asarray(d, dtype=np.float64)
    e = np.array([[eps[0], eps[1]], [eps[1], eps[2]]], dtype=np.float64)
    return Potential("soft_sphere", 0.5 * (d[:, None] + d[None, :]), e, alpha=alpha)


def lj2():
    from oracle import Potential
    return Potential("lj", np.array([[1.0, 0.9], [0.9, 0.8]]), np.array([[1.0, 1.5], [1.5, 0.5]]),
                     r_cut=2.5, shift=True)


def packing(N, phi, seed, d=(1.0, 1.4)):
    L = inputs.box_for_packing(list(d), [N // 2, N - N // 2], phi, 2)
    R = inputs.uniform_torus(N, 2, seed).astype(np.float64) / 2.0 ** 32
    return R, np.array([L, L]), inputs.bidisperse_species(N)


def lj_gas(N, rho, seed):
    L = math.sqrt(N / rho)
    R = inputs.uniform_torus(N, 2, seed).astype(np.float64) / 2.0 ** 32
    return R, np.array([L, 0.8 * L]), inputs.bidisperse_species(N)


def with_sigma(pot, a, b, h):
    from oracle import Potential
    s = np.array(pot.sigma, dtype=np.float64).copy()
    s[a, b] += h
    if a != b:
        s[b, a] += h
    return Potential(pot.kind, s, np.array(pot.epsilon), alpha=pot.alpha, r_cut=pot.r_cut, shift=pot.shift)


def with_eps(pot, a, b, h):
    from oracle import Potential
    e = np.array(pot.epsilon, dtype=np.float64).copy()
    e[a, b] += h
    if a != b:
        e[b, a] += h
    return Potential(pot.kind, np.array(pot.sigma), e, alpha=pot.alpha, r_cut=pot.r_cut, shift=pot.shift)


@pytest.mark.parametrize("case", ["soft_sphere", "soft_sphere_a25", "lj"])
def test_force_jvp_matches_fd(un, case):
    if case == "lj":
        R, L, sp = lj_gas(40, 0.7, 11)
        pot = lj2()
    else:
        R, L, sp = packing(40, 0.9, 12)
        pot = ss(alpha=2.5 if case.endswith("a25") else 2.0)
    rng = np.random.default_rng(3)
    z = rng.standard_normal(R.shape)
    h = 1e-7
    fd = (un.forces(R + h * z / L, L, pot, sp) - un.forces(R - h * z / L, L, pot, sp)) / (2 * h)
    jv = un.force_jvp(R, L, pot, sp, z)
    assert np.abs(jv - fd).max() <= 1e-6 * np.abs(fd).max()
    # symmetry of the Hessian: y . (J z) = z . (J y)
    y = rng.standard_normal(R.shape)
    assert (y * jv).sum() == pytest.approx((z * un.force_jvp(R, L, pot, sp, y)).sum(), rel=1e-10)


@pytest.mark.parametrize("case", ["soft_sphere", "lj"])
def test_force_param_vjp_matches_fd(un, case):
    if case == "lj":
        R, L, sp = lj_gas(40, 0.7, 21)
        pot = lj2()
    else:
        R, L, sp = packing(40, 0.9, 22)
        pot = ss(eps=(1.0, 0.7, 1.3))
    rng = np.random.default_rng(5)
    z = rng.standard_normal(R.shape)
    gs, ge, gl = un.force_param_vjp(R, L, pot, sp, z)
    assert np.allclose(gs, gs.T) and np.allclose(ge, ge.T)
    h = 1e-6
    for a in range(2):
        for b in range(a, 2):
            for g, mod in ((gs, with_sigma), (ge, with_eps)):
                fd = ((un.forces(R, L, mod(pot, a, b, h), sp)
                       - un.forces(R, L, mod(pot, a, b, -h), sp)) * z).sum() / (2 * h)
                want = g[a, b] + (g[b, a] if a != b else 0.0)
                assert want == pytest.approx(fd, rel=1e-6, abs=1e-8 * np.abs(z).sum()), (a, b)
    c = math.exp(h)
    fd = ((un.forces(R, L * c, pot, sp) - un.forces(R, L / c, pot, sp)) * z).sum() / (2 * h)
    assert gl == pytest.approx(fd, rel=1e-6)


def test_energy_grads_match_fd(un):
    R, L, sp = packing(40, 0.9, 31)
    pot = ss(eps=(1.0, 0.7, 1.3))
    E, gs, ge, gl = un.energy_grads(R, L, pot, sp)
    h = 1e-6

    def U(p, LL):
        return un.energy_grads(R, LL, p, sp)[0]
    for a in range(2):
        for b in range(a, 2):
            fd = (U(with_sigma(pot, a, b, h), L) - U(with_sigma(pot, a, b, -h), L)) / (2 * h)
            assert gs[a, b] + (gs[b, a] if a != b else 0.0) == pytest.approx(fd, rel=1e-6)
    fd = (U(pot, L * math.exp(h)) - U(pot, L * math.exp(-h))) / (2 * h)
    assert gl == pytest.approx(fd, rel=1e-6)


def test_fixed_steps_match_c_fire(un):
    """The recorded forward (positions kept as fractions of the box) is md_oracle.c's orc_fire run on x = L R with
    no convergence test: same positions and velocities after K steps, in a rectangular box."""
    import oracle
    R, L, sp = packing(32, 0.9, 41)
    L = L * np.array([1.0, 1.15])
    pot = ss()
    K = 60
    tr = un.fire_fixed_steps(R, L, pot, sp, K)
    r = oracle.fire(R * L, L, pot, sp, max_steps=K, f_tol=0.0)
    assert r["steps"] == K
    d = tr["R"][K] * L - r["x"]
    d -= L * np.round(d / L)
    assert np.abs(d).max() < 1e-10 * L[0]
    assert np.allclose(tr["V"], r["v"], rtol=0, atol=1e-10 * np.abs(r["v"]).max())
    assert (~tr["mixed"]).any() and tr["mixed"].any()   # both branches were taken


@pytest.mark.parametrize("K", [1, 6, 40, 300])
def test_unrolled_grad_matches_fd_of_final_energy(un, K):
    """Every derivative of E_K (diameters through sigma_ab = (d_a + d_b)/2, each eps_ab, the box scale) against
    central differences of the forward recurrence, with the same branch decisions on both sides.  Near
    convergence P at a reset can be ~1e-6 (seed 350 at K = 300 flips a decision under h = 1e-6), so the seeds
    are ones whose branch record is stable under the perturbation; the record is compared on every call."""
    N = 20
    R, L, sp = packing(N, 0.9, 51 + K)
    d = np.array([1.0, 1.4])
    eps = (1.0, 0.8, 1.2)
    res = un.fire_unrolled_grad(R, L, ss(d, eps), sp, K)
    gs, ge, gl = res["g_sigma"], res["g_eps"], res["g_lnc"]
    h = 1e-6

    def E(dd=d, ee=eps, LL=L):
        e, mixed = un.final_energy(R, LL, ss(dd, ee), sp, K)
        assert np.array_equal(mixed, res["traj"]["mixed"])
        return e

    scale = abs(res["E"]) + 1e-3
    for s in range(2):
        dp, dm = d.copy(), d.copy()
        dp[s] += h
        dm[s] -= h
        fd = (E(dd=dp) - E(dd=dm)) / (2 * h)
        g = 0.5 * (gs[s].sum() + gs[:, s].sum())
        assert g == pytest.approx(fd, rel=1e-5, abs=1e-7 * scale), ("d", s)
    for q, (a, b) in enumerate(((0, 0), (0, 1), (1, 1))):
        ep, em = list(eps), list(eps)
        ep[q] += h
        em[q] -= h
        fd = (E(ee=ep) - E(ee=em)) / (2 * h)
        g = ge[a, b] + (ge[b, a] if a != b else 0.0)
        assert g == pytest.approx(fd, rel=1e-5, abs=1e-7 * scale), ("eps", a, b)
    fd = (E(LL=L * math.exp(h)) - E(LL=L * math.exp(-h))) / (2 * h)
    assert gl == pytest.approx(fd, rel=1e-5, abs=1e-7 * scale)


def test_unrolled_grad_initial_positions_match_fd(un):
    N, K = 20, 40
    R, L, sp = packing(N, 0.9, 61)
    pot = ss()
    res = un.fire_unrolled_grad(R, L, pot, sp, K)
    rng = np.random.default_rng(9)
    for _ in range(3):
        z = rng.standard_normal(R.shape)
        h = 1e-8
        ep, mp = un.final_energy(R + h * z, L, pot, sp, K)
        em, mm = un.final_energy(R - h * z, L, pot, sp, K)
        assert np.array_equal(mp, mm)
        fd = (ep - em) / (2 * h)
        assert (res["Rbar0"] * z).sum() == pytest.approx(fd, rel=1e-5, abs=1e-8)


def test_unrolled_grad_tends_to_envelope_at_convergence(un):
    """Run long enough that FIRE has converged inside the fixed K steps: dE_K/dtheta approaches the envelope
    derivative dU/dtheta at the minimum (Sec. 4.2 obtains dE*/dtheta either way)."""
    import oracle
    N = 16
    R, L, sp = packing(N, 0.8, 71)
    pot = ss()
    K = 2500
    res = un.fire_unrolled_grad(R, L, pot, sp, K)
    RK = res["traj"]["R"][K]
    fmax = np.sqrt((res["traj"]["F"][K] ** 2).sum(1)).max() / L[0]
    assert fmax < 1e-9
    g_env = oracle.diameter_grad(RK * L, L, [1.0, 1.4], 1.0, sp)
    g_unr = 0.5 * (res["g_sigma"].sum(1) + res["g_sigma"].sum(0))
    assert np.allclose(g_unr, g_env, rtol=1e-6, atol=1e-9)
    _, _, _, gl_env = un.energy_grads(RK, L, pot, sp)
    assert res["g_lnc"] == pytest.approx(gl_env, rel=1e-6, abs=1e-9)
