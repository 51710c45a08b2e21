"""Pins of the FP64 flocking model (oracle/flocking.py): every gradient against central differences of the
energy terms it belongs to, the reductions of each term, and the behavior the text asks of each rule."""
import math

import numpy as np
import pytest

from paper_1912_04232_amd import inputs


@pytest.fixture(scope="module")
def fl():
    from oracle import flocking
    return flocking


def flock(N, L, seed):
    rng = np.random.default_rng(seed)
    R = inputs.uniform_torus(N, 2, seed).astype(np.float64) * (np.array(L) / 2.0 ** 32)
    return R, rng.uniform(-math.pi, math.pi, N)


def test_gradients_match_finite_differences(fl):
    p = fl.FlockParams()
    L = [14.0, 12.0]
    R, th = flock(60, L, 3)
    C, D = np.array([[4.0, 5.0], [10.0, 9.0]]), np.array([2.5, 1.5])
    gR, gT = fl.gradients(R, th, L, p, C, D)
    rng = np.random.default_rng(1)
    h = 1e-6
    for _ in range(3):
        zR = rng.standard_normal(R.shape)
        zT = rng.standard_normal(th.shape)

        def E_pos(RR):   # the alignment term's position gradient is stopped
            t = fl.energy_terms(RR, th, L, p, C, D)
            return t[1] + t[2] + t[3]

        def E(TT):
            return sum(fl.energy_terms(R, TT, L, p, C, D))
        fdR = (E_pos(R + h * zR) - E_pos(R - h * zR)) / (2 * h)
        fdT = (E(th + h * zT) - E(th - h * zT)) / (2 * h)
        assert (gR * zR).sum() == pytest.approx(fdR, rel=1e-6, abs=1e-9)
        assert (gT * zT).sum() == pytest.approx(fdT, rel=1e-6, abs=1e-9)


def test_terms_reduce_to_their_definitions(fl):
    """Two boids at distance r: avoid = J rho(r; R_avoid) (one pair), align = J rho (1 - cos dtheta)^2; each boid's
    neighbor center of mass is the other boid."""
    p = fl.FlockParams()
    L = [50.0, 50.0]
    R = np.array([[10.0, 10.0], [10.6, 10.0]])
    th = np.array([0.3, 1.1])
    e_al, e_av, e_co, e_ob = fl.energy_terms(R, th, L, p)
    r = 0.6
    assert math.isclose(e_av, p.J_avoid * (1 - r / p.R_avoid) ** p.alpha / p.alpha, rel_tol=1e-13)
    assert math.isclose(e_al, p.J_align * (1 - r / p.R_align) ** p.alpha / p.alpha * (1 - math.cos(0.8)) ** 2,
                        rel_tol=1e-13)
    # boid 0 sees boid 1 along +x, boid 1 sees boid 0 along -x
    want = 0.5 * p.J_coh * ((1 - math.cos(0.3)) ** 2 + (1 + math.cos(1.1)) ** 2)
    assert math.isclose(e_co, want, rel_tol=1e-13)
    assert e_ob == 0.0


def test_rules_have_their_minima_where_the_text_says(fl):
    p = fl.FlockParams()
    L = [50.0, 50.0]
    # alignment: zero for parallel headings
    R = np.array([[10.0, 10.0], [11.0, 10.0]])
    assert fl.energy_terms(R, np.array([0.7, 0.7]), L, p)[0] == pytest.approx(0.0, abs=1e-15)
    # cohesion: zero when each boid points at its neighbors' center of mass
    assert fl.energy_terms(R, np.array([0.0, math.pi]), L, p)[2] == pytest.approx(0.0, abs=1e-15)
    # obstacle: zero facing away from the obstacle, largest facing it
    C, D = np.array([[10.0, 10.0]]), np.array([2.0])
    Rb = np.array([[11.0, 10.0]])
    away = fl.energy_terms(Rb, np.array([0.0]), L, p, C, D)[3]
    toward = fl.energy_terms(Rb, np.array([math.pi]), L, p, C, D)[3]
    assert away == pytest.approx(0.0, abs=1e-15) and toward > 0.0
    # outside every range nothing interacts
    Rf = np.array([[10.0, 10.0], [20.0, 10.0]])
    assert sum(fl.energy_terms(Rf, np.array([0.0, 2.0]), L, p)) == 0.0


def test_step_is_forward_euler(fl):
    p = fl.FlockParams()
    L = [14.0, 12.0]
    R, th = flock(40, L, 5)
    gR, gT = fl.gradients(R, th, L, p)
    R1, th1 = fl.step(R, th, L, p)
    N = np.stack([np.cos(th), np.sin(th)], 1)
    want = R + p.dt * (p.v * N - gR)
    d = R1 - want
    d -= np.array(L) * np.round(d / np.array(L))
    assert np.abs(d).max() < 1e-12 and np.allclose(th1, th - p.dt * gT, rtol=0, atol=1e-14)


def test_predator_gradients_match_finite_differences(fl):
    """Each side's gradient against central differences of its own energy: the boids' flee term in boid positions
    and headings, the predators' chase + obstacle energy in predator positions and headings."""
    p, q = fl.FlockParams(), fl.PredatorParams()
    L = [20.0, 18.0]
    R, th = flock(80, L, 5)
    Rp, thp = flock(3, L, 6)
    C, D = np.array([[4.0, 5.0], [14.0, 9.0]]), np.array([2.5, 3.5])
    gR, gT, gRp, gTp = fl.predator_gradients(R, th, Rp, thp, L, p, q, C, D)
    assert np.abs(gRp).max() > 0 and np.abs(gR).max() > 0
    rng = np.random.default_rng(2)
    h = 1e-6
    for _ in range(3):
        z = rng.standard_normal(R.shape), rng.standard_normal(th.shape)
        zp = rng.standard_normal(Rp.shape), rng.standard_normal(thp.shape)

        def Eb(RR, TT):
            return fl.predator_terms(RR, TT, Rp, thp, L, p, q, C, D)[0]

        def Ep(RR, TT):
            t = fl.predator_terms(R, th, RR, TT, L, p, q, C, D)
            return t[1] + t[2]
        fd_b = (Eb(R + h * z[0], th + h * z[1]) - Eb(R - h * z[0], th - h * z[1])) / (2 * h)
        fd_p = (Ep(Rp + h * zp[0], thp + h * zp[1]) - Ep(Rp - h * zp[0], thp - h * zp[1])) / (2 * h)
        assert (gR * z[0]).sum() + (gT * z[1]).sum() == pytest.approx(fd_b, rel=1e-6, abs=1e-9)
        assert (gRp * zp[0]).sum() + (gTp * zp[1]).sum() == pytest.approx(fd_p, rel=1e-6, abs=1e-9)


def test_predator_terms_closed_forms(fl):
    """One predator and one boid 2 apart along x: the predator's chase energy is 1/2 J (1 - cos theta_p)^2 (its
    neighbors' center of mass is the boid) with d/dtheta_p = J (1 - cos) sin; the boid's flee term vanishes when
    it faces straight away from the predator and is 4 J rho(2; R_flee) when it faces the predator."""
    p, q = fl.FlockParams(), fl.PredatorParams()
    L = [50.0, 50.0]
    Rp, R = np.array([[20.0, 20.0]]), np.array([[22.0, 20.0]])
    for thp in (0.0, 0.7, -2.0):
        _, e_ch, _ = fl.predator_terms(R, np.array([0.0]), Rp, np.array([thp]), L, p, q)
        assert math.isclose(e_ch, 0.5 * q.J_chase * (1 - math.cos(thp)) ** 2, rel_tol=1e-13, abs_tol=1e-15)
        gTp = fl.predator_gradients(R, np.array([0.0]), Rp, np.array([thp]), L, p, q)[3]
        assert math.isclose(gTp[0], q.J_chase * (1 - math.cos(thp)) * math.sin(thp), rel_tol=1e-12, abs_tol=1e-15)
    e_away = fl.predator_terms(R, np.array([0.0]), Rp, np.array([0.0]), L, p, q)[0]
    e_toward = fl.predator_terms(R, np.array([math.pi]), Rp, np.array([0.0]), L, p, q)[0]
    assert e_away == pytest.approx(0.0, abs=1e-15)
    assert e_toward == pytest.approx(4 * q.J_flee * (1 - 2 / q.R_flee) ** p.alpha / p.alpha, rel=1e-13)


def test_predators_out_of_range_leave_the_flock_alone(fl):
    """With every predator farther than R_flee and R_chase from every boid, the boids step exactly as without
    predators, and each predator swims straight (no obstacle in reach)."""
    p, q = fl.FlockParams(), fl.PredatorParams()
    L = [60.0, 60.0]
    R, th = flock(40, [20.0, 20.0], 7)
    Rp, thp = np.array([[45.0, 45.0], [50.0, 35.0]]), np.array([0.4, 2.0])
    R1, t1 = fl.step(R, th, L, p, n_steps=3)
    R2, t2, Rp2, thp2 = fl.step_with_predators(R, th, Rp, thp, L, p, q, n_steps=3)
    assert np.allclose(R1, R2, rtol=0, atol=1e-13) and np.allclose(t1, t2, rtol=0, atol=1e-13)
    want = Rp + 3 * p.dt * q.v * np.stack([np.cos(thp), np.sin(thp)], 1)
    assert np.allclose(Rp2, want, atol=1e-12) and np.array_equal(thp2, thp)
