"""Constant-temperature steps and gradient descent on the GPU against the FP64 oracle (oracle/thermostats.py) on
the same seeded inputs, plus the statistics each scheme is built for."""
import math
import sys

import numpy as np
import pytest

from paper_1912_04232_amd import inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def md():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_1912_04232_amd import md as m
    m.load()
    return m


@pytest.fixture(scope="module")
def th():
    from oracle import thermostats
    return thermostats


def rel_l2(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def torus_x(u, L):
    return np.asarray(u, np.uint32).astype(np.float64) * (np.asarray(L, np.float64)[: u.shape[1]] / 4294967296.0)


def max_image_diff(a, b, L):
    L = np.asarray(L, np.float64)[: a.shape[1]]
    d = a - b
    d -= L * np.rint(d / L)
    return float(np.abs(d).max())


def soft_case(md, orc, N=500, phi=0.85, seed=61, T=0.2):
    L = inputs.box_for_packing([1.0, 1.4], [N // 2, N - N // 2], phi, 2)
    d = np.array([1.0, 1.4])
    sig = 0.5 * (d[:, None] + d[None, :])
    u = inputs.uniform_torus(N, 2, seed)
    v = inputs.maxwell_velocities(N, 2, T, seed + 1)
    sp = inputs.bidisperse_species(N)
    sysm = md.System(md.Box((L, L), 2), md.Potential("soft_sphere", sig, np.ones((2, 2)), alpha=2.0), u, v, sp,
                     skin=0.3)
    return sysm, orc.Potential("soft_sphere", sig, np.ones((2, 2)), alpha=2.0), u, v, sp, np.array([L, L])


def lj_case(md, orc, N=1500, seed=71, T=1.0):
    L = inputs.box_for_density(N, 0.8)
    u = inputs.random_insertion_torus(N, L, 3, 0.85, seed)
    v = inputs.maxwell_velocities(N, 3, T, seed + 1)
    sysm = md.System(md.Box((L, L, L), 3), md.Potential("lj", [[1.0]], [[1.0]], r_cut=2.5), u, v, skin=0.3)
    return sysm, orc.Potential("lj", np.ones((1, 1)), np.ones((1, 1)), r_cut=2.5), u, v, None, np.array([L, L, L])


@pytest.mark.parametrize("case", ["soft2d", "lj3d"])
def test_langevin_steps_match_oracle(md, orc, th, case):
    s, opot, u, v, sp, L = (soft_case if case == "soft2d" else lj_case)(md, orc)
    dt, gamma, kT, seed = (0.01, 1.0, 0.3, 5) if case == "soft2d" else (0.004, 2.0, 1.2, 6)
    init, update = md.nvt_langevin(s, dt, gamma, kT, seed)
    init()
    x = torus_x(u, L)
    F, _, _ = orc.pair_rows(x, L, opot, sp)
    xv = v.astype(np.float64)
    done = 0
    for n in (1, 4):
        update(n)
        x, xv, F = th.langevin_baoab(x, xv, F, L, opot, sp, dt, gamma, kT, seed, done, n)
        done += n
        dx = max_image_diff(torus_x(md.from_device_u32(s.pos), L), x, L)
        ev, ef = rel_l2(s.vel.cpu().numpy(), xv), rel_l2(s.force.cpu().numpy(), F)
        say(case, "steps", done, "dx", dx, "v", ev, "F", ef)
        assert dx < 1e-5 and ev < 1e-5 and ef < 1e-4


@pytest.mark.parametrize("case", ["soft2d", "lj3d"])
def test_fused_langevin_steps_match_oracle(md, orc, th, case):
    """langevin_run (the Verlet step kernel with the BAOAB drift, the list rebuilt inside the run) against the
    oracle's BAOAB from the same seeded state and noise: 1, then 4, then 10 more steps."""
    s, opot, u, v, sp, L = (soft_case if case == "soft2d" else lj_case)(md, orc)
    dt, gamma, kT, seed = (0.01, 1.0, 0.3, 5) if case == "soft2d" else (0.004, 2.0, 1.2, 6)
    init, update = md.nvt_langevin(s, dt, gamma, kT, seed, fused=True)
    init()
    x = torus_x(u, L)
    F, _, _ = orc.pair_rows(x, L, opot, sp)
    xv = v.astype(np.float64)
    done = 0
    for n in (1, 4, 10):
        update(n)
        x, xv, F = th.langevin_baoab(x, xv, F, L, opot, sp, dt, gamma, kT, seed, done, n)
        done += n
        dx = max_image_diff(torus_x(md.from_device_u32(s.pos), L), x, L)
        ev, ef = rel_l2(s.vel.cpu().numpy(), xv), rel_l2(s.force.cpu().numpy(), F)
        say(case, "fused steps", done, "dx", dx, "v", ev, "F", ef, "noise step", int(update.step.item()))
        assert int(update.step.item()) == done
        assert dx < 1e-5 and ev < 1e-5 and ef < 1e-4


def test_fused_langevin_equals_composed_steps(md, orc):
    """The fused run and the composed step (BAOA launch, gated rebuild, force pass, closing kick) do the same
    arithmetic per coordinate: from the same state and noise, while neither has rebuilt its list, the two states are
    identical bit for bit; over 300 steps with rebuilds they agree to float rounding of the force sums for the first
    steps and keep the same temperature."""
    import torch
    a, _, _, _, _, L = lj_case(md, orc, N=1500, seed=72)
    b, _, _, _, _, _ = lj_case(md, orc, N=1500, seed=72)
    dt, gamma, kT, seed = 0.004, 2.0, 1.2, 11
    ia, ua = md.nvt_langevin(a, dt, gamma, kT, seed, fused=True)
    ib, ub = md.nvt_langevin(b, dt, gamma, kT, seed)
    ia()
    ib()
    ua(2)
    ub(2)
    fa, fb = a.nl.read_flags(), b.nl.read_flags()
    say("rebuilds in the first 2 steps: fused", int(fa[md.FLAG_REBUILDS]), "composed", int(fb[md.FLAG_REBUILDS]))
    if fa[md.FLAG_REBUILDS] == 0 and fb[md.FLAG_REBUILDS] == 0:
        assert torch.equal(a.pos, b.pos) and torch.equal(a.vel, b.vel) and torch.equal(a.force, b.force)
    ua(298)
    ub(298)
    Ta = a.kinetic_energy() * 2.0 / (3 * a.N)
    Tb = b.kinetic_energy() * 2.0 / (3 * b.N)
    say("kinetic T after 300 steps: fused", Ta, "composed", Tb)
    assert abs(Ta - kT) < 0.1 * kT and abs(Tb - kT) < 0.1 * kT


def test_noise_matches_oracle_generator(md, orc, th):
    """A force-free Brownian step moves each particle by sqrt(2 kT dt / gamma) xi: the displacements give back the
    GPU's normals, which match the oracle's Philox4x64 + Box-Muller values to float32 rounding."""
    import torch
    N, L = 3000, np.array([50.0, 50.0, 50.0])
    u = inputs.uniform_torus(N, 3, 81)
    s = md.System(md.Box(tuple(L), 3), md.Potential("soft_sphere", [[1e-3]], [[1.0]], alpha=2.0), u, skin=0.3)
    s.build()
    s.force.zero_()
    step = torch.tensor([7], dtype=torch.int64, device="cuda")
    a = math.sqrt(2.0 * 0.5 * 0.1 / 1.0)
    md.brownian_step(s.ctx, s.box, s.pos, s.force, s.nl, 0.1, 1.0, 0.5, 12345, step)
    d = torus_x(md.from_device_u32(s.pos), L) - torus_x(u, L)
    d -= L * np.rint(d / L)
    z = th.normals(N, 3, 12345, 7)
    say("max |xi_gpu - xi_oracle|", np.abs(d / a - z).max())
    assert int(step.item()) == 8
    assert np.abs(d / a - z).max() < 2e-5 * max(1.0, np.abs(z).max())


def test_brownian_and_gradient_descent_match_oracle(md, orc, th):
    s, opot, u, v, sp, L = soft_case(md, orc, seed=91)
    dt, gamma, kT, seed = 0.005, 2.0, 0.1, 9
    init, update = md.brownian(s, dt, gamma, kT, seed)
    init()
    x = torus_x(u, L)
    F, _, _ = orc.pair_rows(x, L, opot, sp)
    x, F = th.brownian(x, F, L, opot, sp, dt, gamma, kT, seed, 0, 6)
    update(6)
    dx = max_image_diff(torus_x(md.from_device_u32(s.pos), L), x, L)
    say("brownian dx", dx, "F", rel_l2(s.force.cpu().numpy(), F))
    assert dx < 1e-5 and rel_l2(s.force.cpu().numpy(), F) < 1e-4
    s, opot, u, v, sp, L = soft_case(md, orc, seed=92)
    init, update = md.gradient_descent(s, 0.05)
    init()
    E0 = s.potential_energy()
    x = torus_x(u, L)
    F, _, _ = orc.pair_rows(x, L, opot, sp)
    x, F, U = th.gradient_descent(x, F, L, opot, sp, 0.05, 10)
    update(10)
    dx = max_image_diff(torus_x(md.from_device_u32(s.pos), L), x, L)
    E = s.potential_energy()
    say("gd dx", dx, "E", E, U, "from", E0)
    assert dx < 1e-5 and abs(E - U) <= 1e-6 * abs(U) and E < E0


def test_nose_hoover_steps_match_oracle(md, orc, th):
    s, opot, u, v, sp, L = soft_case(md, orc, seed=101, T=0.5)
    dt, kT, Q = 0.005, 0.8, [1.0, 0.5, 0.5]
    init, update, state = md.nvt_nose_hoover(s, dt, kT, Q)
    init()
    x = torus_x(u, L)
    F, _, _ = orc.pair_rows(x, L, opot, sp)
    xv, p, eta = v.astype(np.float64), None, None
    done = 0
    for n in (1, 9):
        update(n)
        x, xv, F, p, eta, _ = th.nose_hoover(x, xv, F, L, opot, sp, dt, kT, Q, n, p, eta)
        done += n
        st = md.nhc_state_read(state)
        dx = max_image_diff(torus_x(md.from_device_u32(s.pos), L), x, L)
        say("nhc", done, "dx", dx, "v", rel_l2(s.vel.cpu().numpy(), xv), "p", st["p"], p, "eta", st["eta"], eta)
        assert dx < 1e-5 and rel_l2(s.vel.cpu().numpy(), xv) < 1e-5
        assert np.allclose(st["p"], p, rtol=1e-4, atol=1e-6 * np.abs(p).max())
        assert np.allclose(st["eta"], eta, rtol=1e-4, atol=1e-8)


def test_langevin_graph_replay_matches_eager(md, orc):
    """Chunks replayed from a captured HIP graph draw fresh noise each step (device step counter) and give the
    same state bit for bit as the same steps launched eagerly."""
    import torch
    a = soft_case(md, orc, N=2000, seed=111)[0]
    b = soft_case(md, orc, N=2000, seed=111)[0]
    ia, ua = md.nvt_langevin(a, 0.01, 1.0, 0.5, 3)
    ib, ub = md.nvt_langevin(b, 0.01, 1.0, 0.5, 3)
    ia()
    ib()
    for _ in range(3):
        ua(40, graph=True)
        ub(40, graph=False)
        torch.cuda.synchronize()
        assert torch.equal(a.pos, b.pos) and torch.equal(a.vel, b.vel)


def test_langevin_equipartition_and_nose_hoover_conservation(md, orc):
    """Long runs: Langevin holds the kinetic temperature at kT; the Nose-Hoover chain (harmonic disks, whose forces
    are continuous) holds it at kT while its H' stays constant to second order in dt."""
    import torch
    s = lj_case(md, orc, N=2000, seed=121, T=0.5)[0]
    init, update = md.nvt_langevin(s, 0.005, 1.0, 1.4, 17)
    init()
    update(400, graph=True)
    Ts = []
    for _ in range(20):
        update(40, graph=True)
        Ts.append(float((s.vel.double() ** 2).sum()) / (3 * s.N))
    say("langevin <T>", np.mean(Ts))
    assert abs(np.mean(Ts) - 1.4) < 0.03 * 1.4

    def chain_run(dt):
        s = soft_case(md, orc, N=2000, phi=0.85, seed=122, T=0.3)[0]
        kT, Q = 0.5, [10.0, 5.0]
        init, update, state = md.nvt_nose_hoover(s, dt, kT, Q)
        init()

        def H():
            st = md.nhc_state_read(state)
            K = 0.5 * float((s.vel.double() ** 2).sum())
            nf = s.N * 2
            return K + s.potential_energy() + float((st["p"] ** 2 / (2 * st["Q"])).sum()) \
                + nf * kT * st["eta"][0] + kT * st["eta"][1:].sum(), K
        H0, _ = H()
        Hs, Ts = [], []
        for _ in range(30):
            update(int(round(0.4 / dt)), graph=True)
            h, K = H()
            Hs.append(h)
            Ts.append(2 * K / (2 * s.N))
        return max(abs(h - H0) for h in Hs), abs(H0), np.mean(Ts[10:])

    d1, h1, t1 = chain_run(0.01)
    d2, _, t2 = chain_run(0.005)
    say("nhc H drift", d1, d2, "of", h1, "<T> late", t1, t2)
    assert d1 < 1e-3 * h1
    assert 2.5 < d1 / d2 < 6.5
    assert abs(t1 - 0.5) < 0.05 * 0.5 and abs(t2 - 0.5) < 0.05 * 0.5
