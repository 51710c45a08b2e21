"""Flocking (Sec. 4.3, App. B) on the GPU against the FP64 oracle (oracle/flocking.py) on the same seeded boids:
gradients and steps at a size the all-pairs oracle finishes quickly, sampled boids at the 65536-boid size, graph
replay against eager launches."""
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
def fl():
    from oracle import flocking
    return flocking


def positions(u, L):
    return np.asarray(u, np.uint32).astype(np.float64) * (float(L) / 4294967296.0)


def image_diff(a, b, L):
    d = a - b
    d -= L * np.rint(d / L)
    return np.abs(d)


def cohesion_dn(x, L, R_coh):
    """|dR_i|, the length of each boid's mean displacement to its neighbors within R_coh (inf without any): the
    cohesion gradient goes as 1/|dR_i| and its float32 rounding error as 1/|dR_i|^2, so it sets the tolerance."""
    d = x[None, :, :] - x[:, None, :]
    d -= L * np.rint(d / L)
    m = (d * d).sum(-1) < R_coh * R_coh
    np.fill_diagonal(m, False)
    n = m.sum(1)
    dR = (d * m[..., None]).sum(1) / np.maximum(n, 1)[:, None]
    return np.where(n > 0, np.sqrt((dR * dR).sum(1)), np.inf)


def grad_err(w, gR, gT, dn, J_coh, scale):
    """Largest |GPU - oracle| over boids, each divided by its bound: 2e-5 of the largest gradient plus the float32
    error of the cohesion direction, about 3e-6 J_coh / |dR_i|^2 (positions rounded to 6e-8 relative, summed over
    the neighbors)."""
    e = np.maximum(np.abs(w[:, 0] - gR[:, 0]), np.abs(w[:, 1] - gR[:, 1]))
    e = np.maximum(e, np.abs(w[:, 2] - gT))
    return float((e / (2e-5 * scale + 3e-6 * J_coh / np.minimum(dn, 1e6) ** 2)).max())


def oracle_params(fl, md, flock):
    # the parameters as the kernels see them (float32)
    return fl.FlockParams(**{k: float(np.float32(v)) for k, v in flock.params.items()})


def make(md, N, L, seed, n_obstacles, params=None, capacity=None, lanes=4):
    u, theta, obs = inputs.boids(N, L, seed, n_obstacles)
    f = md.Flock(md.Box((L, L), 2), u, theta, params, obs, capacity=capacity, lanes=lanes)
    return f, u, theta.astype(np.float64), obs.astype(np.float64)


@pytest.mark.parametrize("lanes", [1, 4, 8])
def test_flock_gradients_and_steps_match_oracle(md, fl, lanes):
    """2000 boids at density 0.5 with 4 obstacles, 1, 4 or 8 GPU lanes per boid: the gradients of the first step
    (work array) and the state after 1 and 4 steps."""
    L = 64.0
    f, u, theta, obs = make(md, 2000, L, 17, 4, lanes=lanes)
    p = oracle_params(fl, md, f)
    init, update = md.flocking(f)
    init()
    update(1)
    gR, gT = fl.gradients(positions(u, L), theta, np.array([L, L]), p, obs[:, :2], obs[:, 2])
    w = f.work.cpu().numpy().astype(np.float64)
    scale = max(np.abs(gR).max(), np.abs(gT).max())
    e = grad_err(w, gR, gT, cohesion_dn(positions(u, L), L, p.R_coh), p.J_coh, scale)
    say("gradient err / bound", e, "scale", scale)
    assert e < 1.0
    R, T = positions(u, L), theta
    done = 0
    for n in (1, 3):
        if done:
            update(n)
        R, T = fl.step(R, T, np.array([L, L]), p, obs[:, :2], obs[:, 2], n_steps=n)
        done += n
        dR = image_diff(positions(md.from_device_u32(f.pos), L), R, L).max()
        dT = np.abs(f.theta.cpu().numpy().astype(np.float64) - T).max()
        say("steps", done, "dR", dR, "dtheta", dT)
        # one step moves a boid by dt times its gradient (up to about 0.05 * 25); rounding differences grow
        # through the stiff avoidance term and the cohesion neighbor sets, so the state is held to 1e-3
        assert dR < 1e-3 and dT < 1e-3


def test_flock_without_obstacles_and_cohesion_only(md, fl):
    """Each term alone against the oracle: cohesion only (no avoidance, alignment or obstacles), then avoidance
    and alignment only; a boid with no neighbor in range moves straight at speed v."""
    L = 48.0
    for params in ({"J_align": 0.0, "J_avoid": 0.0, "J_obs": 0.0},
                   {"J_coh": 0.0, "J_obs": 0.0}):
        f, u, theta, obs = make(md, 900, L, 23, 0, params)
        p = oracle_params(fl, md, f)
        init, update = md.flocking(f)
        init()
        update(1)
        gR, gT = fl.gradients(positions(u, L), theta, np.array([L, L]), p)
        w = f.work.cpu().numpy().astype(np.float64)
        scale = max(np.abs(gR).max(), np.abs(gT).max())
        e = grad_err(w, gR, gT, cohesion_dn(positions(u, L), L, p.R_coh), p.J_coh, scale)
        say(params, "err / bound", e, "scale", scale)
        assert scale > 0 and e < 1.0
    # a lone boid: no neighbor, no obstacle: R += dt v N, theta unchanged
    u = np.array([[0, 0], [2 ** 31, 2 ** 31]], np.uint32)
    f = md.Flock(md.Box((L, L), 2), u, np.array([0.3, -2.0], np.float32))
    init, update = md.flocking(f)
    init()
    update(1)
    R = positions(md.from_device_u32(f.pos), L)
    exp = positions(u, L) + 0.05 * np.stack([np.cos([0.3, -2.0]), np.sin([0.3, -2.0])], 1)
    assert image_diff(R, exp, L).max() < 1e-5
    assert np.array_equal(f.theta.cpu().numpy(), np.array([0.3, -2.0], np.float32))


def test_flock_sampled_boids_at_full_size(md, fl):
    """65536 boids in a 512 x 512 box with 16 obstacles (the measured workload): the first step's gradients of
    sampled boids against the oracle on each sample's local patch (every boid within 6.5 of it, unwrapped around
    it: the gradient of a boid depends on boids within 2 R_coh)."""
    L, N = 512.0, 65536
    f, u, theta, obs = make(md, N, L, 29, 16)
    p = oracle_params(fl, md, f)
    init, update = md.flocking(f)
    init()
    update(1)
    w = f.work.cpu().numpy().astype(np.float64)
    x = positions(u, L)
    rng = np.random.Generator(np.random.PCG64(5))
    worst = 0.0
    for i in rng.choice(N, 64, replace=False):
        d = x - x[i]
        d -= L * np.rint(d / L)
        near = np.where((d * d).sum(1) < 6.5 ** 2)[0]
        k = int(np.where(near == i)[0][0])
        c = obs[:, :2] - x[i]
        c -= L * np.rint(c / L)
        big = np.array([1e6, 1e6])
        gR, gT = fl.gradients(d[near] + 5e5, theta[near], big, p, c + 5e5, obs[:, 2])
        dn = cohesion_dn(d[near], 1e6, p.R_coh)[k: k + 1]
        e = grad_err(w[i: i + 1], gR[k: k + 1], gT[k: k + 1], dn, p.J_coh, 25.0)
        worst = max(worst, e)
    say("sampled worst err / bound", worst)
    assert worst < 1.0


def test_flock_graph_replay_matches_eager(md):
    """120 steps (several device-decided list rebuilds) replayed from HIP graphs equal the same steps launched
    eagerly, bit for bit (rows with room for any clumping, so that no regrow moves a rebuild)."""
    import torch
    L = 64.0
    a = make(md, 2000, L, 31, 2, capacity=400)[0]
    b = make(md, 2000, L, 31, 2, capacity=400)[0]
    ia, ua = md.flocking(a)
    ib, ub = md.flocking(b)
    ia()
    ib()
    for _ in range(3):
        ua(40, graph=True)
        ub(40, graph=False)
        torch.cuda.synchronize()
        assert torch.equal(a.pos, b.pos) and torch.equal(a.theta, b.theta)
    assert a.last_flags[md.FLAG_REBUILDS] > 0 and a.nl.capacity == 400


def test_flock_regrow_rebuilds_before_the_rerun(md):
    """Rows that outgrow the list during a run: the run is repeated from its start with a larger list built for
    the restored state, and ends bit for bit where a run whose list never overflowed ends (the same rebuild
    steps, the same row order)."""
    import torch
    L = 40.0
    clump = {"J_avoid": 0.0, "J_coh": 2.0, "J_align": 0.2}   # boids gather: the longest row grows from 60 to ~95
    u, theta, _ = inputs.boids(1600, L, 37, 0)
    a = md.Flock(md.Box((L, L), 2), u, theta, clump, capacity=400, max_per_cell=252)
    b = md.Flock(md.Box((L, L), 2), u, theta, clump, max_per_cell=252)
    ia, ua = md.flocking(a)
    ib, ub = md.flocking(b)
    ia()
    ib()
    W = b.nl.lanes
    tight = (int(b.nl.lengths().max()) + W - 1) // W * W
    b.nl = md.NeighborList(b.N, 2, tight, b.nl.r_list, b.nl.skin, b.ctx.device, b.nl.max_per_cell, W)
    b.build()
    assert b.nl.capacity == tight and a.nl.lanes == W
    ua(60)
    ub(60)
    torch.cuda.synchronize()
    say("capacity", tight, "->", b.nl.capacity, "max row", int(a.nl.lengths().max()))
    assert b.nl.capacity > tight
    assert torch.equal(a.pos, b.pos) and torch.equal(a.theta, b.theta)


def make_with_predators(md, N, L, seed, n_obstacles, P, lanes=4):
    u, theta, obs = inputs.boids(N, L, seed, n_obstacles)
    up, thp, _ = inputs.boids(P, L, seed + 100, 0)
    f = md.Flock(md.Box((L, L), 2), u, theta, None, obs, lanes=lanes, predators=(up, thp))
    return f, u, theta.astype(np.float64), obs.astype(np.float64), up, thp.astype(np.float64)


def test_flock_with_predators_matches_oracle(md, fl):
    """1500 boids, 2 obstacles and 4 predators (App. B's two-player game): the boids' gradients of the first step
    (flee term included), the predators after one step, and both sides after 4 steps."""
    L = 56.0
    f, u, theta, obs, up, thp = make_with_predators(md, 1500, L, 47, 2, 4)
    p = oracle_params(fl, md, f)
    q = fl.PredatorParams(**{k: float(np.float32(v)) for k, v in f.predator_params.items()})
    init, update = md.flocking(f)
    init()
    update(1)
    x, xp, LL = positions(u, L), positions(up, L), np.array([L, L])
    gR, gT = fl.gradients(x, theta, LL, p, obs[:, :2], obs[:, 2])
    fR, fT, _, _ = fl.predator_gradients(x, theta, xp, thp, LL, p, q, obs[:, :2], obs[:, 2])
    w = f.work.cpu().numpy().astype(np.float64)
    scale = max(np.abs(gR + fR).max(), np.abs(gT + fT).max())
    e = grad_err(w, gR + fR, gT + fT, cohesion_dn(x, L, p.R_coh), p.J_coh, scale)
    say("boid gradient err / bound", e, "flee part", np.abs(fR).max())
    assert e < 1.0 and np.abs(fR).max() > 0
    R, T, Rp, Tp = x, theta, xp, thp
    done = 0
    for n in (1, 3):
        if done:
            update(n)
        R, T, Rp, Tp = fl.step_with_predators(R, T, Rp, Tp, LL, p, q, obs[:, :2], obs[:, 2], n_steps=n)
        done += n
        dR = image_diff(positions(md.from_device_u32(f.pos), L), R, L).max()
        dT = np.abs(f.theta.cpu().numpy().astype(np.float64) - T).max()
        dRp = image_diff(positions(md.from_device_u32(f.ppos), L), Rp, L).max()
        dTp = np.abs(f.ptheta.cpu().numpy().astype(np.float64) - Tp).max()
        say("steps", done, "boids dR", dR, "dtheta", dT, "predators dR", dRp, "dtheta", dTp)
        if done == 1:
            assert dRp < 1e-5 and dTp < 1e-5
        assert dR < 1e-3 and dT < 1e-3 and dRp < 1e-3 and dTp < 1e-3


def test_flock_with_predators_graph_replay_matches_eager(md):
    import torch
    L = 56.0
    a = make_with_predators(md, 1500, L, 53, 2, 4)[0]
    b = make_with_predators(md, 1500, L, 53, 2, 4)[0]
    ia, ua = md.flocking(a)
    ib, ub = md.flocking(b)
    ia()
    ib()
    for _ in range(2):
        ua(40, graph=True)
        ub(40, graph=False)
        torch.cuda.synchronize()
        assert torch.equal(a.pos, b.pos) and torch.equal(a.theta, b.theta)
        assert torch.equal(a.ppos, b.ppos) and torch.equal(a.ptheta, b.ptheta)


def test_flock_step_without_boids_moves_predators_like_the_oracle(md, fl):
    """N = 0: the call succeeds with empty (NULL) boid arrays; a predator still swims at its speed and descends its
    obstacle terms (its chase sums are empty), as the oracle's two-player step does with no boids."""
    import torch
    ctx = md.Context()
    L = 32.0
    box = md.Box((L, L), 2)
    nl = md.NeighborList(0, 2, 8, 3.5, 0.5, ctx.device, 8, 4)
    fp = md.c_flock_params(**{k: float(v) for k, v in md.FLOCK_DEFAULTS.items()})
    # one obstacle of radius 5 centred 2 units from the predator, so the obstacle term acts
    fp.n_obstacles = 1
    u0 = np.array([[1 << 31, 1 << 30]], dtype=np.uint32)
    x0 = positions(u0, L)
    fp.obstacles[0:3] = (float(x0[0, 0] + 2.0), float(x0[0, 1] + 1.0), 5.0)
    up = md.to_device_u32(u0, ctx.device)
    thp = torch.tensor([0.5], dtype=torch.float32, device=ctx.device)
    pred = md.c_flock_predators(P=1, **{k: float(v) for k, v in md.PREDATOR_DEFAULTS.items()})
    pred.pos, pred.theta = up.data_ptr(), thp.data_ptr()
    empty_u = torch.empty((0, 2), dtype=torch.int32, device=ctx.device)
    empty_f = torch.empty(0, dtype=torch.float32, device=ctx.device)
    md.flock_step(ctx, box, empty_u, empty_f, nl, fp, torch.empty((0, 8), device=ctx.device), pred)
    torch.cuda.synchronize()
    p = fl.FlockParams(**{k: float(np.float32(v)) for k, v in md.FLOCK_DEFAULTS.items()})
    q = fl.PredatorParams(**{k: float(np.float32(v)) for k, v in md.PREDATOR_DEFAULTS.items()})
    obs = np.array([fp.obstacles[0:3]], dtype=np.float64)
    _, _, Rp, Tp = fl.step_with_predators(np.zeros((0, 2)), np.zeros(0), x0, np.array([0.5]), np.array([L, L]), p, q,
                                          obs[:, :2], obs[:, 2])
    got = positions(md.from_device_u32(up), L)
    moved = image_diff(got, x0, L).max()
    say("predator moved", moved, "dR", image_diff(got, Rp, L).max(), "dtheta", abs(float(thp[0]) - Tp[0]))
    assert moved > 0.01
    assert image_diff(got, Rp, L).max() < 1e-5 and abs(float(thp[0]) - Tp[0]) < 1e-5


def test_flock_alpha_one_matches_oracle(md, fl):
    """alpha = 1 (the cutoff function is linear): t^(alpha - 1) = 1 even where t rounds to 0, no NaN reaches the
    positions; gradients of the first step and the state after one step against the oracle."""
    L = 48.0
    f, u, theta, obs = make(md, 900, L, 31, 2, {"alpha": 1.0})
    p = oracle_params(fl, md, f)
    init, update = md.flocking(f)
    init()
    update(1)
    gR, gT = fl.gradients(positions(u, L), theta, np.array([L, L]), p, obs[:, :2], obs[:, 2])
    w = f.work.cpu().numpy().astype(np.float64)
    assert np.isfinite(w).all()
    scale = max(np.abs(gR).max(), np.abs(gT).max())
    e = grad_err(w, gR, gT, cohesion_dn(positions(u, L), L, p.R_coh), p.J_coh, scale)
    say("alpha 1: gradient err / bound", e)
    assert e < 1.0
    R, T = fl.step(positions(u, L), theta, np.array([L, L]), p, obs[:, :2], obs[:, 2])
    dR = image_diff(positions(md.from_device_u32(f.pos), L), R, L).max()
    assert dR < 1e-3
