"""The Morse pair potential through the list, dense and fused-step paths against the FP64 oracle."""
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


SIG = np.array([[1.12, 1.2], [1.2, 1.3]])
EPS = np.array([[1.0, 0.7], [0.7, 1.4]])


def rel_l2(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def case(md, orc, N=1500, seed=131):
    L = inputs.box_for_density(N, 0.8)
    u = inputs.random_insertion_torus(N, L, 3, 0.9, seed)
    v = inputs.maxwell_velocities(N, 3, 1.0, seed + 1)
    sp = (np.arange(N) % 2).astype(np.int32)
    mpot = md.Potential("morse", SIG, EPS, alpha=5.0, r_cut=2.6, shift=True)
    opot = orc.Potential("morse", SIG, EPS, alpha=5.0, r_cut=2.6, shift=True)
    s = md.System(md.Box((L, L, L), 3), mpot, u, v, sp, skin=0.3)
    return s, opot, u, v, sp, np.array([L, L, L])


def test_morse_forces_energies_list_and_dense(md, orc):
    import torch
    s, opot, u, v, sp, L = case(md, orc)
    s.build()
    e, w = s.forces(energy=True)
    x = u.astype(np.float64) * (L / 2.0 ** 32)
    Fo, eo, wo = orc.pair_rows(x, L, opot, sp)
    say("list F", rel_l2(s.force.cpu().numpy(), Fo), "E", float(e.sum()), eo.sum())
    assert rel_l2(s.force.cpu().numpy(), Fo) <= 1e-5
    assert abs(float(e.sum()) - math.fsum(eo)) <= 1e-6 * math.fsum(np.abs(eo))
    assert abs(float(w.sum()) - math.fsum(wo)) <= 1e-5 * math.fsum(np.abs(wo))
    Fl = s.force.clone()
    s.forces()                                    # forces only: the W-lane pass
    assert rel_l2(s.force.cpu().numpy(), Fl.cpu().numpy()) <= 1e-6
    Fd = torch.zeros_like(s.force)
    ed = torch.zeros(s.N, dtype=torch.float64, device="cuda")
    md.pair_energy_force(s.ctx, s.box, s.pot, s.pos, s.species, None, Fd, ed)
    assert rel_l2(Fd.cpu().numpy(), Fo) <= 1e-5
    assert abs(float(ed.sum()) - math.fsum(eo)) <= 1e-6 * math.fsum(np.abs(eo))


def test_morse_verlet_steps_and_conservation(md, orc):
    s, opot, u, v, sp, L = case(md, orc, seed=141)
    init, update = md.nve(s, 0.004)
    init()
    x = u.astype(np.float64) * (L / 2.0 ** 32)
    F, _, _ = orc.pair_rows(x, L, opot, sp)
    xv = v.astype(np.float64)
    for n in (1, 4):
        update(n)
        x, xv, F = orc.verlet(x, xv, F, L, opot, 0.004, n, sp)
        xg = md.from_device_u32(s.pos).astype(np.float64) * (L / 2.0 ** 32)
        d = xg - x
        d -= L * np.rint(d / L)
        say("verlet", n, np.abs(d).max(), rel_l2(s.vel.cpu().numpy(), xv))
        assert np.abs(d).max() < 1e-5 and rel_l2(s.vel.cpu().numpy(), xv) < 1e-5
        assert rel_l2(s.force.cpu().numpy(), F) < 1e-4
    # the total energy over 8 time units at dt = 0.004 and, from the same state, at dt = 0.002: the spread of the
    # velocity-Verlet energy error shrinks with dt^2 (a force inconsistent with the energy, or a missing pair, would
    # leave an error that does not), and stays below 3e-3 per particle at this stiff, hot state (alpha = 5)
    import torch
    state = [t.clone() for t in (s.pos, s.vel, s.force)]
    spread = {}
    for dt, n in ((0.004, 200), (0.002, 400)):
        for t, v0 in zip((s.pos, s.vel, s.force), state):
            t.copy_(v0)
        s.build()
        init, update = md.nve(s, dt)
        E = []
        for _ in range(10):
            update(n)
            E.append(s.potential_energy() + 0.5 * float((s.vel.double() ** 2).sum()))
        spread[dt] = max(E) - min(E)
        say("dt", dt, "total energy", E[0], "spread", spread[dt])
    assert spread[0.004] < 3e-3 * s.N
    assert spread[0.004] / spread[0.002] > 2.5, spread


def test_replica_paths_refuse_morse(md):
    reps = [dict(N=16, L=np.array([6.0, 6.0, 0.0]), u=inputs.uniform_torus(16, 2, 1), species=None)]
    ctx = md.Context()
    pot = md.Potential("morse", [[1.0]], [[1.0]], alpha=5.0, r_cut=2.5)
    with pytest.raises(md.MDError):
        md.fire_batched(ctx, md.Batch(reps), pot, md.FireParams(), 10, 1e-6)
    with pytest.raises(md.MDError):
        md.envelope_grad(ctx, md.Batch(reps), pot)
    with pytest.raises(md.MDError):
        md.fire_unrolled_grad(ctx, md.Batch(reps), pot, md.FireParams(), 5)


@pytest.mark.parametrize("kind", ["lj", "morse", "soft_sphere"])
def test_half_list_forces_match_full_list_and_oracle(md, orc, kind):
    """Newton's-third-law pass over a half list (each pair in one row): the same forces as the full-list pass and
    the oracle (to
    float rounding; the atomic scatter makes the last bits order-dependent)."""
    import torch
    if kind == "soft_sphere":
        N = 3000
        L = inputs.box_for_packing([1.0, 1.4], [N // 2, N // 2], 0.88, 2)
        d = np.array([1.0, 1.4])
        sig = 0.5 * (d[:, None] + d[None, :])
        u = inputs.uniform_torus(N, 2, 151)
        sp = inputs.bidisperse_species(N)
        mpot = md.Potential("soft_sphere", sig, np.ones((2, 2)), alpha=2.0)
        opot = orc.Potential("soft_sphere", sig, np.ones((2, 2)), alpha=2.0)
        s = md.System(md.Box((L, L), 2), mpot, u, None, sp, skin=0.3)
        Lv = np.array([L, L])
    else:
        s, opot, u, v, sp, Lv = case(md, orc, seed=152)
        if kind == "lj":
            s = md.System(s.box, md.Potential("lj", SIG, EPS, r_cut=2.6), u, v, sp, skin=0.3)
            opot = orc.Potential("lj", SIG, EPS, r_cut=2.6)
    s.build()
    s.forces()
    full = s.force.clone()
    h = md.HalfList(s.ctx, s.nl)
    h.update()
    F = torch.zeros_like(s.force)
    h.forces(s.box, s.pot, s.pos, s.species, F)
    assert int(h.overflow.item()) == 0
    assert int(h.hcount.sum().item()) * 2 == int(s.nl.lengths().sum())
    x = u.astype(np.float64) * (Lv / 2.0 ** 32)
    Fo, _, _ = orc.pair_rows(x, Lv, opot, sp)
    say(kind, "half vs full", rel_l2(F.cpu().numpy(), full.cpu().numpy()), "half vs oracle", rel_l2(F.cpu().numpy(), Fo))
    assert rel_l2(F.cpu().numpy(), full.cpu().numpy()) <= 1e-5
    assert rel_l2(F.cpu().numpy(), Fo) <= 1e-5
