"""The Buckingham (exponential-six) pair potential through the list, dense, W-lane, half-list and fused-step paths
against the FP64 oracle (two species, a third coefficient matrix for the dispersion term)."""
import math
import sys

import numpy as np
import pytest

from paper_1912_04232_amd import inputs

pytestmark = pytest.mark.gpu

A = np.array([[2.6e5, 2.0e5], [2.0e5, 1.6e5]])      # repulsion strength
RHO = np.array([[0.08, 0.085], [0.085, 0.09]])       # repulsion range
C = np.array([[1.0, 1.2], [1.2, 1.4]])               # dispersion coefficient
R_CUT = 2.6


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


def rel_l2(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def case(md, orc, N=1500, seed=171, shift=True, T=0.5):
    """Random insertion at density 0.8 with no pair closer than 0.9 (the repulsive wall), Maxwell velocities."""
    L = inputs.box_for_density(N, 0.8)
    u = inputs.random_insertion_torus(N, L, 3, 0.9, seed)
    v = inputs.maxwell_velocities(N, 3, T, seed + 1)
    sp = (np.arange(N) % 2).astype(np.int32)
    mpot = md.Potential("buckingham", RHO, A, r_cut=R_CUT, shift=shift, coef=C)
    opot = orc.Potential("buckingham", RHO, A, r_cut=R_CUT, shift=shift, coef=C)
    s = md.System(md.Box((L, L, L), 3), mpot, u, v, sp, skin=0.3)
    return s, opot, u, v, sp, np.array([L, L, L])


@pytest.mark.parametrize("shift", [True, False])
def test_buckingham_forces_energies_list_and_dense(md, orc, shift):
    import torch
    s, opot, u, v, sp, L = case(md, orc, shift=shift)
    s.build()
    e, w = s.forces(energy=True)
    x = u.astype(np.float64) * (L / 2.0 ** 32)
    Fo, eo, wo = orc.pair_rows(x, L, opot, sp)
    say("shift", shift, "force rel-L2", rel_l2(s.force.cpu().numpy(), Fo))
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


def test_buckingham_verlet_steps_and_energy_scaling(md, orc):
    """Fused velocity-Verlet steps against the oracle's after 1 and 4 steps; then the total-energy spread over 4
    time units at dt = 0.004 and dt = 0.002 from the same state shrinks with dt^2."""
    s, opot, u, v, sp, L = case(md, orc, seed=181)
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
    state = [t.clone() for t in (s.pos, s.vel, s.force)]
    spread = {}
    for dt, n in ((0.004, 100), (0.002, 200)):
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
    assert spread[0.004] < 1e-3 * s.N
    assert spread[0.004] / spread[0.002] > 2.5, spread


def test_buckingham_half_list_matches_oracle(md, orc):
    import torch
    s, opot, u, v, sp, L = case(md, orc, seed=191)
    s.build()
    h = md.HalfList(s.ctx, s.nl)
    h.update()
    F = torch.zeros_like(s.force)
    h.forces(s.box, s.pot, s.pos, s.species, F)
    x = u.astype(np.float64) * (L / 2.0 ** 32)
    Fo, _, _ = orc.pair_rows(x, L, opot, sp)
    assert int(h.overflow.item()) == 0
    assert rel_l2(F.cpu().numpy(), Fo) <= 1e-5


def test_replica_paths_refuse_buckingham(md):
    reps = [dict(N=16, L=np.array([6.0, 6.0, 0.0]), u=inputs.uniform_torus(16, 2, 1), species=None)]
    ctx = md.Context()
    pot = md.Potential("buckingham", [[0.08]], [[2.6e5]], r_cut=2.5, coef=[[1.0]])
    with pytest.raises(md.MDError):
        md.fire_batched(ctx, md.Batch(reps), pot, md.FireParams(), 10, 1e-6)
    with pytest.raises(md.MDError):
        md.envelope_grad(ctx, md.Batch(reps), pot)
    with pytest.raises(md.MDError):
        md.fire_unrolled_grad(ctx, md.Batch(reps), pot, md.FireParams(), 5)
