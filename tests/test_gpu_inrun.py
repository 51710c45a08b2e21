"""The benchmarked velocity-Verlet path through its device-side rebuilds, against the FP64 oracle.

Inside a verlet_step call the list is rebuilt on the device (bins refreshed from the previous bins, rows of a
second list generation built from them) whenever a particle gets close to moving skin/2.  These tests run that
path through several rebuilds and compare what it leaves behind with the oracle:

- the rows of the list in use are the brute-force r_list sets at the list's own reference positions, bit for bit;
- the forces at the final positions are the oracle's pair sums (rel-L2 <= 1e-5);
- the total-energy excursion over 100 steps from a relaxed FCC start follows the oracle's to 2e-6 eps per particle
  (Sec. 3.3.1).

Inputs are seeded (jittered lattices and random insertion with Maxwell velocities); the oracle is handed the
positions the GPU state holds at that point, which is how a checker of a GPU result is used here: the oracle's
own arithmetic takes nothing else from the HIP path.
"""
import sys

import numpy as np
import pytest

from paper_1912_04232_amd import inputs

pytestmark = pytest.mark.gpu

F_TOL = 1e-5


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
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def lj_system(md, u, v, L, skin=0.3):
    box = md.Box((L, L, L), 3)
    pot = md.Potential("lj", [[1.0]], [[1.0]], r_cut=2.5)
    return md.System(box, pot, u, v, skin=skin)


def lj_oracle_pot(orc):
    return orc.Potential("lj", np.ones((1, 1)), np.ones((1, 1)), r_cut=2.5)


def check_list_in_use(md, orc, s, L, rows=None):
    """Rows of the list the system holds now against the brute-force set at its reference positions."""
    ref = md.from_device_u32(s.nl.pos_ref)
    got = s.nl.rows()
    want = orc.neighbors(ref, [L, L, L], s.nl.r_list, rows=rows)
    ids = range(s.N) if rows is None else rows
    for q, i in enumerate(ids):
        g = np.sort(got[i])
        assert np.array_equal(g, want[q]), (int(i), g[:8], want[q][:8])
    return ref


def check_forces(md, orc, s, L, rows=None):
    u = md.from_device_u32(s.pos)
    Fo, _, _ = orc.pair_rows(orc.decode(u, [L, L, L]), [L, L, L], lj_oracle_pot(orc), rows=rows)
    F = s.force.cpu().numpy()
    if rows is not None:
        F = F[rows]
    err = rel_l2(F, Fo)
    assert err <= F_TOL, err
    return err


def run_and_check(md, orc, s, L, calls, steps, rows=None):
    """Run `calls` verlet_step calls of `steps` steps; after each, compare the list in use and the forces with the
    oracle.  Returns how many of the checked lists were built inside a run (reference positions equal to neither
    the start of that call nor any earlier list's)."""
    init, update = md.nve(s, 0.005)
    init()
    seen = {md.from_device_u32(s.nl.pos_ref).tobytes()}
    inrun = 0
    rebuilds = 0
    for c in range(calls):
        start = md.from_device_u32(s.pos).tobytes()
        update(steps)
        f = s.last_flags
        rebuilds += int(f[md.FLAG_REBUILDS])
        ref = check_list_in_use(md, orc, s, L, rows)
        key = ref.tobytes()
        if key != start and key not in seen:
            inrun += 1
        seen.add(key)
        err = check_forces(md, orc, s, L, rows)
        say(f"call {c}: rebuild launches {int(f[md.FLAG_REBUILDS])}, in-run lists checked so far {inrun}, "
            f"force rel-L2 {err:.2e}")
    return inrun, rebuilds


@pytest.mark.parametrize("case", ["lj2000", "lj3333_ragged"])
def test_inrun_rebuilt_rows_and_forces_match_oracle(md, orc, case):
    """Small systems, every row: N = 2000 at density 0.84 and a ragged N = 3333 (cells hold uneven counts), random
    insertion with Maxwell velocities at T = 1, five calls of 40 steps through several device-side rebuilds."""
    N, seed = (2000, 51) if case == "lj2000" else (3333, 77)
    L = inputs.box_for_density(N, 0.84)
    u = inputs.random_insertion_torus(N, L, 3, 0.8, seed)
    v = inputs.maxwell_velocities(N, 3, 1.0, seed + 1)
    s = lj_system(md, u, v, L)
    say("in-run rebuild parity", case)
    inrun, rebuilds = run_and_check(md, orc, s, L, 5, 40)
    assert inrun >= 2 and rebuilds >= 4, (inrun, rebuilds)


def test_inrun_rebuilt_rows_and_forces_match_oracle_256k(md, orc):
    """The benchmark's size and launch configuration: N = 256000 FCC at density 0.84 moved by seeded offsets of up to
    0.1, Maxwell velocities at T = 1, lanes chosen as the benchmark's default; three calls of 25 steps, each through
    device-side rebuilds.  600 sampled rows bit-exact at the list's reference positions and the sampled forces at
    the final positions within 1e-5."""
    cfg = inputs.lj_large()
    L = cfg["L"][0]
    u = inputs.jittered_torus(cfg["u"], cfg["L"], 0.1, 3101)
    s = lj_system(md, u, cfg["v"], L)
    rows = np.sort(np.random.default_rng(5).choice(cfg["N"], 600, replace=False))
    say("in-run rebuild parity at N = 256000, lanes", s.nl.lanes)
    inrun, rebuilds = run_and_check(md, orc, s, L, 3, 25, rows)
    assert inrun >= 2 and rebuilds >= 6, (inrun, rebuilds)


def test_verlet_energy_conservation_relaxed_fcc(md, orc):
    """NVE from a relaxed start (FCC at density 0.84, every force zero; Maxwell velocities at T = 1), 100 steps at
    dt = 0.005 (Sec. 3.3.1).  The FP64 oracle run from the same start is the checker: the GPU's total energy after
    every 10 steps, taken from each run's own start, equals the oracle's to 2e-6 eps per particle (the energies
    themselves agree to the 1e-6 relative tolerance of single-precision pair terms).  The excursion itself is that of the exact
    velocity-Verlet map, not of FP32 rounding: from a lattice start all energy is potential and the integrator's
    energy error swings by 4.9e-4 per particle while kinetic energy flows into the lattice, then settles below 1e-4
    (the oracle, at these inputs, prints the same figures).  Both are asserted: the swing below 1e-3 and every
    value over the last 50 steps below 1.5e-4."""
    cfg = inputs.lj_large(n_cells=8)   # 2048 particles
    L = cfg["L"][0]
    s = lj_system(md, cfg["u"], cfg["v"], L)
    init, update = md.nve(s, 0.005)
    init()
    E0 = s.potential_energy() + s.kinetic_energy()
    p = lj_oracle_pot(orc)
    x = orc.decode(cfg["u"], cfg["L"])
    v = cfg["v"].astype(np.float64)
    F, e, _ = orc.pair_rows(x, cfg["L"], p)
    Eo0 = float(e.sum() + 0.5 * (v * v).sum())
    assert abs(E0 - Eo0) / abs(Eo0) < 1e-6, (E0, Eo0)
    dev, tail = [], []
    for k in range(10):
        update(10)
        x, v, F = orc.verlet(x, v, F, cfg["L"], p, 0.005, 10)
        _, e, _ = orc.pair_rows(x, cfg["L"], p)
        dE_orc = (float(e.sum() + 0.5 * (v * v).sum()) - Eo0) / s.N
        dE_gpu = (s.potential_energy() + s.kinetic_energy() - E0) / s.N
        dev.append(abs(dE_gpu - dE_orc))
        if k >= 5:
            tail.append(abs(dE_gpu))
        say(f"relaxed FCC, step {10 * (k + 1)}: dE/N gpu {dE_gpu:.3e} oracle {dE_orc:.3e}")
        assert abs(dE_gpu) < 1e-3
    assert max(dev) < 2e-6, dev
    assert max(tail) < 1.5e-4, tail


def test_kinetic_energy_and_sum_against_numpy(md):
    """md_kinetic_energy = 1/2 sum v^2 and md_sum against numpy's float64 sums (math.fsum order-free reference)."""
    import math

    import torch
    ctx = md.Context()
    rng = np.random.default_rng(11)
    for n, dim in ((1, 3), (1000, 3), (65537, 2), (300001, 3)):
        v = rng.standard_normal((n, dim)).astype(np.float32)
        out = torch.zeros(1, dtype=torch.float64, device=ctx.device)
        md.kinetic_energy(ctx, torch.as_tensor(v, device=ctx.device), out)
        want = 0.5 * math.fsum((v.astype(np.float64) ** 2).ravel().tolist())
        assert float(out.item()) == pytest.approx(want, rel=1e-12, abs=1e-300)
        x = rng.standard_normal(n * dim)
        md.md_sum(ctx, torch.as_tensor(x, device=ctx.device), out)
        assert float(out.item()) == pytest.approx(math.fsum(x.tolist()), rel=1e-10, abs=1e-9)


def test_verlet_step_keeps_a_valid_list_and_rebuilds_a_moved_or_overflowed_one(md, orc):
    """verlet_step keeps the list the last build on the context made for the same arrays while the device finds it
    valid for the positions (no build launch runs), rebuilds it when the positions have moved away from its reference
    positions, and after a run whose list overflowed builds again instead of using the truncated rows, even when the
    caller cleared the flags."""
    import torch
    N = 2000
    L = inputs.box_for_density(N, 0.84)
    u = inputs.random_insertion_torus(N, L, 3, 0.8, 91)
    v = inputs.maxwell_velocities(N, 3, 1.0, 92)
    s = lj_system(md, u, v, L)
    s.build()
    s.forces()
    ref0 = md.from_device_u32(s.nl.pos_ref).copy()
    # one step: no rebuild is due, and the list just built is kept (no build counted)
    s.nl.clear_flags()
    md.verlet_step(s.ctx, s.box, s.pot, s.pos, s.vel, s.force, s.species, s.nl, 0.005, 1)
    f = s.nl.read_flags()
    assert f[md.FLAG_REBUILDS] == 0 and f[md.FLAG_STALE] == 0, f
    assert np.array_equal(md.from_device_u32(s.nl.pos_ref), ref0)
    # positions moved by a uniform shift of 0.2 (more than skin/2): the call builds a list for them first
    shifted = (md.from_device_u32(s.pos).astype(np.int64) + int(0.2 / L * 2 ** 32)) & 0xFFFFFFFF
    s.pos.copy_(torch.as_tensor(shifted.astype(np.uint32).view(np.int32), device=s.pos.device).reshape(s.pos.shape))
    s.forces()
    s.nl.clear_flags()
    md.verlet_step(s.ctx, s.box, s.pot, s.pos, s.vel, s.force, s.species, s.nl, 0.005, 1)
    f = s.nl.read_flags()
    assert f[md.FLAG_REBUILDS] >= 1 and f[md.FLAG_STALE] == 0, f
    check_list_in_use(md, orc, s, L)
    # a list too small for the rows: the run overflows; with the flags cleared and the same arrays, the next call
    # builds again (and reports the overflow again) rather than stepping on truncated rows
    small = md.NeighborList(N, 3, 24, s.nl.r_list, s.nl.skin, s.ctx.device, s.nl.max_per_cell, s.nl.lanes)
    md.nl_build(s.ctx, s.box, s.pos, small)
    assert small.read_flags()[md.FLAG_OVERFLOW] == 1
    for _ in range(2):
        small.clear_flags()
        md.verlet_step(s.ctx, s.box, s.pot, s.pos, s.vel, s.force, s.species, small, 0.005, 1)
        f = small.read_flags()
        assert f[md.FLAG_OVERFLOW] == 1 and f[md.FLAG_REBUILDS] >= 1, f


def disks(md, N, phi, seed, skin, lanes=None):
    L = inputs.box_for_packing([1.0, 1.4], [N // 2, N - N // 2], phi, 2)
    d = np.array([1.0, 1.4])
    sig = 0.5 * (d[:, None] + d[None, :])
    box = md.Box((L, L), 2)
    pot = md.Potential("soft_sphere", sig, np.ones((2, 2)), alpha=2.0)
    sp = inputs.bidisperse_species(N)
    return md.System(box, pot, inputs.uniform_torus(N, 2, seed), None, sp, skin=skin, lanes=lanes), L, sig, sp


@pytest.mark.parametrize("case", ["disks2000", "disks3001_ragged"])
def test_fire_inrun_rebuilt_rows_and_forces_match_oracle(md, orc, case):
    """FIRE's step pipeline rebuilds the list inside a fire_step call (bins in one force launch, rows in the next).
    Bidisperse harmonic disks at phi = 0.9 from uniform random positions, skin 0.3 as in the 65536-disk workload:
    300 synchronous steps take the packing past its first, long steps (the pipeline needs about three steps from a
    request to the new list, so it cannot follow steps that need a list every two or three); then four pipelined
    calls of 40 steps run with no list going stale, and
    after each the rows of the list in use are the brute-force r_list sets at its reference positions bit for bit
    and the forces at the final positions are the oracle's (rel-L2 <= 1e-5).  The ragged case (uneven cells) runs
    4 lanes per disk."""
    N, seed, lanes = (2000, 4401, None) if case == "disks2000" else (3001, 4402, 4)
    s, L, sig, sp = disks(md, N, 0.9, seed, 0.3, lanes)
    op = orc.Potential("soft_sphere", sig, np.ones((2, 2)), alpha=2.0)
    fp = md.FireParams()
    init, step, _ = md.fire_descent(s, fp, f_tol=1e-30)
    state = init()
    step(300, sync=True)
    inrun = rebuilds = 0
    seen = {md.from_device_u32(s.nl.pos_ref).tobytes()}
    for c in range(4):
        start = md.from_device_u32(s.pos).tobytes()
        s.nl.clear_flags()
        md.fire_step(s.ctx, s.box, s.pot, s.pos, s.vel, s.force, s.species, s.nl, fp, state, 40, 1e-30,
                     sync_rebuild=False)
        f = s.nl.read_flags()
        assert not (f[md.FLAG_STALE] or f[md.FLAG_OVERFLOW] or f[md.FLAG_CELL_OVERFLOW]), f.tolist()
        rebuilds += int(f[md.FLAG_REBUILDS]) - 1  # less the build at the start of the call
        ref = md.from_device_u32(s.nl.pos_ref)
        got = s.nl.rows()
        want = orc.neighbors(ref, [L, L], s.nl.r_list)
        for i in range(N):
            assert np.array_equal(np.sort(got[i]), want[i]), (c, i)
        key = ref.tobytes()
        if key != start and key not in seen:
            inrun += 1
        seen.add(key)
        u = md.from_device_u32(s.pos)
        Fo, _, _ = orc.pair_rows(orc.decode(u, [L, L]), [L, L], op, sp)
        err = rel_l2(s.force.cpu().numpy(), Fo)
        say(f"FIRE call {c}: in-run builds {int(f[md.FLAG_REBUILDS]) - 1}, in-run lists checked {inrun}, "
            f"force rel-L2 {err:.2e}")
        assert err <= F_TOL, err
    assert inrun >= 2 and rebuilds >= 4, (inrun, rebuilds)


def test_fire_pipelined_and_synchronous_agree_while_no_rebuild_runs(md):
    """The two ways fire_step keeps the list share their arithmetic: the mixing launch (rules, mixing, drift) and the
    force pass.  The packing is first relaxed to max |F| < 1e-4; from rest there, 40 FIRE steps move no disk near
    skin/2, so neither mode rebuilds inside the call, and the positions, velocities, forces and FIRE state after the
    40 steps agree bit for bit."""
    import torch
    s0, L, sig, sp = disks(md, 3000, 0.9, 4501, 0.3)
    fp = md.FireParams()
    init, _, minimize = md.fire_descent(s0, fp, f_tol=1e-4)
    init()
    assert minimize(200000, chunk=500)["converged"]
    init, _, _ = md.fire_descent(s0, fp, f_tol=1e-30)
    state = init()  # a fresh FIRE state at the relaxed packing: v = 0, dt = dt_start
    saved = (s0.pos.clone(), s0.vel.clone(), s0.force.clone(), state.clone())
    out = {}
    for sync in (False, True):
        for t, v in zip((s0.pos, s0.vel, s0.force, state), saved):
            t.copy_(v)
        s0.build()
        s0.nl.clear_flags()
        md.fire_step(s0.ctx, s0.box, s0.pot, s0.pos, s0.vel, s0.force, s0.species, s0.nl, fp, state, 40, 1e-30,
                     sync_rebuild=sync)
        f = s0.nl.read_flags()
        say(f"sync {sync}: list builds {int(f[md.FLAG_REBUILDS])}, flags {f.tolist()}")
        assert int(f[md.FLAG_REBUILDS]) == 1  # the build at the start of the call only
        assert not (f[md.FLAG_STALE] or f[md.FLAG_OVERFLOW] or f[md.FLAG_NONFINITE])
        out[sync] = (s0.pos.clone(), s0.vel.clone(), s0.force.clone(), state.clone())
    for a, b in zip(out[False], out[True]):
        assert torch.equal(a, b)
