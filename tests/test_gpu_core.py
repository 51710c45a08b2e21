"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Bars: neighbor rows bit-identical to brute force after sorting; forces
||F_gpu - F_orc||_2 / ||F_orc||_2 <= 1e-5 over all components; energies
|E_gpu - E_orc| / |E_orc| <= 1e-6 (or relative to sum |e_i| when E is near 0).
"""
import math
import sys

import numpy as np
import pytest

from paper_1912_04232_amd import inputs

pytestmark = pytest.mark.gpu

F_TOL = 1e-5
E_TOL = 1e-6


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


def torus_x(u, L):
    """Torus coordinates of a GPU state -> float64 positions (u L / 2^32), for comparisons in the tests."""
    u = np.asarray(u, dtype=np.uint32)
    return u.astype(np.float64) * (np.asarray(L, dtype=np.float64)[: u.shape[1]] / 4294967296.0)


def pairs_within(u, L, r):
    """Every pair (i, j), i != j, with nearest-image distance < r, by brute force in numpy (validity checks of GPU
    states; parity against the oracle always starts from seeded inputs)."""
    x = torus_x(u, L)
    Lv = np.asarray(L, dtype=np.float64)[: x.shape[1]]
    out = []
    for i in range(x.shape[0]):
        d = x - x[i]
        d -= Lv * np.rint(d / Lv)
        r2 = (d * d).sum(1)
        r2[i] = np.inf
        out.append(np.nonzero(r2 < r * r)[0])
    return out


def make_system(md, cfg, skin=None, capacity=None):
    dim = cfg["dim"]
    box = md.Box(tuple(cfg["L"][:dim]), dim)
    if cfg["kind"] == "lj":
        pot = md.Potential("lj", cfg["sigma"], cfg["epsilon"], r_cut=cfg["r_cut"])
    else:
        pot = md.Potential("soft_sphere", cfg["sigma"], cfg["epsilon"], alpha=cfg.get("alpha", 2.0))
    sp = cfg.get("species") if pot.n_species > 1 else None
    return md.System(box, pot, cfg["u"], cfg.get("v"), sp, skin=cfg.get("skin", 0.3) if skin is None else skin,
                     capacity=capacity)


def orc_pot(orc, cfg):
    if cfg["kind"] == "lj":
        return orc.Potential("lj", np.array(cfg["sigma"]), np.array(cfg["epsilon"]), r_cut=cfg["r_cut"])
    return orc.Potential("soft_sphere", np.array(cfg["sigma"]), np.array(cfg["epsilon"]), alpha=cfg.get("alpha", 2.0))


def lj_cfg(N, rho, seed, skin=0.3, rmin=0.8):
    L = inputs.box_for_density(N, rho)
    u = inputs.random_insertion_torus(N, L, 3, rmin, seed)
    return dict(N=N, dim=3, L=[L, L, L], u=u, v=inputs.maxwell_velocities(N, 3, 1.0, seed + 1), kind="lj",
                sigma=[[1.0]], epsilon=[[1.0]], r_cut=2.5, skin=skin)


def ss_cfg(N, phi, seed, skin=0.3):
    L = inputs.box_for_packing([1.0, 1.4], [N // 2, N - N // 2], phi, 2)
    d = np.array([1.0, 1.4])
    return dict(N=N, dim=2, L=[L, L, 0.0], u=inputs.uniform_torus(N, 2, seed), species=inputs.bidisperse_species(N),
                kind="soft_sphere", sigma=(0.5 * (d[:, None] + d[None, :])).tolist(),
                epsilon=[[1.0, 1.0], [1.0, 1.0]], alpha=2.0, skin=skin)


def check_rows(orc, sysm, cfg, rows=None):
    got = sysm.nl.rows()
    want = orc.neighbors(cfg["u"], cfg["L"], sysm.nl.r_list, rows=rows)
    ids = range(len(got)) if rows is None else rows
    for q, i in enumerate(ids):
        g = np.sort(got[i])
        assert np.array_equal(g, want[q]), (i, g[:10], want[q][:10])


# ------------------------------------------------------------------ neighbor list

@pytest.mark.parametrize("case", ["lj1000", "lj_ragged", "lj_blocks6", "lj_blocks7", "ss2d", "lj_dilute", "tiny_box",
                                  "two", "one"])
def test_nl_build_bitexact(md, orc, case):
    """Rows against the brute-force sets.  Dense cells (LJ at density 0.84, about 18 per cell) are built one wave per
    cell; sparse ones (the 2D packing and the dilute gas, about 2 per cell, and the few-particle boxes) one particle
    per W lanes."""
    say("nl_build", case)
    if case == "lj1000":
        cfg = inputs.lj_small()
    elif case == "lj_ragged":
        cfg = lj_cfg(3333, 0.84, 77)
    elif case == "lj_blocks6":
        cfg = lj_cfg(4500, 0.84, 78)                 # 6 cells a side: smallest box of LDS-staged cell blocks
    elif case == "lj_blocks7":
        cfg = lj_cfg(8000, 0.84, 79)                 # 7 cells a side: a ragged last cell block
    elif case == "ss2d":
        cfg = ss_cfg(5000, 0.9, 21)
    elif case == "lj_dilute":
        cfg = lj_cfg(3000, 0.1, 80)                  # about 2.2 particles per cell
    elif case == "tiny_box":
        cfg = lj_cfg(40, 0.12, 5, rmin=0.9)         # L = 6.93 < 3 r_list: whole-box scan
    elif case == "two":
        cfg = lj_cfg(2, 0.01, 6)
    else:
        cfg = lj_cfg(1, 0.002, 6)
    s = make_system(md, cfg)
    s.build()
    check_rows(orc, s, cfg)
    f = s.nl.read_flags()
    assert f[md.FLAG_OVERFLOW] == 0
    cnt = s.nl.count.cpu().numpy()[: s.N]
    assert f[md.FLAG_MAXCOUNT] == cnt.max(initial=0) * s.nl.lanes


def boundary_pairs(dim, L, r_list, sites, seed):
    """Isolated pairs on a grid of sites (spacing L / sites > 2.5 r_list, so no pair meets another): member B sits
    at r_list (1 + delta) from member A along a random direction, delta drawn from +-1e-7 .. +-2e-2 and 0."""
    rng = np.random.default_rng(seed)
    g = np.arange(sites, dtype=np.float64) * (L / sites)
    grid = np.stack(np.meshgrid(*([g] * dim), indexing="ij"), axis=-1).reshape(-1, dim)
    a = grid + rng.uniform(0.0, 0.2, size=grid.shape)
    dirs = rng.standard_normal(a.shape)
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    deltas = np.array([-2e-2, -5e-3, -1.3e-3, -1e-3, -1e-4, -1e-6, -1e-7, 0.0, 1e-7, 1e-6, 1e-4, 1e-3, 1.3e-3, 5e-3,
                       2e-2])
    delta = deltas[rng.integers(0, len(deltas), size=len(a))]
    b = a + dirs * (r_list * (1.0 + delta))[:, None]
    x = np.concatenate([a, b])
    return inputs.to_torus(x, [L] * dim)


@pytest.mark.parametrize("dim,L,sites,lanes", [(3, 42.0, 5, 4), (3, 42.0, 5, 1), (2, 60.0, 7, 2), (3, 8.0, 1, 8)])
def test_nl_boundary_pairs_bitexact(md, orc, dim, L, sites, lanes):
    """Pairs within a relative 2e-2 of r_list, many inside the uncertain band of the single-precision and of the
    packed 16-bit candidate tests (where the defining double expression decides): rows equal the oracle's sets.
    The last case is a box with fewer than 3 cells a side (whole-box scan)."""
    say("nl boundary pairs", dim, L, sites, lanes)
    r_list = 2.8
    u = boundary_pairs(dim, L, r_list, sites, 1000 + dim + sites)
    N = len(u)
    box = md.Box(tuple([L] * dim), dim)
    import torch
    ctx = md.Context()
    pos = torch.as_tensor(u.view(np.int32), device="cuda").contiguous()
    nl = md.NeighborList(N, dim, 16, r_list, 0.3, max_per_cell=64, lanes=lanes)
    md.nl_build(ctx, box, pos, nl)
    f = nl.read_flags()
    assert f[md.FLAG_OVERFLOW] == 0 and f[md.FLAG_CELL_OVERFLOW] == 0
    rows = nl.rows()
    want = orc.neighbors(u, [L] * dim + [0.0] * (3 - dim), nl.r_list)
    inside = 0
    for i in range(N):
        assert np.array_equal(np.sort(rows[i]), want[i]), (i, rows[i], want[i])
        inside += len(want[i])
    if sites > 1:
        assert 0 < inside < N   # both sides of r_list are present


def test_nl_rows_are_canonical(md):
    """Two builds give identical rows (same order), dealt round-robin over the sub-rows."""
    cfg = lj_cfg(4000, 0.84, 3)
    s = make_system(md, cfg)
    s.build()
    rows0, cnt0 = s.nl.rows(), s.nl.count.cpu().numpy().copy()
    s.build()
    rows1, cnt1 = s.nl.rows(), s.nl.count.cpu().numpy()
    assert np.array_equal(cnt0, cnt1)
    assert all(np.array_equal(a, b) for a, b in zip(rows0, rows1))
    # neighbors are dealt round-robin, so the sub-row lengths of a row differ by at most one
    spread = cnt1.max(axis=1) - cnt1.min(axis=1)
    assert spread.max() <= 1
    assert (cnt1[:, 0] >= cnt1[:, -1]).all()


@pytest.mark.parametrize("lanes", [1, 2, 4, 8])
def test_nl_rows_every_lane_count(md, orc, lanes):
    """Rows built by 1, 2, 4 or 8 lanes per particle (each lane count numbers the neighbors by its own prefix
    sums across the particle's lanes) are the oracle's rows, dealt round-robin over the sub-rows."""
    say("nl lanes", lanes)
    cfg = lj_cfg(3333, 0.84, 81)
    box = md.Box(tuple(cfg["L"]), 3)
    pot = md.Potential("lj", cfg["sigma"], cfg["epsilon"], r_cut=cfg["r_cut"])
    s = md.System(box, pot, cfg["u"], cfg["v"], skin=0.3, lanes=lanes)
    s.build()
    assert s.nl.lanes == lanes
    check_rows(orc, s, cfg)
    cnt = s.nl.count.cpu().numpy()[: s.N]
    assert (cnt.max(axis=1) - cnt.min(axis=1)).max() <= 1
    assert s.nl.read_flags()[md.FLAG_OVERFLOW] == 0


def test_segmented_list_matches_per_system_oracle(md, orc):
    """A list over three independent systems of 700 particles each (segment = 700, same box) holds exactly the
    rows of each system on its own, with indices offset by the system's first particle."""
    import torch
    S, n = 3, 700
    cfgs = [lj_cfg(n, 0.84, 40 + k) for k in range(S)]
    L = cfgs[0]["L"]
    box = md.Box(tuple(L), 3)
    u = np.concatenate([c["u"] for c in cfgs])
    ctx = md.Context()
    pos = torch.as_tensor(u.view(np.int32), device="cuda").contiguous()
    nl = md.NeighborList(S * n, 3, 96, 2.8, 0.3, max_per_cell=64, lanes=2, segment=n)
    md.nl_build(ctx, box, pos, nl)
    f = nl.read_flags()
    assert f[md.FLAG_OVERFLOW] == 0 and f[md.FLAG_CELL_OVERFLOW] == 0
    rows = nl.rows()
    for k in range(S):
        want = orc.neighbors(cfgs[k]["u"], L, nl.r_list)
        for i in range(n):
            assert np.array_equal(np.sort(rows[k * n + i]), want[i] + k * n), (k, i)


def test_nl_overflow_flag_and_regrow(md, orc):
    cfg = lj_cfg(2000, 0.84, 8)
    s = make_system(md, cfg, capacity=16)
    s.nl.clear_flags()
    md.nl_build(s.ctx, s.box, s.pos, s.nl)
    f = s.nl.read_flags()
    assert f[md.FLAG_OVERFLOW] == 1 and f[md.FLAG_MAXCOUNT] > 16
    s.build()   # grows and rebuilds
    assert s.nl.capacity >= f[md.FLAG_MAXCOUNT]
    check_rows(orc, s, cfg, rows=list(range(0, 2000, 7)))


def test_nl_box_too_small_is_rejected(md):
    cfg = lj_cfg(10, 0.5, 4)
    cfg["L"] = [5.0, 5.0, 5.0]
    s = make_system(md, cfg)
    with pytest.raises(md.MDError) as e:
        md.nl_build(s.ctx, s.box, s.pos, s.nl)    # r_list 2.8 >= L/2
    assert e.value.code == -2


# ------------------------------------------------------------------------- forces

@pytest.mark.parametrize("case", ["lj1000", "lj_ragged", "ss2d", "ss2d_alpha25", "lj_species"])
def test_forces_energy_virial_vs_oracle(md, orc, case):
    say("pair_energy_force", case)
    if case == "lj1000":
        cfg = inputs.lj_small()
    elif case == "lj_ragged":
        cfg = lj_cfg(3333, 0.84, 77)
    elif case == "lj_blocks6":
        cfg = lj_cfg(4500, 0.84, 78)                 # 6 cells a side: smallest box of LDS-staged cell blocks
    elif case == "lj_blocks7":
        cfg = lj_cfg(8000, 0.84, 79)                 # 7 cells a side: a ragged last cell block
    elif case.startswith("ss2d"):
        cfg = ss_cfg(3000, 0.9, 22)
        if case == "ss2d_alpha25":
            cfg["alpha"] = 2.5
    else:
        cfg = lj_cfg(2500, 0.8, 31)
        cfg["species"] = inputs.bidisperse_species(2500)
        cfg["sigma"] = [[1.0, 0.8], [0.8, 0.88]]
        cfg["epsilon"] = [[1.0, 1.5], [1.5, 0.5]]
    s = make_system(md, cfg)
    s.build()
    e, w = s.forces(energy=True)
    F = s.force.cpu().numpy()
    x = orc.decode(cfg["u"], cfg["L"])
    sp = cfg.get("species")
    Fo, eo, wo = orc.pair_rows(x, cfg["L"], orc_pot(orc, cfg), sp)
    assert rel_l2(F, Fo) <= F_TOL
    eg = e.cpu().numpy()
    scale = max(abs(math.fsum(eo)), math.fsum(np.abs(eo)) * 1e-3)
    assert abs(math.fsum(eg) - math.fsum(eo)) / scale <= E_TOL
    assert abs(math.fsum(w.cpu().numpy()) - math.fsum(wo)) / max(abs(math.fsum(wo)), 1e-12) <= 10 * E_TOL
    assert rel_l2(eg, eo) <= 1e-5
    assert s.potential_energy() == pytest.approx(math.fsum(eg), rel=1e-12)


@pytest.mark.parametrize("case", ["lj1000", "ss_small", "ragged"])
def test_dense_vs_oracle_and_nl(md, orc, case):
    say("dense", case)
    if case == "lj1000":
        cfg = inputs.lj_small()
    elif case == "ss_small":
        cfg = ss_cfg(700, 0.9, 9)
    else:
        cfg = lj_cfg(517, 0.6, 12)
    s = make_system(md, cfg)
    import torch
    Fd = torch.zeros_like(s.force)
    ed = torch.zeros(s.N, dtype=torch.float64, device=s.force.device)
    md.pair_energy_force(s.ctx, s.box, s.pot, s.pos, s.species, None, Fd, ed, None)
    Fo, eo, _ = orc.pair_rows(orc.decode(cfg["u"], cfg["L"]), cfg["L"], orc_pot(orc, cfg), cfg.get("species"))
    assert rel_l2(Fd.cpu().numpy(), Fo) <= F_TOL
    assert abs(float(ed.sum()) - math.fsum(eo)) / max(abs(math.fsum(eo)), 1e-9) <= E_TOL
    s.build()
    s.forces()
    assert rel_l2(s.force.cpu().numpy(), Fd.cpu().numpy()) <= F_TOL


def test_nonfinite_flag(md):
    cfg = lj_cfg(64, 0.3, 2)
    u = cfg["u"].copy()
    u[1] = u[0]
    u[1, 0] += 1000   # r ~ 2e-5 sigma: force overflows float
    cfg["u"] = u
    s = make_system(md, cfg)
    s.build()
    s.nl.clear_flags()
    s.forces()
    assert s.nl.read_flags()[md.FLAG_NONFINITE] == 1


# --------------------------------------------------------------- velocity Verlet

def test_verlet_steps_vs_oracle(md, orc):
    """A few velocity-Verlet steps from identical states agree with the FP64 oracle."""
    cfg = lj_cfg(1500, 0.84, 41)
    s = make_system(md, cfg)
    init, update = md.nve(s, 0.005)
    init()
    x = orc.decode(cfg["u"], cfg["L"])
    p = orc_pot(orc, cfg)
    F, _, _ = orc.pair_rows(x, cfg["L"], p)
    v = cfg["v"].astype(np.float64)
    for n in (1, 4):
        say("verlet", n)
        update(n)
        x, v, F = orc.verlet(x, v, F, cfg["L"], p, 0.005, n)
        xg = torus_x(md.from_device_u32(s.pos), cfg["L"])
        d = xg - x
        d -= np.array(cfg["L"]) * np.rint(d / np.array(cfg["L"]))
        assert np.abs(d).max() < 1e-5
        assert rel_l2(s.vel.cpu().numpy(), v) < 1e-5
        assert rel_l2(s.force.cpu().numpy(), F) < 1e-4


def test_verlet_rectangular_box_vs_oracle(md, orc):
    """LJ in a box with a different edge along each axis (the force loop's per-axis scale path) agrees with the
    FP64 oracle over a few velocity-Verlet steps and in the list, from a jittered grid at density ~0.75."""
    counts = (14, 11, 9)
    L = [inputs.f32(14 * 1.10), inputs.f32(11 * 1.12), inputs.f32(9 * 1.14)]
    N = counts[0] * counts[1] * counts[2]
    u = inputs.jittered_grid_torus(counts, 0.15, 91)
    cfg = dict(N=N, dim=3, L=L, u=u, v=inputs.maxwell_velocities(N, 3, 1.0, 92), kind="lj", sigma=[[1.0]],
               epsilon=[[1.0]], r_cut=2.5, skin=0.3)
    s = make_system(md, cfg)
    s.build()
    check_rows(orc, s, cfg)
    init, update = md.nve(s, 0.005)
    init()
    x = orc.decode(cfg["u"], cfg["L"])
    p = orc_pot(orc, cfg)
    F, _, _ = orc.pair_rows(x, cfg["L"], p)
    assert rel_l2(s.force.cpu().numpy(), F) < F_TOL
    v = cfg["v"].astype(np.float64)
    for n in (1, 4):
        say("verlet rect", n)
        update(n)
        x, v, F = orc.verlet(x, v, F, cfg["L"], p, 0.005, n)
        xg = torus_x(md.from_device_u32(s.pos), cfg["L"])
        d = xg - x
        d -= np.array(cfg["L"]) * np.rint(d / np.array(cfg["L"]))
        assert np.abs(d).max() < 1e-5
        assert rel_l2(s.vel.cpu().numpy(), v) < 1e-5
        assert rel_l2(s.force.cpu().numpy(), F) < 1e-4


@pytest.mark.parametrize("case", ["2d_square", "2d_rect", "3d_two_species"])
def test_verlet_lj_variants_vs_oracle(md, orc, case):
    """LJ through the Verlet step kernel in 2D (square box: integer-unit displacements; rectangular: per-axis
    scale) and in 3D with two species (species of neighbors through the range-checked loads)."""
    say("verlet lj", case)
    if case == "3d_two_species":
        counts, a = (12, 12, 12), 1.12
        sigma, eps = [[1.0, 1.05], [1.05, 1.1]], [[1.0, 0.8], [0.8, 1.2]]
    else:
        counts = (40, 40) if case == "2d_square" else (44, 34)
        a = 1.08
        sigma, eps = [[1.0]], [[1.0]]
    dim = len(counts)
    L = [inputs.f32(n * a) for n in counts] + [0.0] * (3 - dim)
    N = int(np.prod(counts))
    u = inputs.jittered_grid_torus(counts, 0.12, 95)
    cfg = dict(N=N, dim=dim, L=L, u=u, v=inputs.maxwell_velocities(N, dim, 0.8, 96), kind="lj", sigma=sigma,
               epsilon=eps, r_cut=2.5, skin=0.3)
    if len(sigma) > 1:
        cfg["species"] = inputs.bidisperse_species(N)
    s = make_system(md, cfg)
    init, update = md.nve(s, 0.004)
    init()
    x = orc.decode(cfg["u"], cfg["L"][:dim])
    p = orc_pot(orc, cfg)
    sp = cfg.get("species")
    F, _, _ = orc.pair_rows(x, cfg["L"][:dim], p, sp) if sp is not None else orc.pair_rows(x, cfg["L"][:dim], p)
    assert rel_l2(s.force.cpu().numpy(), F) < F_TOL
    v = cfg["v"].astype(np.float64)
    update(3)
    if sp is not None:
        x, v, F = orc.verlet(x, v, F, cfg["L"][:dim], p, 0.004, 3, sp)
    else:
        x, v, F = orc.verlet(x, v, F, cfg["L"][:dim], p, 0.004, 3)
    assert rel_l2(s.force.cpu().numpy(), F) < 1e-4
    assert rel_l2(s.vel.cpu().numpy(), v) < 1e-5


def test_verlet_rebuilds_keep_every_pair(md, orc):
    """Over 300 steps with device-side rebuilds the list always contains every pair inside the cutoff and the
    final forces agree with a fresh evaluation from a fresh list (a fresh build orders rows differently, so the
    float sums agree to rounding, not bit for bit)."""
    cfg = lj_cfg(2000, 0.84, 51)
    s = make_system(md, cfg)
    init, update = md.nve(s, 0.005)
    init()
    s.nl.clear_flags()
    reb = 0
    for _ in range(6):
        update(50)
        f = s.nl.read_flags()
        reb += int(f[md.FLAG_REBUILDS])
        u = md.from_device_u32(s.pos)
        rows = s.nl.rows()
        inner = pairs_within(u, cfg["L"], 2.5)
        for i in range(0, 2000, 11):
            assert set(inner[i].tolist()) <= set(rows[i].tolist())
        s.nl.clear_flags()
    assert reb >= 2
    F_run = s.force.clone()
    s.build()
    s.forces()
    assert rel_l2(F_run.cpu().numpy(), s.force.cpu().numpy()) <= 1e-6


def test_verlet_energy_conservation(md):
    cfg = inputs.lj_large(n_cells=6)   # 864-particle FCC at rho 0.84, T = 1
    s = make_system(md, cfg)
    init, update = md.nve(s, 0.005)
    init()
    E0 = s.potential_energy() + s.kinetic_energy()
    worst = 0.0
    for _ in range(10):
        update(20)
        worst = max(worst, abs(s.potential_energy() + s.kinetic_energy() - E0))
    say("max |dE|/N", worst / s.N)
    assert worst / s.N < 2e-3


def test_verlet_deterministic_and_overflow_regrow(md):
    """Two runs are bitwise identical; a run whose list is sized exactly to the first build overflows at a later
    device-side rebuild, is re-run from its saved input with a larger list, and still equals the others bit for bit
    (rows are canonical, so the capacity does not change the summation order)."""
    cfg = lj_cfg(3000, 0.84, 61)
    outs = []
    grew = False
    for tight in (False, False, True):
        s = make_system(md, cfg, capacity=256)
        init, update = md.nve(s, 0.005)
        init()
        if tight:
            need = int(s.nl.read_flags()[md.FLAG_MAXCOUNT])
            s.nl = md.NeighborList(s.N, 3, need, s.nl.r_list, s.nl.skin, s.ctx.device, s.nl.max_per_cell,
                                   s.nl.lanes)
            s.build()
            s.forces()
        update(150)
        if tight:
            grew = s.nl.capacity > need
        outs.append((md.from_device_u32(s.pos).copy(), s.vel.cpu().numpy(), s.force.cpu().numpy()))
    say("tight list grew:", grew)
    for k in range(3):
        assert np.array_equal(outs[0][k], outs[1][k])
        assert np.array_equal(outs[0][k], outs[2][k])


def test_verlet_2d_soft_spheres(md, orc):
    cfg = ss_cfg(2000, 0.8, 71)
    cfg["v"] = inputs.maxwell_velocities(2000, 2, 0.01, 3)
    s = make_system(md, cfg)
    init, update = md.nve(s, 0.01)
    init()
    x = orc.decode(cfg["u"], cfg["L"][:2])
    p = orc_pot(orc, cfg)
    F, _, _ = orc.pair_rows(x, cfg["L"][:2], p, cfg["species"])
    update(3)
    x, v, F = orc.verlet(x, cfg["v"].astype(np.float64), F, cfg["L"][:2], p, 0.01, 3, cfg["species"])
    assert rel_l2(s.force.cpu().numpy(), F) < 1e-4
    assert rel_l2(s.vel.cpu().numpy(), v) < 1e-5


# ---------------------------------------------------------------------------- FIRE

def test_fire_one_step_vs_oracle(md, orc):
    cfg = ss_cfg(1000, 0.9, 81)
    s = make_system(md, cfg)
    init, step, _ = md.fire_descent(s, f_tol=1e-6)
    init()
    st = step(1)
    p = orc_pot(orc, cfg)
    res = orc.fire(orc.decode(cfg["u"], cfg["L"][:2]), cfg["L"][:2], p, cfg["species"], max_steps=1, f_tol=0.0)
    # the GPU applies the velocity mixing of a step at the start of the next one
    v = st["mix_v"] * s.vel.cpu().numpy().astype(np.float64) + st["mix_f"] * s.force.cpu().numpy()
    assert rel_l2(v, res["v"]) < 1e-4
    assert rel_l2(s.force.cpu().numpy(), res["F"]) < 1e-4
    assert st["dt"] == pytest.approx(res["dt"]) and st["n_pos"] == res["n_pos"] and st["steps"] == 1


@pytest.mark.parametrize("K,skin", [(10, 0.3), (30, 0.3), (30, 0.05)])
def test_fire_steps_vs_oracle(md, orc, K, skin):
    """K FIRE steps from the same start in one fire_step call (each step the mixing launch, which applies the FIRE
    rules of the previous step, and the force launch): positions, mixed velocities and the FIRE scalars follow the
    FP64 oracle's.  With skin 0.05 the list is rebuilt inside the call several times."""
    cfg = ss_cfg(1000, 0.9, 81, skin=skin)
    s = make_system(md, cfg)
    init, step, _ = md.fire_descent(s, f_tol=1e-30)
    init()
    st = step(K)
    builds = int(s.nl.read_flags()[md.FLAG_REBUILDS])
    say("K", K, "skin", skin, "list builds", builds)
    if skin < 0.1:
        assert builds >= 3
    p = orc_pot(orc, cfg)
    L = np.asarray(cfg["L"][:2], dtype=np.float64)
    res = orc.fire(orc.decode(cfg["u"], L), L, p, cfg["species"], max_steps=K, f_tol=0.0)
    dx = orc.decode(s.pos.cpu().numpy(), L) - res["x"]
    dx -= L * np.round(dx / L)
    v = st["mix_v"] * s.vel.cpu().numpy().astype(np.float64) + st["mix_f"] * s.force.cpu().numpy()
    say("K", K, "position rms", np.sqrt((dx ** 2).sum(1).mean()), "v rel-L2", rel_l2(v, res["v"]))
    assert np.sqrt((dx ** 2).sum(1).mean()) < 1e-4
    assert rel_l2(v, res["v"]) < 1e-3
    assert rel_l2(s.force.cpu().numpy(), res["F"]) < 1e-3
    assert st["dt"] == pytest.approx(res["dt"]) and st["n_pos"] == res["n_pos"] and st["steps"] == K


def test_fire_lattice_reaches_closed_form(md):
    """A jittered compressed triangular lattice relaxes to E/N = 3/2 (1 - a)^2 with max |F| < 1e-6."""
    a = 0.98
    u, Lx, Ly = inputs.triangular_torus(40, 40, a)
    rng = np.random.default_rng(5)
    jit = inputs.to_torus(rng.normal(0, 0.01, (1600, 2)), [Lx, Ly])
    u = (u.astype(np.uint64) + jit.astype(np.uint64)) % 2 ** 32
    cfg = dict(N=1600, dim=2, L=[Lx, Ly, 0.0], u=u.astype(np.uint32), kind="soft_sphere", sigma=[[1.0]],
               epsilon=[[1.0]], alpha=2.0, skin=0.3)
    s = make_system(md, cfg)
    init, step, minimize = md.fire_descent(s, f_tol=1e-6)
    init()
    st = minimize(20000)
    assert st["converged"] and st["fmax"] < 1e-6
    assert s.potential_energy() / 1600 == pytest.approx(1.5 * (1 - a) ** 2, rel=1e-5)


def test_fire_converges_and_forces_vanish(md):
    """C2-style packing at N=4096: GPU FIRE reaches max |F| < 1e-6, and an independent GPU evaluation (dense pair
    sum, no list) at the final positions agrees: forces below 2e-6 and the same energy."""
    cfg = ss_cfg(4096, 0.9, 2001)
    s = make_system(md, cfg)
    init, step, minimize = md.fire_descent(s, f_tol=1e-6)
    init()
    st = minimize(200000, chunk=500)
    say("fire steps", st["steps"], "fmax", st["fmax"])
    assert st["converged"]
    import torch
    Fd = torch.zeros_like(s.force)
    ed = torch.zeros(s.N, dtype=torch.float64, device=s.pos.device)
    md.pair_energy_force(s.ctx, s.box, s.pot, s.pos, s.species, None, Fd, ed)
    Fd = Fd.cpu().numpy().astype(np.float64)
    assert np.sqrt((Fd ** 2).sum(1)).max() < 2e-6
    E = s.potential_energy()
    e = ed.cpu().numpy()
    assert abs(E - math.fsum(e)) <= 1e-6 * max(abs(math.fsum(e)), math.fsum(np.abs(e)))


def test_fire_graph_replay_matches_eager(md):
    """FIRE chunks replayed from a captured HIP graph (with eager work and synchronisations between replays)
    give the same state bit for bit as the same chunks launched directly."""
    import torch
    cfg = ss_cfg(2048, 0.9, 2301)
    a, b = make_system(md, cfg), make_system(md, cfg)
    ia, _, ma = md.fire_descent(a, f_tol=1e-30)
    ib, _, mb = md.fire_descent(b, f_tol=1e-30)
    ia()
    ib()
    for k in range(1, 4):
        sa = ma(100 * k, chunk=100, graph=True)
        torch.cuda.synchronize()
        sb = mb(100 * k, chunk=100, graph=False)
        torch.cuda.synchronize()
        assert sa["steps"] == sb["steps"] == 100 * k
        assert torch.equal(a.pos, b.pos) and torch.equal(a.vel, b.vel), k
        assert sa["fmax"] == sb["fmax"]


def test_fire_full_size_packing(md):
    """The C2 workload itself: 65536 bidisperse harmonic disks at phi = 0.90 from uniform positions reach
    max |F| < 1e-6 (graph-replayed chunks), confirmed by the oracle on sampled disks."""
    import time
    import torch
    cfg = inputs.ss_fire()
    c = dict(N=cfg["N"], dim=2, L=cfg["L"], u=cfg["u"], species=cfg["species"], kind="soft_sphere",
             sigma=cfg["sigma"], epsilon=cfg["epsilon"], alpha=2.0, skin=cfg.get("skin", 0.3))
    s = make_system(md, c)
    init, step, minimize = md.fire_descent(s, f_tol=1e-6)
    init()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = minimize(400000, chunk=500, graph=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    say("C2 fire steps", st["steps"], "fmax", st["fmax"], "s", dt, "us/step", 1e6 * dt / max(st["steps"], 1))
    assert st["converged"] and st["fmax"] < 1e-6
    # the FP64 oracle as the checker, on 4096 sampled disks: forces at the returned positions below 2e-6 and the
    # per-disk energies those of the GPU's energy pass (1e-6 of their absolute sum)
    import oracle as orc
    e, _ = s.forces(energy=True)
    rows = np.sort(np.random.default_rng(2002).choice(s.N, 4096, replace=False))
    L = c["L"][:2]
    x = orc.decode(md.from_device_u32(s.pos), L)
    op = orc.Potential("soft_sphere", np.array(c["sigma"]), np.array(c["epsilon"]), alpha=2.0)
    Fo, eo, _ = orc.pair_rows(x, L, op, c["species"], rows=rows)
    assert np.sqrt((Fo ** 2).sum(1)).max() < 2e-6
    eg = e.cpu().numpy()[rows]
    assert np.abs(eg - eo).sum() <= 1e-6 * np.abs(eo).sum()


# --------------------------------------------------------------- full-size sample

def test_lj_large_sampled_parity(md, orc):
    """N = 256000 LJ at the benchmark's box and density: sampled rows bit-exact and sampled forces within
    tolerance, on the FCC lattice moved by seeded offsets of up to 0.1 (so that no two distances coincide)."""
    cfg = dict(inputs.lj_large())
    cfg["u"] = inputs.jittered_torus(cfg["u"], cfg["L"], 0.1, 3101)
    s = make_system(md, cfg)
    s.build()
    s.forces()
    u = cfg["u"]
    rows = np.random.default_rng(0).choice(cfg["N"], 600, replace=False)
    got = s.nl.rows()
    want = orc.neighbors(u, cfg["L"], s.nl.r_list, rows=rows)
    for q, i in enumerate(rows):
        assert np.array_equal(np.sort(got[i]), want[q])
    Fo, _, _ = orc.pair_rows(orc.decode(u, cfg["L"]), cfg["L"], orc_pot(orc, cfg), rows=rows)
    assert rel_l2(s.force.cpu().numpy()[rows], Fo) <= F_TOL


def test_min_distance_and_rms_diff(md, orc):
    """md_min_distance against the brute-force closest pair; md_rms_diff against numpy."""
    import torch
    cfg = lj_cfg(1000, 0.8, 4)
    s = make_system(md, cfg)
    s.build()
    x = orc.decode(cfg["u"], cfg["L"])
    L = np.asarray(cfg["L"], dtype=np.float64)
    d = x[:, None, :] - x[None, :, :]
    d -= L * np.rint(d / L)
    r = np.sqrt((d ** 2).sum(-1))
    np.fill_diagonal(r, np.inf)
    got = float(md.min_distance(s.ctx, s.box, s.pos, s.nl))
    assert got == pytest.approx(r.min(), rel=1e-12)
    a = torch.linspace(-1, 1, 3001, device="cuda")
    b = torch.cos(a * 3)
    want = float(np.sqrt(np.mean((a.cpu().numpy().astype(np.float64) - b.cpu().numpy().astype(np.float64)) ** 2)))
    assert float(md.rms_diff(s.ctx, a, b)) == pytest.approx(want, rel=1e-12)


# ---------------------------------------------------------------------------- degenerate sizes

def test_empty_and_tiny_systems(md, orc):
    """The degenerate sizes of the path.  N = 0: list build, forces, Verlet steps, FIRE, the kinetic energy and the
    energy sum accept the empty system (FIRE reports it converged).  N = 1: no neighbors, zero force, and Verlet
    moves the particle as the oracle does.  N = 2: an LJ dimer's rows, forces and 50 Verlet steps against the
    oracle; two overlapping soft disks relax to contact under FIRE."""
    import torch
    for dim in (2, 3):
        box = md.Box((6.0,) * dim, dim)
        s = md.System(box, md.Potential("lj", [[1.0]], [[1.0]], r_cut=2.5), np.zeros((0, dim), np.uint32),
                      np.zeros((0, dim), np.float32), skin=0.3)
        s.build()
        s.forces()
        init, update = md.nve(s, 0.005)
        init()
        update(5)
        f = s.nl.read_flags()
        assert not (f[md.FLAG_OVERFLOW] or f[md.FLAG_NONFINITE] or f[md.FLAG_STALE]), f
        assert s.kinetic_energy() == 0.0 and s.potential_energy() == 0.0
        d = md.System(box, md.Potential("soft_sphere", [[1.0]], [[1.0]], alpha=2.0), np.zeros((0, dim), np.uint32),
                      None, skin=0.3)
        fi, _, fmin = md.fire_descent(d, f_tol=1e-6)
        fi()
        st = fmin(100)
        assert st["converged"] and st["fmax"] == 0.0, st

    # one particle in a 3D box: no neighbors, ballistic motion
    L = [6.0, 6.0, 6.0]
    x0 = np.array([[1.0, 2.0, 3.0]])
    v0 = np.array([[0.3, -0.2, 0.1]])
    s = md.System(md.Box(tuple(L), 3), md.Potential("lj", [[1.0]], [[1.0]], r_cut=2.5), inputs.to_torus(x0, L),
                  v0.astype(np.float32), skin=0.3)
    init, update = md.nve(s, 0.005)
    init()
    update(40)
    p = orc.Potential("lj", np.ones((1, 1)), np.ones((1, 1)), r_cut=2.5)
    xo, vo, Fo = orc.verlet(orc.decode(inputs.to_torus(x0, L), L), v0, np.zeros((1, 3)), L, p, 0.005, 40)
    dx = torus_x(s.pos.cpu().numpy(), L) - xo
    dx -= np.asarray(L) * np.round(dx / np.asarray(L))
    say("N = 1: position error", np.abs(dx).max(), "force", s.force.cpu().numpy())
    assert np.abs(dx).max() < 1e-6 and not s.force.cpu().numpy().any()
    assert s.nl.lengths().tolist() == [0]

    # an LJ dimer at r = 1.1 in a 3D box
    L = [8.0, 8.0, 8.0]
    u = inputs.to_torus(np.array([[1.0, 1.0, 1.0], [2.1, 1.0, 1.0]]), L)
    s = md.System(md.Box(tuple(L), 3), md.Potential("lj", [[1.0]], [[1.0]], r_cut=2.5), u,
                  np.zeros((2, 3), np.float32), skin=0.3)
    s.build()
    assert [sorted(r.tolist()) for r in s.nl.rows()] == [[1], [0]]
    init, update = md.nve(s, 0.005)
    init()
    x = orc.decode(u, L)
    Fo, _, _ = orc.pair_rows(x, L, p)
    assert rel_l2(s.force.cpu().numpy(), Fo) < F_TOL
    update(50)
    xo, vo, Fo = orc.verlet(x, np.zeros((2, 3)), Fo, L, p, 0.005, 50)
    dx = torus_x(s.pos.cpu().numpy(), L) - xo
    dx -= np.asarray(L) * np.round(dx / np.asarray(L))
    say("dimer: position error", np.abs(dx).max(), "velocity rel-L2", rel_l2(s.vel.cpu().numpy(), vo))
    assert np.abs(dx).max() < 1e-5
    assert rel_l2(s.vel.cpu().numpy(), vo) < 1e-4

    # two overlapping soft disks relax to contact
    L = [8.0, 8.0]
    u = inputs.to_torus(np.array([[3.0, 4.0], [3.7, 4.0]]), L)
    d = md.System(md.Box(tuple(L), 2), md.Potential("soft_sphere", [[1.0]], [[1.0]], alpha=2.0), u, None, skin=0.3)
    fi, _, fmin = md.fire_descent(d, f_tol=1e-6)
    fi()
    st = fmin(20000)
    xd = torus_x(d.pos.cpu().numpy(), L)
    r = xd[1] - xd[0]
    r -= np.asarray(L) * np.round(r / np.asarray(L))
    say("two disks: steps", st["steps"], "fmax", st["fmax"], "r", np.linalg.norm(r))
    assert st["converged"] and st["fmax"] < 1e-6
    assert 1.0 - 2e-6 < np.linalg.norm(r) < 1.05
