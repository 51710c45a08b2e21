"""Batched FIRE and the envelope adjoint on the GPU, against the FP64 oracle and finite differences."""
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


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def replicas(B, seed, n_lo=256, n_hi=700):
    return inputs.ss_batch(B=B, seed=seed, n_lo=n_lo, n_hi=n_hi)


def ss_pot(md, d=(1.0, 1.4), eps=1.0):
    d = np.asarray(d, dtype=np.float64)
    return md.Potential("soft_sphere", 0.5 * (d[:, None] + d[None, :]), np.full((len(d), len(d)), eps), alpha=2.0)


def orc_pot(orc, d=(1.0, 1.4), eps=1.0):
    d = np.asarray(d, dtype=np.float64)
    return orc.Potential("soft_sphere", 0.5 * (d[:, None] + d[None, :]), np.full((len(d), len(d)), eps), alpha=2.0)


def test_batched_fire_converges(md):
    """Every replica reaches max |F| < 1e-6; a second GPU path (the dense pair sum of pair_energy_force, one
    replica at a time) confirms the forces and the energies at the returned positions."""
    import torch
    reps = replicas(6, 4101)
    say("sizes", [r["N"] for r in reps])
    ctx = md.Context()
    bt = md.Batch(reps)
    e, fmax, steps, status = md.fire_batched(ctx, bt, ss_pot(md), md.FireParams(), 200000, 1e-6)
    e, fmax, steps, status = (t.cpu().numpy() for t in (e, fmax, steps, status))
    say("steps", steps.tolist(), "fmax", fmax.tolist())
    assert (status == 1).all() and (fmax < 1e-6).all()
    for b, r in enumerate(reps):
        box = md.Box(tuple(float(x) for x in r["L"][:2]), 2)
        pos = md.to_device_u32(bt.replica_positions(b), "cuda")
        sp = torch.as_tensor(np.asarray(r["species"], dtype=np.int32), device="cuda")
        F = torch.zeros((r["N"], 2), dtype=torch.float32, device="cuda")
        eg = torch.zeros(r["N"], dtype=torch.float64, device="cuda")
        md.pair_energy_force(ctx, box, ss_pot(md), pos, sp, None, F, eg)
        F = F.cpu().numpy().astype(np.float64)
        eg = eg.cpu().numpy()
        assert np.sqrt((F ** 2).sum(1)).max() < 2e-6
        assert abs(e[b] - math.fsum(eg)) <= 1e-6 * max(abs(math.fsum(eg)), math.fsum(np.abs(eg)))


def test_batched_fire_matches_oracle_fire_from_same_start(md, orc):
    """Small packings, where the float32 and float64 minimizations from the same seeded start end in the same
    minimum: the minimized energies agree with the oracle's FIRE run from that start (GPU to max |F| < 1e-7,
    above its float32 force floor of ~1e-8; oracle to 1e-11)."""
    reps = []
    for N, phi, seed in ((40, 0.9, 4111), (48, 0.88, 4112), (64, 0.85, 4113)):
        L = inputs.box_for_packing([1.0, 1.4], [N // 2, N // 2], phi, 2)
        reps.append(dict(N=N, L=np.array([L, L, 0.0]), u=inputs.uniform_torus(N, 2, seed),
                         species=inputs.bidisperse_species(N)))
    ctx = md.Context()
    e, fmax, steps, status = (t.cpu().numpy() for t in
                              md.fire_batched(ctx, md.Batch(reps), ss_pot(md), md.FireParams(), 400000, 1e-7))
    for b, r in enumerate(reps):
        L = r["L"][:2]
        o = orc.fire(orc.decode(r["u"], L), L, orc_pot(orc), r["species"], f_tol=1e-11, max_steps=400000)
        assert o["converged"]
        Eo = orc.energy(o["x"], L, orc_pot(orc), r["species"])
        say("N", r["N"], "E* gpu", e[b], "oracle", Eo, "fmax", fmax[b], "steps", steps[b], o["steps"])
        assert status[b] == 1
        assert abs(e[b] - Eo) <= 1e-6 * abs(Eo) + 1e-12


@pytest.mark.parametrize("K", [1, 5])
def test_batched_fire_first_steps_match_oracle_at_workload_sizes(md, orc, K):
    """K FIRE steps (f_tol 0) of fire_batched against the oracle's FIRE from the same seeded starts, at the replica
    sizes of the batched workload (N = 1024 and 4096, which fill the 512-thread workgroup and its LDS cell list, and
    a ragged 1538), at packing fractions 0.84 and 0.92: the displacements from the start agree to 1e-4 (rel-L2) and
    the energies after K steps to 1e-6."""
    reps = []
    for N, phi, seed in ((1024, 0.84, 4501), (4096, 0.92, 4502), (1538, 0.88, 4503)):
        L = inputs.box_for_packing([1.0, 1.4], [N // 2, N // 2], phi, 2)
        reps.append(dict(N=N, L=np.array([L, L, 0.0]), u=inputs.uniform_torus(N, 2, seed),
                         species=inputs.bidisperse_species(N)))
    ctx = md.Context()
    bt = md.Batch(reps)
    e, fmax, steps, status = (t.cpu().numpy() for t in
                              md.fire_batched(ctx, bt, ss_pot(md), md.FireParams(), K, 0.0))
    op = orc_pot(orc)
    for b, r in enumerate(reps):
        L = r["L"][:2]
        x0 = orc.decode(r["u"], L)
        o = orc.fire(x0, L, op, r["species"], max_steps=K, f_tol=0.0)
        xg = orc.decode(bt.replica_positions(b), L)
        dg = xg - x0
        dg -= np.asarray(L) * np.rint(dg / np.asarray(L))
        do = o["x"] - x0
        do -= np.asarray(L) * np.rint(do / np.asarray(L))
        Eo = orc.energy(o["x"], L, op, r["species"])
        say("K", K, "N", r["N"], "displacement rel-L2", rel_l2(dg, do), "E", e[b], Eo)
        assert steps[b] == K and status[b] == 0
        assert rel_l2(dg, do) < 1e-4
        assert abs(e[b] - Eo) <= 1e-6 * abs(Eo)


def test_batched_replicas_are_independent(md):
    """A replica's result does not depend on the other replicas in the batch (bitwise)."""
    reps = replicas(5, 4202)
    ctx = md.Context()
    full = md.Batch(reps)
    out_full = md.fire_batched(ctx, full, ss_pot(md), md.FireParams(), 50000, 1e-6)
    one = md.Batch([reps[3]])
    out_one = md.fire_batched(ctx, one, ss_pot(md), md.FireParams(), 50000, 1e-6)
    assert np.array_equal(full.replica_positions(3), one.replica_positions(0))
    assert out_full[0].cpu().numpy()[3] == out_one[0].cpu().numpy()[0]
    assert out_full[2].cpu().numpy()[3] == out_one[2].cpu().numpy()[0]


def test_envelope_grad_matches_oracle_at_same_positions(md, orc):
    """dU/dsigma_ab, dU/deps_ab and U at the seeded positions of uneven replicas (the kernel is a function of the
    positions; at a minimum it is dE*/dtheta)."""
    reps = replicas(4, 4303)
    ctx = md.Context()
    bt = md.Batch(reps)
    d = np.array([1.0, 1.4])
    import torch
    pot = ss_pot(md, d)
    gs, ge, e = (t.cpu().numpy() for t in md.envelope_grad(ctx, bt, pot))
    # the library's chain rule: per-species diameters (sigma_ab = (d_a + d_b)/2) and one shared epsilon
    gd = md.envelope_grad_wrt(ctx, bt, pot, md.WRT_DIAMETER).cpu().numpy()
    gE = md.envelope_grad_wrt(ctx, bt, pot, md.WRT_EPSILON_COMMON).cpu().numpy()[:, 0]
    w = torch.tensor([0.5, -1.0, 2.0, 0.25][: len(reps)], dtype=torch.float64, device=bt.pos.device)
    gdw = md.envelope_grad_wrt(ctx, bt, pot, md.WRT_DIAMETER, weights=w).cpu().numpy()
    g_all = []
    for b, r in enumerate(reps):
        x = orc.decode(r["u"], r["L"][:2])
        g_orc = orc.diameter_grad(x, r["L"][:2], d, 1.0, r["species"])
        g_all.append(g_orc)
        g_gpu = 0.5 * (gs[b].sum(1) + gs[b].sum(0))
        assert np.allclose(g_gpu, g_orc, rtol=1e-5, atol=1e-9 * np.abs(g_orc).max()), (b, g_gpu, g_orc)
        assert np.allclose(gd[b], g_orc, rtol=1e-5, atol=1e-9 * np.abs(g_orc).max()), (b, gd[b], g_orc)
        # dE/deps = E/eps at any positions
        assert ge[b].sum() == pytest.approx(e[b], rel=1e-6)
        assert gE[b] == pytest.approx(e[b], rel=1e-6)
    want = (w.cpu().numpy()[:, None] * np.array(g_all)).sum(0)
    assert np.allclose(gdw, want, rtol=1e-5, atol=1e-9 * np.abs(want).max())


def test_adjoint_autograd_matches_finite_differences(md):
    """d E*/d d_s from the autograd.Function (batched FIRE forward, envelope_grad backward) against central
    differences of the same GPU pipeline, h = 1e-4, box fixed.  The perturbed minimizations start from the
    minimum R* itself, so they follow that minimum (at a few hundred particles a restart from the random
    initial state can land in another basin, where E* jumps)."""
    import torch

    from paper_1912_04232_amd.adjoint import minimized_energy
    reps = replicas(3, 4404, 256, 400)
    ctx = md.Context()
    bt = md.Batch(reps)
    u0 = bt.pos.clone()
    d = torch.tensor([1.0, 1.4], dtype=torch.float64, requires_grad=True)
    eps = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    E = minimized_energy(d, eps, bt, u0, f_tol=1e-7, md_ctx=ctx)
    u_star = bt.pos.clone()
    w = torch.tensor([1.0, -0.5, 2.0], dtype=torch.float64)
    (E.cpu() * w).sum().backward()
    grad = d.grad.numpy().copy()
    h = 1e-4
    fd = []
    for s in range(2):
        vals = []
        for sgn in (1, -1):
            dd = d.detach().clone()
            dd[s] += sgn * h
            vals.append(float((minimized_energy(dd, eps.detach(), bt, u_star, f_tol=1e-7, md_ctx=ctx).cpu()
                               * w).sum()))
        fd.append((vals[0] - vals[1]) / (2 * h))
    say("adjoint", grad, "fd", fd, "E*", E.detach().cpu().numpy())
    assert np.allclose(grad, fd, rtol=2e-3, atol=1e-6)
    assert float(eps.grad) == pytest.approx(float((E.detach().cpu() * w).sum()), rel=1e-6)


def test_adjoint_same_start_small_packing(md, orc):
    """The App. A protocol at a size where every restart stays in one basin: N = 40 bidisperse disks at
    phi = 0.9, each E*(d +- h) minimized from the same random start.  The GPU adjoint matches the central
    differences of the oracle's own FIRE (FP64) and the oracle's gradient at the oracle's minimum."""
    import torch

    from paper_1912_04232_amd.adjoint import minimized_energy
    N = 40
    L = inputs.box_for_packing([1.0, 1.4], [N // 2, N // 2], 0.9, 2)
    u = inputs.uniform_torus(N, 2, 77)
    sp = inputs.bidisperse_species(N)
    rep = dict(N=N, L=np.array([L, L, 0.0]), u=u, species=sp)
    ctx = md.Context()
    bt = md.Batch([rep])
    u0 = bt.pos.clone()
    d = torch.tensor([1.0, 1.4], dtype=torch.float64, requires_grad=True)
    E = minimized_energy(d, torch.tensor(1.0, dtype=torch.float64), bt, u0, f_tol=1e-7, md_ctx=ctx)
    E.sum().backward()
    grad = d.grad.numpy()
    x0 = orc.decode(u, [L, L])
    o_star = orc.fire(x0, [L, L], orc_pot(orc), sp, f_tol=1e-11, max_steps=200000)
    assert o_star["converged"]
    g_orc = orc.diameter_grad(o_star["x"], [L, L], np.array([1.0, 1.4]), 1.0, sp)
    h = 1e-4
    fd = []
    for s in range(2):
        vals = []
        for sgn in (1, -1):
            dd = np.array([1.0, 1.4])
            dd[s] += sgn * h
            r = orc.fire(x0, [L, L], orc_pot(orc, dd), sp, f_tol=1e-11, max_steps=200000)
            assert r["converged"]
            vals.append(orc.energy(r["x"], [L, L], orc_pot(orc, dd), sp))
        fd.append((vals[0] - vals[1]) / (2 * h))
    say("adjoint", grad, "oracle grad at its own minimum", g_orc, "oracle fd", fd)
    assert np.allclose(grad, g_orc, rtol=1e-4, atol=1e-8)
    assert np.allclose(grad, fd, rtol=1e-3, atol=1e-8)


def test_batch_of_uneven_sizes_full_range(md, orc):
    """The C4 shape: 64 packings with N from 256 to 4096 in one launch all reach max |F| < 1e-6, confirmed by the
    oracle's forces and energies at the returned positions."""
    reps = inputs.ss_batch()
    ctx = md.Context()
    bt = md.Batch(reps)
    e, fmax, steps, status = (t.cpu().numpy() for t in
                              md.fire_batched(ctx, bt, ss_pot(md), md.FireParams(), 400000, 1e-6))
    say("N range", min(bt.sizes), max(bt.sizes), "steps", int(steps.min()), int(steps.max()),
        "converged", int((status == 1).sum()))
    assert (status == 1).all()
    assert (fmax < 1e-6).all()
    # the FP64 oracle, as the checker of these results: every replica's forces at the returned positions are
    # below 2e-6 (the single-precision force floor adds ~1e-9) and its energy is the returned one
    op = orc_pot(orc)
    for b, r in enumerate(reps):
        L = r["L"][:2]
        x = orc.decode(bt.replica_positions(b), L)
        F, ei, _ = orc.pair_rows(x, L, op, r["species"])
        Eo = math.fsum(ei)
        assert np.sqrt((F ** 2).sum(1)).max() < 2e-6, (b, np.sqrt((F ** 2).sum(1)).max())
        assert abs(e[b] - Eo) <= 1e-6 * math.fsum(np.abs(ei)) + 1e-12, (b, e[b], Eo)


def test_adjoint_matches_oracle_fd_at_workload_size(md, orc):
    """The C4 check at replica size N = 256: for seeded packings where the GPU's and the oracle's FIRE from the same
    start reach the same minimum (the same E* to 1e-6; float32 and float64 runs can part at a P > 0 decision), the
    GPU adjoint (envelope_grad_wrt through the autograd function) equals central differences (h = 1e-4) of the
    oracle's minimized energy, each E*(d +- h) minimized by the oracle from the oracle's own minimum at d so that it
    follows that basin.  Two packings (phi 0.84 and 0.88) are required."""
    import torch

    from paper_1912_04232_amd.adjoint import minimized_energy
    ctx = md.Context()
    op = orc_pot(orc)
    done = 0
    for phi, seed in ((0.84, 4601), (0.84, 4602), (0.88, 4603), (0.88, 4604), (0.84, 4605), (0.88, 4606)):
        if done >= 2:
            break
        N = 256
        L = inputs.box_for_packing([1.0, 1.4], [N // 2, N // 2], phi, 2)
        u = inputs.uniform_torus(N, 2, seed)
        sp = inputs.bidisperse_species(N)
        bt = md.Batch([dict(N=N, L=np.array([L, L, 0.0]), u=u, species=sp)])
        u0 = bt.pos.clone()
        d = torch.tensor([1.0, 1.4], dtype=torch.float64, requires_grad=True)
        E = minimized_energy(d, torch.tensor(1.0, dtype=torch.float64), bt, u0, f_tol=1e-7, md_ctx=ctx)
        E.sum().backward()
        grad = d.grad.numpy()
        o = orc.fire(orc.decode(u, [L, L]), [L, L], op, sp, f_tol=1e-11, max_steps=400000)
        assert o["converged"]
        Eo = orc.energy(o["x"], [L, L], op, sp)
        if abs(float(E[0]) - Eo) > 1e-6 * abs(Eo):
            say("phi", phi, "seed", seed, "different minima", float(E[0]), Eo)
            continue
        h = 1e-4
        fd = []
        for sidx in range(2):
            vals = []
            for sgn in (1, -1):
                dd = np.array([1.0, 1.4])
                dd[sidx] += sgn * h
                r = orc.fire(o["x"], [L, L], orc_pot(orc, dd), sp, f_tol=1e-11, max_steps=400000)
                assert r["converged"]
                vals.append(orc.energy(r["x"], [L, L], orc_pot(orc, dd), sp))
            fd.append((vals[0] - vals[1]) / (2 * h))
        say("phi", phi, "seed", seed, "E*", Eo, "adjoint", grad, "oracle fd", fd)
        assert np.allclose(grad, fd, rtol=1e-4, atol=1e-7)
        done += 1
    assert done >= 2, done


def test_autotuned_launch_shapes_give_the_same_minima(md, orc):
    """autotune_fire_batched times every launch shape on the batch and returns one of them; every shape minimizes
    small packings (unique basins) to the oracle's minimized energies."""
    reps = []
    for N, phi, seed in ((40, 0.9, 4111), (48, 0.88, 4112), (64, 0.85, 4113)):
        L = inputs.box_for_packing([1.0, 1.4], [N // 2, N // 2], phi, 2)
        reps.append(dict(N=N, L=np.array([L, L, 0.0]), u=inputs.uniform_torus(N, 2, seed),
                         species=inputs.bidisperse_species(N)))
    ctx = md.Context()
    bt = md.Batch(reps)
    u0 = bt.pos.clone()
    tune = md.autotune_fire_batched(ctx, bt, ss_pot(md), trial_steps=50)
    say("autotune", tune)
    assert tune["config"] in md.BATCH_CONFIGS and len(tune["ms_per_trial"]) == len(md.BATCH_CONFIGS)
    assert np.array_equal(bt.pos.cpu().numpy(), u0.cpu().numpy())   # the trials leave the batch where it was
    op = orc_pot(orc)
    want = []
    for r in reps:
        L = r["L"][:2]
        o = orc.fire(orc.decode(r["u"], L), L, op, r["species"], f_tol=1e-11, max_steps=400000)
        want.append(orc.energy(o["x"], L, op, r["species"]))
    for cfg in md.BATCH_CONFIGS:
        bt.pos.copy_(u0)
        e, fmax, steps, status = (t.cpu().numpy() for t in
                                  md.fire_batched(ctx, bt, ss_pot(md), md.FireParams(), 400000, 1e-7, config=cfg))
        assert (status == 1).all(), cfg
        for b in range(len(reps)):
            assert abs(e[b] - want[b]) <= 1e-6 * abs(want[b]) + 1e-12, (cfg, b, e[b], want[b])


# ------------------------------------------------------------ box rescaled with the small-disk diameter

def fig3_starts(n, count, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return [rng.integers(0, 2 ** 32, size=(n, 2), dtype=np.uint64).astype(np.uint32) for _ in range(count)]


def test_rescaled_box_grad_matches_oracle(md, orc):
    """dU/dD with the box rescaled with D (App. A) at fixed fractional positions (envelope_grad_wrt, diameter of
    species 0, packing box), against the FP64 oracle at the same seeded positions, for several D around the
    disorder maximum."""
    ctx = md.Context()
    starts = fig3_starts(64, 4, 5101)
    sp = inputs.bidisperse_species(64)
    for D in (0.6, 0.8, 1.0):
        L = inputs.box_for_packing([D, 1.0], [32, 32], 0.9, 2)
        reps = [dict(N=64, L=[L, L, 0.0], u=u, species=sp) for u in starts]
        bt = md.Batch(reps)
        pot = ss_pot(md, (D, 1.0))
        _, _, e = md.envelope_grad(ctx, bt, pot)
        g = md.envelope_grad_wrt(ctx, bt, pot, md.WRT_DIAMETER, md.BOX_PACKING)[:, 0].cpu().numpy()
        e = e.cpu().numpy()
        for b, u in enumerate(starts):
            U, go = orc.rescaled_box_grad(u, float(np.float32(L)), D, sp)
            say("D", D, "b", b, "U", e[b], U, "dU/dD", g[b], go)
            assert abs(e[b] - U) <= 1e-6 * max(abs(U), 1e-12) + 1e-12
            assert abs(g[b] - go) <= 1e-5 * max(abs(go), 1e-3)


def test_rescaled_box_sweep_minima_and_fd(md):
    """The sweep's minimizations converge, and its envelope dE*/dD matches central differences of the GPU's own
    minimized energy E*(D +- h), each re-minimized from the minimum at D (h = 1e-3: float32 resolves E* to ~1e-7)."""
    from paper_1912_04232_amd import adjoint
    ctx = md.Context()
    starts = fig3_starts(64, 3, 5202)
    D, h = 0.8, 1e-3
    res, batches = adjoint.rescaled_box_sweep(ctx, [D], starts, 0.9, f_tol=1e-7)
    assert (res["status"] == 1).all() and (res["fmax"] < 1e-7).all()
    mins = [batches[0].replica_positions(b) for b in range(len(starts))]
    rp, _ = adjoint.rescaled_box_sweep(ctx, [D + h], mins, 0.9, f_tol=1e-8)
    rm, _ = adjoint.rescaled_box_sweep(ctx, [D - h], mins, 0.9, f_tol=1e-8)
    fd = (rp["energy"][0] - rm["energy"][0]) / (2 * h)
    say("fd", fd, "envelope", res["dEdD"][0])
    assert np.allclose(res["dEdD"][0], fd, rtol=2e-3, atol=1e-4)
