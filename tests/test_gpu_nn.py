"""Neural pair potential kernels (descriptors, BF16-MFMA MLP, forces, training pass) against the FP64 oracle.

The MLP's weights are BF16 (the model's own values; the oracle uses the same values, upcast exactly) and its
activations enter the MFMA products as BF16 pairs (value + remainder), so inference matches the oracle to
~1e-5; the weight-gradient products take plain BF16 operands, so the gradient matches to ~1e-2.
"""
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


def bf16_round(a):
    """Nearest bfloat16 of the float32 value (ties to even), as float64: the weights the model holds."""
    a32 = np.ascontiguousarray(a, dtype=np.float32)
    b = a32.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64).reshape(np.shape(a))


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def model_params(nn_oracle, W1, b1, W2, b2, w3, b3, m, s):
    """The oracle's copy of the seeded network: BF16 weight matrices and float32 vectors, rounded here."""
    return nn_oracle.NNParams(W1=bf16_round(W1), b1=f32(b1), W2=bf16_round(W2), b2=f32(b2), w3=f32(w3),
                              b3=float(np.float32(b3)), m=f32(m), s=f32(s))


def setup(md, nn_oracle, orc, N=2000, seed=12):
    L = inputs.box_for_density(N, 0.84)
    u = inputs.random_insertion_torus(N, L, 3, 0.85, seed)
    x = orc.decode(u, [L] * 3)
    spec = nn_oracle.NNSpec()
    G, _ = nn_oracle.descriptors(x, [L] * 3, spec)
    P = nn_oracle.init_params(spec, 3, m=G.mean(0), s=G.std(0) + 1e-3)
    P.b1 = np.random.default_rng(1).normal(0, 0.2, 64)
    P.b2 = np.random.default_rng(2).normal(0, 0.2, 64)
    nn = md.NNParams(P.W1, P.b1, P.W2, P.b2, P.w3, P.b3, P.m, P.s)
    Q = model_params(nn_oracle, P.W1, P.b1, P.W2, P.b2, P.w3, P.b3, P.m, P.s)
    h = nn.host()   # the device copy holds exactly those values
    for k in ("W1", "W2", "b1", "b2", "w3", "m", "s"):
        assert np.array_equal(h[k], getattr(Q, k)), k
    box = md.Box((L, L, L), 3)
    s = md.System(box, md.Potential("lj", [[1.0]], [[1.0]], r_cut=2.5), u, skin=0.3)
    s.build()
    return s, nn, Q, spec, x, [L] * 3


def test_descriptors_match_oracle(md):
    from oracle import nn_oracle
    import oracle as orc
    s, nn, Q, spec, x, L = setup(md, nn_oracle, orc)
    G = md.nn_descriptors(s.ctx, s.box, nn, s.pos, s.nl).cpu().numpy()
    Go, _ = nn_oracle.descriptors(x, L, spec)
    say("G rel-L2", rel_l2(G, Go))
    assert rel_l2(G, Go) < 1e-5


@pytest.mark.parametrize("eta", [15.0, 120.0])
def test_descriptors_and_forces_at_other_widths_match_oracle(md, eta):
    """A width parameter eta given in the parameter block (here wider and narrower Gaussians than the default
    1/(2 Delta^2) = 38.9) gives the oracle's descriptors, and the network forces through it the oracle's."""
    from oracle import nn_oracle
    import oracle as orc
    s, nn, Q, spec, x, L = setup(md, nn_oracle, orc)
    nn.eta = eta
    spec = nn_oracle.NNSpec(width=eta)
    G = md.nn_descriptors(s.ctx, s.box, nn, s.pos, s.nl)
    Go, _ = nn_oracle.descriptors(x, L, spec)
    say("eta", eta, "G rel-L2", rel_l2(G.cpu().numpy(), Go))
    assert rel_l2(G.cpu().numpy(), Go) < 1e-5
    import torch
    _, e = md.nn_mlp(s.ctx, nn, G)
    F = torch.zeros_like(s.force)
    md.nn_forces(s.ctx, s.box, nn, s.pos, s.nl, e, F)
    _, _, Fo, _, _ = nn_oracle.energy_forces(x, L, Q, spec)
    say("eta", eta, "F rel-L2", rel_l2(F.cpu().numpy(), Fo))
    assert rel_l2(F.cpu().numpy(), Fo) < 1e-4


def test_mlp_matches_oracle(md):
    from oracle import nn_oracle
    import oracle as orc
    s, nn, Q, spec, x, L = setup(md, nn_oracle, orc)
    import torch
    # both networks read the same descriptor matrix: the oracle's, from the seeded positions, in float32
    Go, _ = nn_oracle.descriptors(x, L, spec)
    G32 = Go.astype(np.float32)
    G = torch.as_tensor(G32, device="cuda").contiguous()
    Ei, e = md.nn_mlp(s.ctx, nn, G)
    Eo, eo, _ = nn_oracle.mlp(G32.astype(np.float64), Q, spec)
    say("Ei rel-L2", rel_l2(Ei.cpu().numpy(), Eo), "e rel-L2", rel_l2(e.cpu().numpy(), eo))
    assert rel_l2(Ei.cpu().numpy(), Eo) < 1e-4
    assert rel_l2(e.cpu().numpy(), eo) < 1e-4
    # a partial last tile: N not a multiple of 32
    Ei2, e2 = md.nn_mlp(s.ctx, nn, G[:1001].contiguous())
    assert np.array_equal(Ei2.cpu().numpy(), Ei.cpu().numpy()[:1001])


def test_forces_match_oracle(md):
    from oracle import nn_oracle
    import oracle as orc
    import torch
    s, nn, Q, spec, x, L = setup(md, nn_oracle, orc)
    G = md.nn_descriptors(s.ctx, s.box, nn, s.pos, s.nl)
    Ei, e = md.nn_mlp(s.ctx, nn, G)
    F = torch.zeros_like(s.force)
    md.nn_forces(s.ctx, s.box, nn, s.pos, s.nl, e, F)
    Eo, _, Fo, _, _ = nn_oracle.energy_forces(x, L, Q, spec)
    say("F rel-L2", rel_l2(F.cpu().numpy(), Fo), "E", float(Ei.double().sum()), Eo)
    assert rel_l2(F.cpu().numpy(), Fo) < 1e-4
    assert abs(float(Ei.double().sum()) - Eo) / abs(Eo) < 1e-4
    assert np.abs(F.cpu().numpy().astype(np.float64).sum(0)).max() < 1e-3 * np.abs(Fo).max()


def train_setup(md, S=3, n=400, seed=21):
    """S independent LJ-like configurations of n atoms as one segmented system, a network with nonzero biases,
    and arbitrary reference energies / forces (the gradient check does not need physical references)."""
    import torch
    from paper_1912_04232_amd import nn as nnmod
    import oracle as orc
    from oracle import nn_oracle
    L = inputs.box_for_density(n, 0.84)
    us = [inputs.random_insertion_torus(n, L, 3, 0.85, seed + k) for k in range(S)]
    xs = [orc.decode(u, [L] * 3) for u in us]
    spec = nn_oracle.NNSpec()
    G0 = np.concatenate([nn_oracle.descriptors(x, [L] * 3, spec)[0] for x in xs])
    w = inputs.nn_init(7)
    rng = np.random.default_rng(seed)
    w["b1"], w["b2"], w["b3"] = rng.normal(0, 0.3, 64), rng.normal(0, 0.3, 64), 0.4
    ctx = md.Context()
    net = nnmod.Network(ctx, w, G0.mean(0), G0.std(0) + 1e-3)
    box = md.Box((L, L, L), 3)
    pos = torch.as_tensor(np.concatenate(us).view(np.int32), device="cuda").contiguous()
    E_np = rng.normal(-5.0 * n, 30.0, S)
    F_np = rng.normal(0, 3.0, (S * n, 3)).astype(np.float32)
    E_ref = torch.as_tensor(E_np, dtype=torch.float64, device="cuda")
    F_ref = torch.as_tensor(F_np, device="cuda")
    batch = nnmod.Batch(ctx, box, net, pos, E_ref, F_ref, n, 2.5)
    Q = model_params(nn_oracle, w["W1"], w["b1"], w["W2"], w["b2"], w["w3"], w["b3"], G0.mean(0), G0.std(0) + 1e-3)
    h = net.host()   # the device copy (float32 master values, BF16 matrices from the cast kernel) holds them exactly
    for k in ("W1", "W2", "b1", "b2", "w3", "m", "s"):
        assert np.array_equal(h[k], getattr(Q, k)), k
    snaps = [(xs[k], [L] * 3, float(E_np[k]), F_np[k * n:(k + 1) * n].astype(np.float64)) for k in range(S)]
    return ctx, box, net, batch, Q, spec, snaps, xs, [L] * 3, nnmod


def test_loss_and_pair_adjoint_match_oracle(md):
    ctx, box, net, batch, Q, spec, snaps, xs, L, nnmod = train_setup(md)
    from oracle import nn_oracle
    Ei, e = nnmod.mlp(ctx, net, batch.G)
    F = nnmod.forces(ctx, box, net, batch.pos, batch.nl, e)
    loss, gE, lam = nnmod.loss(ctx, Ei, F, batch.E_ref, batch.F_ref, batch.n)
    lo, _ = nn_oracle.loss_and_grad(snaps, Q, spec)
    say("loss", float(loss), lo)
    assert abs(float(loss) - lo) / lo < 1e-4
    # the pair adjoint is linear in lam: both sides transpose the same seeded vector
    import torch
    n = batch.n
    lam_h = np.random.default_rng(77).normal(0.0, 1.0, (len(xs) * n, 3)).astype(np.float32)
    lam_d = torch.as_tensor(lam_h, device="cuda").contiguous()
    ebar = nnmod.pair_adjoint(ctx, box, net, batch.pos, batch.nl, lam_d).cpu().numpy()
    lam_h = lam_h.astype(np.float64)
    want = np.concatenate([nn_oracle.pair_adjoint(xs[k], L, spec, lam_h[k * n:(k + 1) * n]) for k in range(len(xs))])
    say("ebar rel-L2", rel_l2(ebar, want))
    assert rel_l2(ebar, want) < 1e-5


def test_weight_gradient_matches_oracle(md):
    """The full training gradient (energy and force terms, through the pair adjoint and the network's tangent)
    against the oracle's analytic gradient, parameter group by parameter group."""
    ctx, box, net, batch, Q, spec, snaps, xs, L, nnmod = train_setup(md)
    from oracle import nn_oracle
    Ei, e = nnmod.mlp(ctx, net, batch.G)
    F = nnmod.forces(ctx, box, net, batch.pos, batch.nl, e)
    loss, gE, lam = nnmod.loss(ctx, Ei, F, batch.E_ref, batch.F_ref, batch.n)
    ebar = nnmod.pair_adjoint(ctx, box, net, batch.pos, batch.nl, lam)
    grad = nnmod.mlp_grad(ctx, net, batch.G, batch.n, gE, ebar).cpu().numpy().astype(np.float64)
    _, go = nn_oracle.loss_and_grad(snaps, Q, spec)
    K, H = 16, 64
    parts = dict(W1=grad[:H * K].reshape(H, K), b1=grad[H * K:H * K + H],
                 W2=grad[H * K + H:H * K + H + H * H].reshape(H, H), b2=grad[H * K + H + H * H:H * K + 2 * H + H * H],
                 w3=grad[H * K + 2 * H + H * H:H * K + 3 * H + H * H], b3=grad[-1:])
    for k, v in parts.items():
        r = rel_l2(v, np.atleast_1d(go[k]))
        say("grad", k, r)
        assert r < 2e-2, (k, r)


def test_adam_step_and_bf16_copies(md):
    """One Adam step from zero moments moves every parameter with a nonzero gradient by lr (bias-corrected), and
    the BF16 copies are the master weights rounded to nearest even."""
    import torch
    ctx, box, net, batch, Q, spec, snaps, xs, L, nnmod = train_setup(md, S=1)
    th0 = net.theta.clone()
    g = torch.linspace(-1.0, 1.0, net.P, device="cuda")
    net.adam(ctx, g, 1e-3)
    step = (net.theta - th0).cpu().numpy()
    gg = g.cpu().numpy()
    nz = np.abs(gg) > 1e-3
    assert np.allclose(step[nz], -1e-3 * np.sign(gg[nz]), rtol=1e-3, atol=1e-9)
    w1 = net.theta[:16 * 64].cpu().numpy()
    want = torch.as_tensor(w1).to(torch.bfloat16).view(torch.int16).numpy()
    assert np.array_equal(net.W1.cpu().numpy(), want)


def test_network_md_graph_replay_matches_eager_and_judge_falls_back(md):
    """Network NVE: the captured HIP graph of 20 steps, replayed with eager work and synchronisations in between,
    gives bit-identical states to the same steps run eagerly; a threshold below the untrained network's force
    RMSE hands the run to plain LJ."""
    import torch
    from paper_1912_04232_amd import nn as nnmod
    ctx = md.Context()
    n_cells = 6
    N = 4 * n_cells ** 3
    L = inputs.box_for_density(N, 0.84)
    u = inputs.fcc_torus(n_cells, L)
    v = inputs.maxwell_velocities(N, 3, 1.0, 9)
    box = md.Box((L, L, L), 3)
    w = inputs.nn_init(3)
    w["w3"] = w["w3"] * 0.01  # a gentle untrained network, so the dynamics stay bounded
    net = nnmod.Network(ctx, w, np.full(16, 2.0), np.full(16, 3.0))
    a = nnmod.NNMD(ctx, net, box, u, v, chunk=20, max_rmse=1e9)
    b = nnmod.NNMD(ctx, net, box, u, v, chunk=20, max_rmse=1e9)
    for rep in range(3):
        a._replay(20 if rep else 21)
        torch.cuda.synchronize()
        b._eager(20 if rep else 21)
        torch.cuda.synchronize()
        assert torch.equal(a.sys.pos, b.sys.pos), rep
        assert torch.equal(a.sys.vel, b.sys.vel), rep
    c = nnmod.NNMD(ctx, net, box, u, v, chunk=20, max_rmse=1e-3, check_every=20)
    done = c.run(100)
    say("fallback after", done, "rmse", c.rmse_log)
    assert c.fallback and done == 20 and c.steps == 100


def test_trained_network_beats_untrained_and_runs_md(md):
    """What training buys: on held-out plain-engine snapshots the trained network's force RMSE is a small
    fraction of the untrained one's; network MD at N = 4000 then runs with the LJ judge below threshold."""
    from paper_1912_04232_amd import nn as nnmod
    ctx = md.Context()
    net, box, test, rec = nnmod.train_network(ctx, n_runs=6, per_run=20, steps=3000, per_batch=8, progress=say)
    say("training record", rec)
    assert rec["force_rmse"] < 0.1 * rec["force_rmse_untrained"]
    assert rec["force_rmse"] < 0.1 * rec["force_rms_reference"]
    u = inputs.fcc_torus(10, box.L[0])
    v = inputs.maxwell_velocities(4000, 3, 1.0, 17)
    sim = nnmod.NNMD(ctx, net, box, u, v, max_rmse=5.0 * rec["force_rmse"], check_every=100)
    done = sim.run(500)
    say("md rmse", sim.rmse_log, "fallback", sim.fallback)
    assert all(np.isfinite(sim.rmse_log))
    assert sim.steps == 500
