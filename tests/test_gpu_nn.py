"""Neural pair potential kernels (descriptors, BF16-MFMA MLP, forces) against the FP64 oracle."""
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
    h = nn.host()   # the oracle uses the BF16-rounded weights, upcast exactly
    Q = nn_oracle.NNParams(W1=h["W1"], b1=h["b1"], W2=h["W2"], b2=h["b2"], w3=h["w3"], b3=h["b3"], m=h["m"],
                           s=h["s"])
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


def test_mlp_matches_oracle_at_bf16_tolerance(md):
    from oracle import nn_oracle
    import oracle as orc
    s, nn, Q, spec, x, L = setup(md, nn_oracle, orc)
    G = md.nn_descriptors(s.ctx, s.box, nn, s.pos, s.nl)
    Ei, e = md.nn_mlp(s.ctx, nn, G)
    Eo, eo, _ = nn_oracle.mlp(G.cpu().numpy().astype(np.float64), Q, spec)
    say("Ei rel-L2", rel_l2(Ei.cpu().numpy(), Eo), "e rel-L2", rel_l2(e.cpu().numpy(), eo))
    assert rel_l2(Ei.cpu().numpy(), Eo) < 1e-2
    assert rel_l2(e.cpu().numpy(), eo) < 2e-2
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
    assert rel_l2(F.cpu().numpy(), Fo) < 1e-2
    assert abs(float(Ei.double().sum()) - Eo) / abs(Eo) < 1e-2
    assert np.abs(F.cpu().numpy().astype(np.float64).sum(0)).max() < 1e-3 * np.abs(Fo).max()
