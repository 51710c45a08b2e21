"""Pins of the FP64 neural-potential oracle: finite differences, a linear network that reduces to a pair
potential, invariances, and finite differences of the training loss (including its force term)."""
import math

import numpy as np
import pytest

from paper_1912_04232_amd import inputs


@pytest.fixture(scope="module")
def nn():
    from oracle import nn_oracle
    return nn_oracle


def config(N=60, rho=0.84, seed=3):
    L = inputs.box_for_density(N, rho)
    u = inputs.random_insertion_torus(N, L, 3, 0.85, seed)
    from oracle import decode
    return decode(u, [L] * 3), [L, L, L]


def params(nn, spec, seed=5):
    P = nn.init_params(spec, seed)
    P.m = np.linspace(0.1, 1.5, spec.K)
    P.s = np.linspace(0.5, 2.0, spec.K)
    rng = np.random.default_rng(seed)
    P.b1 = rng.normal(0, 0.3, spec.H)
    P.b2 = rng.normal(0, 0.3, spec.H)
    P.b3 = 0.7
    return P


@pytest.mark.parametrize("width", [0.0, 15.0, 120.0])
def test_descriptor_width_from_a_dimer(nn, width):
    """A dimer at r = mu_5 (a basis centre): G^5 = f_c(r) of each atom, the neighbors G^4 = G^6 by symmetry, and
    -ln(G^6 / G^5) / Delta^2 recovers the width eta (the default 1/(2 Delta^2) when width is 0).  A wrong width, a
    sign or a missing square in the Gaussian fails one of these."""
    spec = nn.NNSpec(width=width)
    delta = (spec.mu1 - spec.mu0) / (spec.K - 1)
    eta = width if width > 0 else 1.0 / (2.0 * delta * delta)
    r = spec.mu[5]
    L = [10.0, 10.0, 10.0]
    x = np.array([[1.0, 2.0, 3.0], [1.0 + r, 2.0, 3.0]])
    G, _ = nn.descriptors(x, L, spec)
    fc = 0.5 * (math.cos(math.pi * r / spec.r_c) + 1.0)
    assert np.allclose(G[0], G[1], rtol=0, atol=1e-15)
    assert math.isclose(G[0, 5], fc, rel_tol=1e-12)
    assert math.isclose(G[0, 4], G[0, 6], rel_tol=1e-9)
    assert math.isclose(-math.log(G[0, 6] / G[0, 5]) / delta ** 2, eta, rel_tol=1e-9)


def test_basis_constants(nn):
    spec = nn.NNSpec()
    assert np.allclose(spec.mu[[0, -1]], [0.8, 2.5])
    assert math.isclose(spec.eta, 1.0 / (2 * (1.7 / 15) ** 2))
    g, dg = nn.basis(np.array([2.5 - 1e-12, 1.2]), spec)
    assert np.abs(g[0]).max() < 1e-20 and np.abs(dg[0]).max() < 1e-9   # smooth cutoff at r_c


def test_forces_are_minus_gradient(nn):
    spec = nn.NNSpec()
    x, L = config()
    P = params(nn, spec)
    E, Ei, F, e, G = nn.energy_forces(x, L, P, spec)
    h = 1e-5
    rng = np.random.default_rng(0)
    for i in rng.choice(len(x), 5, replace=False):
        for k in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, k] += h
            xm[i, k] -= h
            fd = -(nn.energy_forces(xp, L, P, spec)[0] - nn.energy_forces(xm, L, P, spec)[0]) / (2 * h)
            assert abs(fd - F[i, k]) < 1e-6 * max(1.0, abs(F[i, k])), (i, k, fd, F[i, k])
    assert np.abs(F.sum(0)).max() < 1e-10 * max(1.0, np.abs(F).max())


def test_linear_network_is_a_pair_potential(nn):
    """With identity activations E = sum_{i<j} 2 u(r_ij) + const, u(r) = sum_k c_k exp(-eta (r-mu_k)^2) f_c(r),
    c = W1^T W2^T w3 / s: compare with a pair loop written from that formula."""
    spec = nn.NNSpec(act="linear")
    x, L = config(N=40, seed=9)
    P = params(nn, spec)
    E, _, F, _, _ = nn.energy_forces(x, L, P, spec)
    c = (P.W1.T @ (P.W2.T @ P.w3)) / P.s
    const = len(x) * (float(P.w3 @ (P.W2 @ (P.b1 - P.W1 @ (P.m / P.s)) + P.b2)) + P.b3)
    mu = 0.8 + np.arange(16) * 1.7 / 15
    eta = 1.0 / (2 * (1.7 / 15) ** 2)

    def u(r):
        return sum(c[k] * math.exp(-eta * (r - mu[k]) ** 2) for k in range(16)) * 0.5 * (math.cos(math.pi * r / 2.5) + 1)

    Lv = np.array(L)
    Epair, Fpair = 0.0, np.zeros_like(x)
    for i in range(len(x)):
        for j in range(i + 1, len(x)):
            d = x[i] - x[j]
            d -= Lv * np.rint(d / Lv)
            r = float(np.linalg.norm(d))
            if r < 2.5:
                Epair += 2 * u(r)
                h = 1e-6
                du = (u(r + h) - u(r - h)) / (2 * h)
                Fpair[i] -= 2 * du * d / r
                Fpair[j] += 2 * du * d / r
    assert math.isclose(E, Epair + const, rel_tol=1e-10, abs_tol=1e-9)
    assert np.abs(F - Fpair).max() < 1e-7 * max(1.0, np.abs(F).max())


def test_invariances(nn):
    spec = nn.NNSpec()
    x, L = config(N=50, seed=11)
    P = params(nn, spec)
    E0, _, F0, _, _ = nn.energy_forces(x, L, P, spec)
    E1, _, F1, _, _ = nn.energy_forces(np.mod(x + np.array([1.3, -2.1, 0.4]), L[0]), L, P, spec)
    assert math.isclose(E0, E1, rel_tol=1e-12)
    assert np.abs(F0 - F1).max() < 1e-9


def test_loss_gradients_match_fd(nn):
    """Energy + force loss gradients w.r.t. every weight group (the force term is a gradient of a gradient)."""
    spec = nn.NNSpec()
    P = params(nn, spec, seed=7)
    snaps = []
    for sd in (21, 22):
        x, L = config(N=30, rho=0.7, seed=sd)
        E, _, F, _, _ = nn.energy_forces(x, L, params(nn, spec, seed=99), spec)
        snaps.append((x, L, E + 0.3, F * 0.9 + 0.05))
    loss, g = nn.loss_and_grad(snaps, P, spec, lam_f=0.5)
    rng = np.random.default_rng(1)
    h = 1e-6
    for name in P.names():
        arr = np.atleast_1d(np.asarray(getattr(P, name), dtype=np.float64))
        flat = arr.reshape(-1)
        for q in rng.choice(flat.size, min(4, flat.size), replace=False):
            vals = []
            for sgn in (1, -1):
                Q = nn.NNParams(**{k: (np.array(getattr(P, k), dtype=np.float64, copy=True)
                                       if k not in ("b3",) else float(P.b3)) for k in P.names()}, m=P.m, s=P.s)
                if name == "b3":
                    Q.b3 = P.b3 + sgn * h
                else:
                    a = getattr(Q, name).reshape(-1)
                    a[q] += sgn * h
                vals.append(nn.loss_and_grad(snaps, Q, spec, lam_f=0.5)[0])
            fd = (vals[0] - vals[1]) / (2 * h)
            an = float(np.atleast_1d(g[name]).reshape(-1)[q])
            assert abs(fd - an) <= 1e-5 * max(abs(fd), 1e-3), (name, q, fd, an)


def test_pair_adjoint_is_transpose_of_force_map(nn):
    """At fixed positions F is linear in e; the pair adjoint must satisfy <lam, F(e)> = <ebar(lam), e> for any
    lam and e, and forces_from_e at e = dE_i/dG_i must equal the oracle's energy_forces forces."""
    spec = nn.NNSpec()
    x, L = config()
    rng = np.random.default_rng(11)
    e = rng.normal(size=(x.shape[0], spec.K))
    lam = rng.normal(size=(x.shape[0], 3))
    lhs = float(np.sum(lam * nn.forces_from_e(x, L, spec, e)))
    rhs = float(np.sum(nn.pair_adjoint(x, L, spec, lam) * e))
    assert math.isclose(lhs, rhs, rel_tol=1e-12, abs_tol=1e-12)
    P = params(nn, spec)
    _, _, F, ee, _ = nn.energy_forces(x, L, P, spec)
    assert np.allclose(nn.forces_from_e(x, L, spec, ee), F, rtol=1e-12, atol=1e-12)
