"""Pins of the FP64 constant-temperature integrators and gradient descent (oracle/thermostats.py): the random
generator against numpy's Philox, limits that reduce to velocity Verlet or to each other, closed forms, and the
statistics (equipartition, diffusion, conserved quantity) the schemes are built to reproduce."""
import math

import numpy as np
import pytest

from paper_1912_04232_amd import inputs


@pytest.fixture(scope="module")
def th():
    from oracle import thermostats
    return thermostats


def soft(orc, d=(1.0, 1.4)):
    d = np.asarray(d, dtype=np.float64)
    return orc.Potential("soft_sphere", 0.5 * (d[:, None] + d[None, :]), np.ones((2, 2)), alpha=2.0)


def disks(N, phi, seed):
    L = inputs.box_for_packing([1.0, 1.4], [N // 2, N - N // 2], phi, 2)
    return inputs.uniform_torus(N, 2, seed).astype(np.float64) * (L / 2.0 ** 32), np.array([L, L]), \
        inputs.bidisperse_species(N)


def test_philox_matches_numpy(th):
    """numpy's Philox bit generator (4x64, 10 rounds) advances its counter before each block: block c of ours is
    its output after counter c - 1."""
    for key, ctr in (([7, 11], [5, 0, 0, 0]), ([2 ** 64 - 1, 3], [123456789, 42, 0, 0]), ([0, 0], [1, 0, 0, 0])):
        c = list(ctr)
        c0 = np.array([(c[0] - 1) % 2 ** 64] + c[1:], dtype=np.uint64)
        bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=c0)
        want = [int(w) for w in bg.random_raw(4)]
        assert th.philox4x64(c, key) == want


def test_normals_statistics(th):
    z = np.concatenate([th.normals(500, 3, 99, s) for s in range(40)])      # 60000 samples
    assert abs(z.mean()) < 0.02
    assert abs(z.var() - 1.0) < 0.03
    assert abs((z[:, 0] * z[:, 1]).mean()) < 0.02                           # components independent
    assert abs(np.mean(z ** 4) - 3.0) < 0.15                                 # Gaussian kurtosis
    a, b = th.normals(200, 2, 5, 0), th.normals(200, 2, 5, 1)
    assert abs((a * b).mean()) < 0.1                                         # steps independent


def test_baoab_without_friction_is_velocity_verlet(th, orc):
    x, L, sp = disks(64, 0.9, 1)
    pot = soft(orc)
    v = inputs.maxwell_velocities(64, 2, 0.5, 2).astype(np.float64)
    F, _, _ = orc.pair_rows(x, L, pot, sp)
    xa, va, Fa = th.langevin_baoab(x, v, F, L, pot, sp, 0.01, 0.0, 1.0, 3, 0, 20)
    xb, vb, Fb = orc.verlet(x, v, F, L, pot, 0.01, 20, sp)
    d = xa - xb
    d -= L * np.rint(d / L)
    assert np.abs(d).max() < 1e-12 and np.abs(va - vb).max() < 1e-12


def test_baoab_free_particles(th, orc):
    """No interactions (disks far apart): with kT = 0 the velocity decays by exp(-gamma dt) per step exactly;
    with kT > 0 the O step alone drives <v^2> per degree of freedom to kT."""
    N, L = 40, np.array([1000.0, 1000.0])
    x = inputs.uniform_torus(N, 2, 8).astype(np.float64) * (L / 2.0 ** 32)
    pot = soft(orc, (1e-3, 1e-3))
    v0 = inputs.maxwell_velocities(N, 2, 1.0, 9).astype(np.float64)
    F = np.zeros_like(x)
    _, v, _ = th.langevin_baoab(x, v0, F, L, pot, None, 0.05, 2.0, 0.0, 1, 0, 10)
    assert np.allclose(v, v0 * math.exp(-2.0 * 0.05 * 10), rtol=1e-13, atol=0)
    kT, vs = 0.7, []
    xx, vv = x, v0
    for k in range(30):
        xx, vv, _ = th.langevin_baoab(xx, vv, F, L, pot, None, 0.05, 5.0, kT, 1, 10 * k, 10)
        vs.append(vv.copy())
    t = np.mean(np.concatenate(vs) ** 2)
    assert abs(t - kT) < 0.05 * kT


def test_brownian_without_noise_is_gradient_descent(th, orc):
    x, L, sp = disks(64, 0.9, 11)
    pot = soft(orc)
    F, _, _ = orc.pair_rows(x, L, pot, sp)
    xa, Fa = th.brownian(x, F, L, pot, sp, 0.02, 2.0, 0.0, 5, 0, 7)
    xb, Fb, _ = th.gradient_descent(x, F, L, pot, sp, 0.01, 7)
    assert np.array_equal(xa, xb) and np.array_equal(Fa, Fb)


def test_gradient_descent_harmonic_contact_closed_form(th, orc):
    """Two disks of diameter 1 overlapping by delta: each step moves both apart by dt F with F = (1 - r), so the
    overlap shrinks by the factor 1 - 2 dt per step."""
    L = np.array([20.0, 20.0])
    x = np.array([[5.0, 5.0], [5.7, 5.0]])
    pot = soft(orc, (1.0, 1.0))
    F, _, _ = orc.pair_rows(x, L, pot, None)
    dt = 0.05
    for n in (1, 5, 20):
        xn, _, U = th.gradient_descent(x, F, L, pot, None, dt, n)
        r = abs(xn[1, 0] - xn[0, 0])
        assert math.isclose(1.0 - r, 0.3 * (1.0 - 2.0 * dt) ** n, rel_tol=1e-12)
        assert math.isclose(U, 0.5 * (1.0 - r) ** 2, rel_tol=1e-12)


def test_brownian_free_diffusion(th, orc):
    """Without interactions the mean-square displacement is 2 dim (kT / gamma) t."""
    N, L = 400, np.array([1e4, 1e4])
    x0 = inputs.uniform_torus(N, 2, 21).astype(np.float64) * (L / 2.0 ** 32)
    pot = soft(orc, (1e-3, 1e-3))
    dt, gamma, kT, n = 0.01, 2.0, 1.5, 50
    x, _ = th.brownian(x0, np.zeros_like(x0), L, pot, None, dt, gamma, kT, 4, 0, n)
    msd = float(((x - x0) ** 2).sum(1).mean())
    assert abs(msd / (2 * 2 * kT / gamma * dt * n) - 1.0) < 0.1


def test_nose_hoover_heavy_thermostat_is_verlet_and_chain_conserves(th, orc):
    x, L, sp = disks(48, 0.85, 31)
    pot = soft(orc)
    v = inputs.maxwell_velocities(48, 2, 0.3, 32).astype(np.float64)
    F, _, _ = orc.pair_rows(x, L, pot, sp)
    xa, va, _, _, _, _ = th.nose_hoover(x, v, F, L, pot, sp, 0.01, 1.0, [1e15], 30)
    xb, vb, _ = orc.verlet(x, v, F, L, pot, 0.01, 30, sp)
    d = xa - xb
    d -= L * np.rint(d / L)
    assert np.abs(d).max() < 1e-9 and np.abs(va - vb).max() < 1e-9
    # a chain of three thermostats: H' holds to O(dt^2) while K and U exchange energy with the bath, and the
    # mean kinetic temperature is kT
    Q = [1.0, 0.5, 0.5]
    _, _, _, _, _, H0 = th.nose_hoover(x, v, F, L, pot, sp, 0.005, 0.8, Q, 0)
    drift = []
    for dt in (0.005, 0.0025):
        xs, vs, Fs, p, eta = x, v, F, None, None
        Hs, Ks = [], []
        for k in range(20):
            xs, vs, Fs, p, eta, H = th.nose_hoover(xs, vs, Fs, L, pot, sp, dt, 0.8, Q, int(round(0.1 / dt)), p, eta)
            Hs.append(H)
            Ks.append(0.5 * (vs * vs).sum())
        drift.append(max(abs(h - H0) for h in Hs))
        assert max(Ks) - min(Ks) > 1.0                     # the bath does move energy
        assert abs(np.mean(Ks) / 48 - 0.8) < 0.05         # 2K / n_f, n_f = 96
    assert drift[0] < 1e-2
    assert 3.0 < drift[0] / drift[1] < 5.0                 # second order in dt
