"""Seeded synthetic inputs shared by the GPU path, the oracle and the benchmark.

This module only draws random numbers and lays out lattices: it holds none of
the method's arithmetic (no energies, forces, neighbor lists or integrators).
Positions are returned as uint32 torus coordinates (x = u * L / 2^32, see
include/md.h); boxes are float32 values so every consumer sees the same box.

Workloads (the paper benchmarks Lennard-Jones MD, Sec. 3.1; minimizes
bidisperse soft disks, Sec. 4.2 / App. A; fits a neural potential, Sec. 4.1):
  lj_small   3D LJ N=1000, rho 0.8, random insertion rejecting r < 0.8
  ss_fire    2D harmonic soft disks N=65536, 50:50 d=1.0/1.4, phi 0.90
  lj_large   3D LJ N=256000 = 4*40^3 FCC, rho 0.84
  ss_batch   64 soft-disk packings, N ~ U{256..4096}, phi ~ U[0.84, 0.92]
  lj_train   3D LJ N=4000, rho 0.84 (neural-potential training snapshots)
"""
from __future__ import annotations

import math

import numpy as np

TWO32 = 4294967296.0


def f32(v) -> float:
    """Round to the nearest float32 (boxes and scalars are float32 values)."""
    return float(np.float32(v))


def box_for_density(N: int, rho: float, dim: int = 3) -> float:
    return f32((N / rho) ** (1.0 / dim))


def box_for_packing(diameters, counts, phi: float, dim: int = 2) -> float:
    """Square/cubic edge at packing fraction phi for disks (dim 2) or spheres (dim 3)."""
    d = np.asarray(diameters, dtype=np.float64)
    n = np.asarray(counts, dtype=np.float64)
    if dim == 2:
        vol = float(np.sum(n * np.pi * d ** 2 / 4.0))
    else:
        vol = float(np.sum(n * np.pi * d ** 3 / 6.0))
    return f32((vol / phi) ** (1.0 / dim))


def to_torus(x: np.ndarray, L) -> np.ndarray:
    """float positions -> uint32 torus coordinates (nearest, wrapped)."""
    x = np.asarray(x, dtype=np.float64)
    L = np.asarray(L, dtype=np.float64)[: x.shape[1]]
    q = np.rint(x / L * TWO32).astype(np.int64)
    return (q & 0xFFFFFFFF).astype(np.uint32)


def uniform_torus(N: int, dim: int, seed: int) -> np.ndarray:
    """Uniform positions on the torus: independent uniform uint32 per coordinate."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(0, 2 ** 32, size=(N, dim), dtype=np.uint64).astype(np.uint32)


def jittered_grid_torus(counts, jitter: float, seed: int) -> np.ndarray:
    """A simple grid of counts[0] x counts[1] (x counts[2]) sites, each moved by a uniform offset of up to
    +-jitter of its grid spacing along every axis; the box edges may differ per axis."""
    rng = np.random.Generator(np.random.PCG64(seed))
    axes = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in counts], indexing="ij")
    frac = np.stack([a.ravel() for a in axes], axis=1)
    frac = (frac + 0.5 + rng.uniform(-jitter, jitter, size=frac.shape)) / np.asarray(counts, dtype=np.float64)
    return np.floor(np.mod(frac, 1.0) * 2.0 ** 32).astype(np.uint64).astype(np.uint32)


def fcc_torus(n_cells: int, L: float) -> np.ndarray:
    """FCC lattice with n_cells^3 cubic cells (4 sites each) filling a cube of edge L."""
    base = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]], dtype=np.float64)
    g = np.arange(n_cells, dtype=np.float64)
    cz, cy, cx = np.meshgrid(g, g, g, indexing="ij")
    cells = np.stack([cx.ravel(), cy.ravel(), cz.ravel()], axis=1)
    pts = (cells[:, None, :] + base[None, :, :] + 0.25).reshape(-1, 3) / n_cells
    return to_torus(pts * L, [L, L, L])


def jittered_torus(u: np.ndarray, L, amplitude: float, seed: int) -> np.ndarray:
    """Torus coordinates u moved by independent uniform offsets of up to +-amplitude (length units) per axis."""
    rng = np.random.Generator(np.random.PCG64(seed))
    L = np.asarray(L, dtype=np.float64)[: u.shape[1]]
    off = rng.uniform(-amplitude, amplitude, size=u.shape) / L * TWO32
    q = u.astype(np.int64) + np.rint(off).astype(np.int64)
    return (q & 0xFFFFFFFF).astype(np.uint32)


def triangular_torus(nx: int, ny: int, a: float):
    """2D triangular lattice nx x ny (ny even) with spacing a; returns (u, Lx, Ly)."""
    Lx = f32(nx * a)
    Ly = f32(ny * a * math.sqrt(3.0) / 2.0)
    j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    x = (i + 0.5 * (j % 2) + 0.25) * a
    y = (j + 0.25) * a * math.sqrt(3.0) / 2.0
    pts = np.stack([x.ravel(), y.ravel()], axis=1)
    return to_torus(pts, [Lx, Ly]), Lx, Ly


def random_insertion_torus(N: int, L: float, dim: int, r_min: float, seed: int, max_tries: int = 10_000_000):
    """Random sequential insertion on the torus, rejecting a trial closer than r_min to any placed point.

    Uses a grid of buckets of edge >= r_min so each trial checks 3^dim buckets.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    nb = max(1, int(L / r_min))
    while nb > 1 and L / nb < r_min:
        nb -= 1
    buckets: dict = {}
    pts = np.zeros((N, dim), dtype=np.float64)
    r2min = r_min * r_min
    n = 0
    tries = 0
    offs = np.array(np.meshgrid(*([[-1, 0, 1]] * dim), indexing="ij")).reshape(dim, -1).T
    while n < N:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("random insertion did not finish")
        p = rng.random(dim) * L
        b = tuple(int(c) % nb for c in (p / L * nb))
        ok = True
        for o in offs:
            key = tuple((b[k] + int(o[k])) % nb for k in range(dim))
            for q in buckets.get(key, ()):
                d = p - pts[q]
                d -= L * np.rint(d / L)
                if float(d @ d) < r2min:
                    ok = False
                    break
            if not ok:
                break
        if ok:
            pts[n] = p
            buckets.setdefault(b, []).append(n)
            n += 1
    return to_torus(pts, [L] * dim)


def boids(N: int, L: float, seed: int, n_obstacles: int = 0, D_lo: float = 2.0, D_hi: float = 6.0):
    """Flocking start: uniform positions on the 2D torus (uint32), headings uniform in [-pi, pi) (float32 values),
    and n_obstacles disks (C_x, C_y, D) with centers uniform in [0, L) and radii uniform in [D_lo, D_hi), all
    float32-representable so that every consumer sees the same numbers."""
    u = uniform_torus(N, 2, seed)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    theta = rng.uniform(-np.pi, np.pi, N).astype(np.float32)
    obs = np.stack([rng.uniform(0.0, L, n_obstacles), rng.uniform(0.0, L, n_obstacles),
                    rng.uniform(D_lo, D_hi, n_obstacles)], 1).astype(np.float32).reshape(-1, 3)
    return u, theta, obs


def maxwell_velocities(N: int, dim: int, T: float, seed: int) -> np.ndarray:
    """Gaussian velocities (unit mass), net momentum removed, rescaled so sum v^2 = dim (N-1) T."""
    rng = np.random.Generator(np.random.PCG64(seed))
    v = rng.normal(0.0, math.sqrt(T), size=(N, dim))
    v -= v.mean(axis=0, keepdims=True)
    s = float(np.sum(v * v))
    if s > 0:
        v *= math.sqrt(dim * (N - 1) * T / s)
    return v.astype(np.float32)


# ----------------------------------------------------------------- workloads

def lj_small(seed: int = 1001):
    """3D LJ N=1000 at rho 0.8: insertion rejecting r < 0.8, Maxwell T=1 (seed+1), rc 2.5, skin 0.3, dt 0.005."""
    N, rho = 1000, 0.8
    L = box_for_density(N, rho)
    u = random_insertion_torus(N, L, 3, 0.8, seed)
    v = maxwell_velocities(N, 3, 1.0, seed + 1)
    return dict(name="lj_small", N=N, dim=3, L=[L, L, L], u=u, v=v, species=np.zeros(N, np.int32),
                kind="lj", sigma=[[1.0]], epsilon=[[1.0]], r_cut=2.5, skin=0.3, dt=0.005, steps=100)


def lj_large(n_cells: int = 40, seed: int = 3001, rho: float = 0.84):
    """3D LJ FCC 4*n_cells^3 at rho 0.84 (N=256000 for 40), Maxwell T=1, rc 2.5, skin 0.3, dt 0.005."""
    N = 4 * n_cells ** 3
    L = box_for_density(N, rho)
    u = fcc_torus(n_cells, L)
    v = maxwell_velocities(N, 3, 1.0, seed)
    return dict(name="lj_large", N=N, dim=3, L=[L, L, L], u=u, v=v, species=np.zeros(N, np.int32),
                kind="lj", sigma=[[1.0]], epsilon=[[1.0]], r_cut=2.5, skin=0.3, dt=0.005, steps=10000)


def bidisperse_species(N: int) -> np.ndarray:
    """First half species 0, second half species 1 (the App. A layout)."""
    return np.array([0] * (N // 2) + [1] * (N - N // 2), dtype=np.int32)


def ss_fire(N: int = 65536, phi: float = 0.90, seed: int = 2001, d_small: float = 1.0, d_large: float = 1.4):
    """2D harmonic soft disks, 50:50 diameters d_small/d_large, uniform positions (overlaps allowed)."""
    L = box_for_packing([d_small, d_large], [N // 2, N - N // 2], phi, 2)
    u = uniform_torus(N, 2, seed)
    d = np.array([d_small, d_large])
    sigma = 0.5 * (d[:, None] + d[None, :])
    return dict(name="ss_fire", N=N, dim=2, L=[L, L, 0.0], u=u, species=bidisperse_species(N), kind="soft_sphere",
                sigma=sigma.tolist(), epsilon=[[1.0, 1.0], [1.0, 1.0]], alpha=2.0, skin=0.3, diameters=[d_small,
                                                                                                       d_large])


def ss_batch(B: int = 64, seed: int = 4001, n_lo: int = 256, n_hi: int = 4096, phi_lo: float = 0.84,
             phi_hi: float = 0.92):
    """B soft-disk packings: N_b ~ U{n_lo..n_hi} (even), phi_b ~ U[phi_lo, phi_hi], d 1.0/1.4, positions uniform."""
    rng = np.random.Generator(np.random.PCG64(seed))
    reps = []
    for b in range(B):
        N = int(rng.integers(n_lo // 2, n_hi // 2 + 1)) * 2
        phi = float(rng.uniform(phi_lo, phi_hi))
        L = box_for_packing([1.0, 1.4], [N // 2, N // 2], phi, 2)
        frac = rng.integers(0, 2 ** 32, size=(N, 2), dtype=np.uint64).astype(np.uint32)
        reps.append(dict(N=N, phi=phi, L=[L, L, 0.0], u=frac, species=bidisperse_species(N)))
    return reps


def rescaled_box_starts(count: int = 100, N: int = 128, seed: int = 7001):
    """Random starts for the small-disk-diameter sweep (Sec. 4.2, App. A): `count` configurations of N disks,
    fractional positions uniform in the unit square (as uint32 torus coordinates, so one start serves every box)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return [rng.integers(0, 2 ** 32, size=(N, 2), dtype=np.uint64).astype(np.uint32) for _ in range(count)]


def lj_train_box(N: int = 4000, rho: float = 0.84) -> float:
    return box_for_density(N, rho)


def bcc_torus(n_cells: int, L: float) -> np.ndarray:
    """BCC lattice with n_cells^3 cubic cells (2 sites each) filling a cube of edge L."""
    base = np.array([[0, 0, 0], [0.5, 0.5, 0.5]], dtype=np.float64)
    g = np.arange(n_cells, dtype=np.float64)
    cz, cy, cx = np.meshgrid(g, g, g, indexing="ij")
    cells = np.stack([cx.ravel(), cy.ravel(), cz.ravel()], axis=1)
    pts = (cells[:, None, :] + base[None, :, :] + 0.25).reshape(-1, 3) / n_cells
    return to_torus(pts * L, [L, L, L])


def lj_train_runs(n_runs: int = 20, n_cells: int = 10, rho: float = 0.84, T_lo: float = 0.5, T_hi: float = 1.5,
                  seed: int = 5001):
    """Independent 3D LJ runs that supply neural-potential training snapshots: N = 4 n_cells^3 (4000) on an FCC
    lattice at rho with Maxwell velocities at T_k, T evenly spaced over [T_lo, T_hi] (the runs melt or stay
    crystalline according to T)."""
    N = 4 * n_cells ** 3
    L = box_for_density(N, rho)
    u = fcc_torus(n_cells, L)
    runs = []
    for k in range(n_runs):
        T = T_lo + (T_hi - T_lo) * k / max(n_runs - 1, 1)
        runs.append(dict(N=N, L=[L, L, L], T=T, u=u.copy(), v=maxwell_velocities(N, 3, T, seed + k)))
    return runs


def lj_nn_deploy(seed: int = 6001, rho: float = 0.84, T: float = 1.0):
    """3D LJ N = 65536 (BCC 32^3) at rho 0.84 with Maxwell velocities at T: the neural-potential MD workload."""
    n = 32
    N = 2 * n ** 3
    L = box_for_density(N, rho)
    return dict(N=N, L=[L, L, L], u=bcc_torus(n, L), v=maxwell_velocities(N, 3, T, seed), dt=0.005, skin=0.3)


def nn_init(seed: int, K: int = 16, H: int = 64) -> dict:
    """Glorot-uniform weights, zero biases, output layer scaled by 0.1 (float64)."""
    rng = np.random.Generator(np.random.PCG64(seed))

    def glorot(o, i):
        lim = math.sqrt(6.0 / (o + i))
        return rng.uniform(-lim, lim, size=(o, i))

    return dict(W1=glorot(H, K), b1=np.zeros(H), W2=glorot(H, H), b2=np.zeros(H), w3=glorot(1, H)[0] * 0.1, b3=0.0)
