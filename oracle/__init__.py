"""FP64 CPU oracle for the short-range MD path.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the ``cpu_baseline`` leg of ``bench.py``; never by the product package.
It shares no code with the HIP path.  ``md_oracle.c`` holds the brute-force
definitions (see its header for the passage of the paper each one follows);
``nn_oracle.py`` holds the neural pair potential.  This module only marshals
numpy arrays into the C functions and builds ``liboracle.so`` with gcc.

Positions arrive as the same uint32 torus coordinates the GPU path uses
(x = u * L / 2**32); the oracle decodes them to float64 once and then works
with real coordinates and the textbook nearest-image formula
d = a - b - L * round((a - b) / L).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "md_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

TWO32 = 4294967296.0


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (IEEE double, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
             "-pthread", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Pot(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n_species", ctypes.c_int32),
                ("sigma", ctypes.c_double * 64), ("epsilon", ctypes.c_double * 64),
                ("alpha", ctypes.c_double), ("r_cut", ctypes.c_double), ("shift", ctypes.c_int32),
                ("coef", ctypes.c_double * 64)]


class _FireParams(ctypes.Structure):
    _fields_ = [("dt_start", ctypes.c_double), ("dt_max", ctypes.c_double), ("f_inc", ctypes.c_double),
                ("f_dec", ctypes.c_double), ("alpha_start", ctypes.c_double), ("f_alpha", ctypes.c_double),
                ("n_min", ctypes.c_int32)]


class _FireState(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("alpha", ctypes.c_double), ("n_pos", ctypes.c_int64),
                ("steps", ctypes.c_int64), ("converged", ctypes.c_int32)]


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        P = ctypes.c_void_p
        lib.orc_pair_rows.argtypes = [ctypes.c_int, P, ctypes.c_int64, P, P, P, P, ctypes.c_int64, P, P, P,
                                      ctypes.c_int]
        lib.orc_neighbors.argtypes = [ctypes.c_int, P, ctypes.c_int64, P, ctypes.c_float, P, ctypes.c_int64,
                                      ctypes.c_int32, P, P, ctypes.c_int]
        lib.orc_verlet.argtypes = [ctypes.c_int, P, ctypes.c_int64, P, P, P, P, P, ctypes.c_double,
                                   ctypes.c_int64, ctypes.c_int]
        lib.orc_fire.argtypes = [ctypes.c_int, P, ctypes.c_int64, P, P, P, P, P, P, P, ctypes.c_int64,
                                 ctypes.c_double, ctypes.c_int]
        lib.orc_param_grad.argtypes = [ctypes.c_int, P, ctypes.c_int64, P, P, P, P, P]
        for f in ("orc_pair_rows", "orc_neighbors", "orc_verlet", "orc_fire", "orc_param_grad"):
            getattr(lib, f).restype = ctypes.c_int
        _lib = lib
    return _lib


def default_threads() -> int:
    return max(1, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count() or 1)


@dataclass
class Potential:
    """Pair potential parameters (paper Sec. 3.3.2; species matrices as App. A)."""
    kind: str = "lj"                      # "lj", "soft_sphere", "morse" or "buckingham"
    sigma: np.ndarray = field(default_factory=lambda: np.ones((1, 1)))
    epsilon: np.ndarray = field(default_factory=lambda: np.ones((1, 1)))
    alpha: float = 2.0
    r_cut: float = 2.5
    shift: bool = True
    coef: np.ndarray | None = None        # Buckingham: dispersion coefficients C_ab (S x S)

    def _c(self) -> _Pot:
        s = np.atleast_2d(np.asarray(self.sigma, dtype=np.float64))
        e = np.atleast_2d(np.asarray(self.epsilon, dtype=np.float64))
        S = s.shape[0]
        p = _Pot()
        p.kind = {"lj": 0, "soft_sphere": 1, "morse": 2, "buckingham": 3}[self.kind]
        p.n_species = S
        c = np.zeros((S, S)) if self.coef is None else np.atleast_2d(np.asarray(self.coef, dtype=np.float64))
        for q in range(S * S):
            p.sigma[q] = float(s.reshape(-1)[q])
            p.epsilon[q] = float(e.reshape(-1)[q])
            p.coef[q] = float(c.reshape(-1)[q])
        p.alpha = float(self.alpha)
        p.r_cut = float(self.r_cut)
        p.shift = 1 if self.shift else 0
        return p


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a if shape is None else a.reshape(shape)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def decode(u: np.ndarray, L) -> np.ndarray:
    """Torus coordinates (uint32 [N][dim]) -> float64 positions x = u * L / 2^32."""
    u = np.asarray(u, dtype=np.uint32)
    L = np.asarray(L, dtype=np.float64)[: u.shape[1]]
    return u.astype(np.float64) * (L / TWO32)


def _species(species, N):
    if species is None:
        return None
    return np.ascontiguousarray(species, dtype=np.int32).reshape(N)


def pair_rows(x, L, pot: Potential, species=None, rows=None, nthreads=None):
    """F_i, e_i = 1/2 sum_j u(r_ij), w_i = 1/2 sum_j r_ij f(r_ij) for `rows` (default all), by brute force.

    ``x`` is float64 [N][dim] (use ``decode`` for torus coordinates).
    """
    lib = _load()
    x = _f64(x)
    N, dim = x.shape
    Lv = _f64(np.asarray(L, dtype=np.float64)[:dim])
    sp = _species(species, N)
    r = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    nr = N if r is None else r.shape[0]
    F = np.zeros((nr, dim))
    e = np.zeros(nr)
    w = np.zeros(nr)
    cp = pot._c()
    rc = lib.orc_pair_rows(dim, _ptr(Lv), N, _ptr(x), _ptr(sp), ctypes.byref(cp), _ptr(r), nr, _ptr(F), _ptr(e),
                           _ptr(w), nthreads or default_threads())
    assert rc == 0
    return F, e, w


def energy(x, L, pot: Potential, species=None, nthreads=None) -> float:
    """U = 1/2 sum_{i != j} u(r_ij) (paper Sec. 3.2.2), summed exactly rounded (math.fsum)."""
    _, e, _ = pair_rows(x, L, pot, species, nthreads=nthreads)
    return math.fsum(e.tolist())


def neighbors(u, L, r_list: float, rows=None, cap: int = 512, nthreads=None):
    """Brute-force neighbor set on the torus (definition in md_oracle.c): list of sorted int arrays."""
    lib = _load()
    u = np.ascontiguousarray(u, dtype=np.uint32)
    N, dim = u.shape
    Lv = _f64(np.asarray(L, dtype=np.float64)[:dim])
    r = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    nr = N if r is None else r.shape[0]
    count = np.zeros(nr, dtype=np.int32)
    idx = np.full((nr, cap), -1, dtype=np.int32)
    rc = lib.orc_neighbors(dim, _ptr(Lv), N, _ptr(u), ctypes.c_float(np.float32(r_list)), _ptr(r), nr, cap,
                           _ptr(count), _ptr(idx), nthreads or default_threads())
    assert rc == 0
    if count.max(initial=0) > cap:
        return neighbors(u, L, r_list, rows, int(count.max()) + 16, nthreads)
    return [idx[q, : count[q]].copy() for q in range(nr)]


def verlet(x, v, F, L, pot: Potential, dt: float, n_steps: int, species=None, nthreads=None):
    """n_steps of velocity Verlet in float64 (paper Sec. 3.3.1, m = 1).  Returns new (x, v, F)."""
    lib = _load()
    x = _f64(x).copy()
    v = _f64(v).copy()
    F = _f64(F).copy()
    N, dim = x.shape
    Lv = _f64(np.asarray(L, dtype=np.float64)[:dim])
    sp = _species(species, N)
    cp = pot._c()
    rc = lib.orc_verlet(dim, _ptr(Lv), N, _ptr(x), _ptr(v), _ptr(F), _ptr(sp), ctypes.byref(cp), dt, n_steps,
                        nthreads or default_threads())
    assert rc == 0
    return x, v, F


@dataclass
class FireParams:
    """FIRE parameters; Bitzek et al. (2006) published n_min, f_inc, f_dec, alpha_start, f_alpha."""
    dt_start: float = 0.1
    dt_max: float = 0.4
    n_min: int = 5
    f_inc: float = 1.1
    f_dec: float = 0.5
    alpha_start: float = 0.1
    f_alpha: float = 0.99


def fire(x, L, pot: Potential, species=None, params: FireParams | None = None, max_steps: int = 100000,
         f_tol: float = 1e-6, nthreads=None, v=None, state=None):
    """FIRE descent in float64 (paper Sec. 3.3.1 / App. A).  Returns dict with x, v, F, dt, alpha, steps, converged."""
    lib = _load()
    params = params or FireParams()
    x = _f64(x).copy()
    N, dim = x.shape
    Lv = _f64(np.asarray(L, dtype=np.float64)[:dim])
    sp = _species(species, N)
    F, _, _ = pair_rows(x, L, pot, species, nthreads=nthreads)
    v = np.zeros_like(x) if v is None else _f64(v).copy()
    cp = pot._c()
    fp = _FireParams(params.dt_start, params.dt_max, params.f_inc, params.f_dec, params.alpha_start,
                     params.f_alpha, params.n_min)
    st = _FireState(params.dt_start, params.alpha_start, 0, 0, 0)
    if state is not None:
        st.dt, st.alpha, st.n_pos, st.steps = state["dt"], state["alpha"], state["n_pos"], state["steps"]
    rc = lib.orc_fire(dim, _ptr(Lv), N, _ptr(x), _ptr(v), _ptr(F), _ptr(sp), ctypes.byref(cp), ctypes.byref(fp),
                      ctypes.byref(st), max_steps, f_tol, nthreads or default_threads())
    assert rc == 0
    return {"x": x, "v": v, "F": F, "dt": st.dt, "alpha": st.alpha, "n_pos": st.n_pos, "steps": st.steps,
            "converged": bool(st.converged)}


def param_grad(x, L, pot: Potential, species=None):
    """(G_sigma, G_eps): dU/dparam at fixed positions, per ordered species pair (see md_oracle.c)."""
    lib = _load()
    x = _f64(x)
    N, dim = x.shape
    Lv = _f64(np.asarray(L, dtype=np.float64)[:dim])
    sp = _species(species, N)
    S = np.atleast_2d(pot.sigma).shape[0]
    gs = np.zeros(S * S)
    ge = np.zeros(S * S)
    cp = pot._c()
    rc = lib.orc_param_grad(dim, _ptr(Lv), N, _ptr(x), _ptr(sp), ctypes.byref(cp), _ptr(gs), _ptr(ge))
    assert rc == 0
    return gs.reshape(S, S), ge.reshape(S, S)


def diameter_grad(x, L, diameters, epsilon, species, alpha: float = 2.0):
    """dU/dd_s for soft spheres with sigma_ab = (d_a + d_b)/2 (App. A mixing), at fixed positions."""
    d = np.asarray(diameters, dtype=np.float64)
    S = d.shape[0]
    sig = 0.5 * (d[:, None] + d[None, :])
    pot = Potential("soft_sphere", sig, np.broadcast_to(np.asarray(epsilon, dtype=np.float64), (S, S)).copy(),
                    alpha=alpha)
    gs, _ = param_grad(x, L, pot, species)
    g = np.zeros(S)
    for a in range(S):
        for b in range(S):
            g[a] += 0.5 * gs[a, b]
            g[b] += 0.5 * gs[a, b]
    return g


def rescaled_box_grad(u, L, D: float, species, epsilon: float = 1.0, alpha: float = 2.0):
    """(U, dU/dD) for the bidisperse disks of Sec. 4.2 / App. A: species 0 has diameter D and species 1 diameter 1
    (sigma_ab = (d_a + d_b)/2), and the square box edge follows the packing-fraction law L(D) ~ sqrt(D^2 + 1), so at
    fixed fractional positions s = u / 2^32 every distance scales with L.  The derivative at fixed s is the
    derivative in the diameters at fixed real positions plus the box term (dL/dD)/L * sum_pairs r du/dr, with
    (dL/dD)/L = D / (D^2 + 1).  L is the box edge at D (the caller's value)."""
    d = np.array([D, 1.0])
    x = decode(u, [L, L])
    sig = 0.5 * (d[:, None] + d[None, :])
    pot = Potential("soft_sphere", sig, np.full((2, 2), float(epsilon)), alpha=alpha)
    g = diameter_grad(x, [L, L], d, epsilon, species, alpha)
    _, e, w = pair_rows(x, [L, L], pot, species)
    U = math.fsum(e)
    W = math.fsum(w)   # sum over pairs of -r du/dr
    return U, float(g[0]) - D / (D * D + 1.0) * W

