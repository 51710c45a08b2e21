"""Python binding of libmdcore.so (include/md.h): argument marshalling only.

Every array is a torch tensor on the GPU; its ``data_ptr()`` and the current
torch stream are handed to the C ABI.  All arithmetic of the path runs in the
HIP kernels behind these calls.  If the library is missing, or there is no GPU,
the first call raises: there is no fallback.

The functions keep the C names (``nl_build``, ``pair_energy_force``,
``verlet_step``, ``fire_init``, ``fire_step``, ...).  On top of them sit small
init/update helpers in the style of the paper's ``simulate.nve`` and
``minimize.fire_descent`` (Sec. 3.3.1).
"""
from __future__ import annotations

import ctypes
import time
import os
import re
from dataclasses import dataclass

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmdcore.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "md.h")

MD_LJ, MD_SOFT_SPHERE, MD_MORSE, MD_BUCKINGHAM = 0, 1, 2, 3
WRT_SIGMA, WRT_EPSILON, WRT_DIAMETER, WRT_EPSILON_COMMON = 0, 1, 2, 3
BOX_FIXED, BOX_PACKING = 0, 1
FLAG_OVERFLOW, FLAG_MAXCOUNT, FLAG_NONFINITE, FLAG_REBUILDS = 0, 1, 2, 3
FLAG_CELL_OVERFLOW, FLAG_STALE, FLAG_MAXCELL, FLAG_STEPS, NFLAGS = 4, 5, 6, 7, 8

STATUS = {0: "MD_OK", -1: "MD_ERR_ARG", -2: "MD_ERR_BOX", -3: "MD_ERR_CAPACITY", -4: "MD_ERR_HIP",
          -5: "MD_ERR_NOT_CONVERGED", -6: "MD_ERR_NONFINITE"}


class MDError(RuntimeError):
    def __init__(self, fn, code):
        super().__init__(f"{fn} returned {STATUS.get(code, code)}")
        self.code = code


class c_box(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("L", ctypes.c_float * 3)]


class c_potential(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n_species", ctypes.c_int32), ("sigma", ctypes.c_double * 64),
                ("epsilon", ctypes.c_double * 64), ("alpha", ctypes.c_float), ("r_cut", ctypes.c_float),
                ("shift", ctypes.c_int32), ("reserved", ctypes.c_int32), ("coef", ctypes.c_double * 64)]


class c_nlist(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("capacity", ctypes.c_int32), ("lanes", ctypes.c_int32),
                ("segment", ctypes.c_int32), ("r_list", ctypes.c_float), ("skin", ctypes.c_float),
                ("idx", ctypes.c_void_p), ("count", ctypes.c_void_p), ("pos_ref", ctypes.c_void_p),
                ("flags", ctypes.c_void_p)]


class c_fire_params(ctypes.Structure):
    _fields_ = [("dt_start", ctypes.c_float), ("dt_max", ctypes.c_float), ("f_inc", ctypes.c_float),
                ("f_dec", ctypes.c_float), ("alpha_start", ctypes.c_float), ("f_alpha", ctypes.c_float),
                ("n_min", ctypes.c_int32), ("sync_rebuild", ctypes.c_int32)]


class c_fire_state(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("alpha", ctypes.c_double), ("fmax", ctypes.c_double),
                ("power", ctypes.c_double), ("mix_v", ctypes.c_double), ("mix_f", ctypes.c_double),
                ("steps", ctypes.c_int64), ("n_pos", ctypes.c_int32), ("converged", ctypes.c_int32)]


class c_nhc_state(ctypes.Structure):
    _fields_ = [("p", ctypes.c_double * 8), ("eta", ctypes.c_double * 8), ("Q", ctypes.c_double * 8),
                ("kT", ctypes.c_double), ("scale", ctypes.c_double), ("M", ctypes.c_int32), ("n_dof", ctypes.c_int32)]


class c_batch_config(ctypes.Structure):
    _fields_ = [("threads", ctypes.c_int32), ("cell_factor", ctypes.c_float)]


class c_batch(ctypes.Structure):
    _fields_ = [("B", ctypes.c_int32), ("dim", ctypes.c_int32), ("max_n", ctypes.c_int32),
                ("max_cells", ctypes.c_int32), ("offset", ctypes.c_void_p), ("box", ctypes.c_void_p),
                ("pos", ctypes.c_void_p), ("species", ctypes.c_void_p)]


class c_nn_params(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int32), ("H", ctypes.c_int32), ("mu0", ctypes.c_float), ("mu1", ctypes.c_float),
                ("r_c", ctypes.c_float), ("eta", ctypes.c_float), ("W1", ctypes.c_void_p),
                ("W2", ctypes.c_void_p), ("b1", ctypes.c_void_p), ("b2", ctypes.c_void_p), ("w3", ctypes.c_void_p),
                ("b3", ctypes.c_void_p), ("m", ctypes.c_void_p), ("s", ctypes.c_void_p)]


class c_flock_params(ctypes.Structure):
    _fields_ = [("J_align", ctypes.c_float), ("R_align", ctypes.c_float), ("J_avoid", ctypes.c_float),
                ("R_avoid", ctypes.c_float), ("J_coh", ctypes.c_float), ("R_coh", ctypes.c_float),
                ("J_obs", ctypes.c_float), ("alpha", ctypes.c_float), ("v", ctypes.c_float), ("dt", ctypes.c_float),
                ("n_obstacles", ctypes.c_int32), ("reserved", ctypes.c_int32), ("obstacles", ctypes.c_float * 48)]


class c_flock_predators(ctypes.Structure):
    _fields_ = [("P", ctypes.c_int32), ("J_flee", ctypes.c_float), ("R_flee", ctypes.c_float),
                ("J_chase", ctypes.c_float), ("R_chase", ctypes.c_float), ("v", ctypes.c_float),
                ("pos", ctypes.c_void_p), ("theta", ctypes.c_void_p)]


FIRE_STATE_BYTES = ctypes.sizeof(c_fire_state)
_lib = None

P = ctypes.c_void_p
_SIGNATURES = {
    "md_ctx_create": [ctypes.c_int, ctypes.POINTER(P)],
    "md_ctx_destroy": [P],
    "md_ctx_reserve": [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                       ctypes.c_int32],
    "md_cell_count": [ctypes.POINTER(c_box), ctypes.c_float],
    "md_positions_from_float": [ctypes.POINTER(c_box), P, P, ctypes.c_int32, P],
    "md_positions_to_float": [ctypes.POINTER(c_box), P, P, ctypes.c_int32, P],
    "nl_build": [P, ctypes.POINTER(c_box), P, ctypes.c_int32, ctypes.POINTER(c_nlist), P],
    "pair_energy_force": [P, ctypes.POINTER(c_box), ctypes.POINTER(c_potential), P, P, ctypes.c_int32,
                          ctypes.POINTER(c_nlist), P, P, P, P],
    "verlet_step": [P, ctypes.POINTER(c_box), ctypes.POINTER(c_potential), P, P, P, P, ctypes.c_int32,
                    ctypes.POINTER(c_nlist), ctypes.c_float, ctypes.c_int32, P],
    "langevin_run": [P, ctypes.POINTER(c_box), ctypes.POINTER(c_potential), P, P, P, P, ctypes.c_int32,
                     ctypes.POINTER(c_nlist), ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_uint64, P,
                     ctypes.c_int32, P],
    "fire_init": [P, ctypes.POINTER(c_box), ctypes.POINTER(c_potential), P, P, P, P, ctypes.c_int32,
                  ctypes.POINTER(c_nlist), ctypes.POINTER(c_fire_params), P, ctypes.c_double, P],
    "fire_step": [P, ctypes.POINTER(c_box), ctypes.POINTER(c_potential), P, P, P, P, ctypes.c_int32,
                  ctypes.POINTER(c_nlist), ctypes.POINTER(c_fire_params), P, ctypes.c_int32, ctypes.c_double, P],
    "fire_batched": [P, ctypes.POINTER(c_batch), ctypes.POINTER(c_potential), ctypes.POINTER(c_fire_params),
                     ctypes.POINTER(c_batch_config), ctypes.c_int32, ctypes.c_double, P, P, P, P, P],
    "envelope_grad": [P, ctypes.POINTER(c_batch), ctypes.POINTER(c_potential), P, P, P, P, P],
    "envelope_grad_wrt": [P, ctypes.POINTER(c_batch), ctypes.POINTER(c_potential), ctypes.c_int32, ctypes.c_int32, P,
                          P, P, P, P],
    "md_diameter_grad": [P, ctypes.POINTER(c_batch), ctypes.POINTER(c_potential), P, P, P, ctypes.c_int32, P, P, P],
    "nn_descriptor_stats": [P, P, ctypes.c_int32, P, P, P],
    "fire_unrolled_workspace_bytes": [ctypes.c_int32, ctypes.c_int64, ctypes.c_int32],
    "fire_unrolled_grad": [P, ctypes.POINTER(c_batch), ctypes.POINTER(c_potential), P, ctypes.POINTER(c_fire_params),
                           ctypes.c_int32, P, ctypes.c_uint64, P, P, P, P, P, P, P, P],
    "nn_descriptors": [P, ctypes.POINTER(c_box), ctypes.POINTER(c_nn_params), P, ctypes.c_int32,
                       ctypes.POINTER(c_nlist), P, P],
    "nn_mlp": [P, ctypes.POINTER(c_nn_params), P, ctypes.c_int32, P, P, P],
    "nn_forces": [P, ctypes.POINTER(c_box), ctypes.POINTER(c_nn_params), P, ctypes.c_int32, ctypes.POINTER(c_nlist),
                  P, P, P],
    "nn_param_count": [],
    "nn_loss": [P, P, P, P, P, ctypes.c_int32, ctypes.c_int32, ctypes.c_float, P, P, P, P],
    "nn_pair_adjoint": [P, ctypes.POINTER(c_box), ctypes.POINTER(c_nn_params), P, ctypes.c_int32,
                        ctypes.POINTER(c_nlist), P, P, P],
    "nn_mlp_grad": [P, ctypes.POINTER(c_nn_params), P, ctypes.c_int32, ctypes.c_int32, P, P, P, P],
    "nn_adam": [P, P, P, P, P, ctypes.c_int32, ctypes.c_int32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                ctypes.c_float, P, P, P],
    "nn_cast_weights": [P, P, P, P, P],
    "md_sum": [P, P, ctypes.c_int64, P, P],
    "md_kinetic_energy": [P, P, ctypes.c_int32, ctypes.c_int32, P, P],
    "md_kinetic_energy_noalloc": [P, ctypes.c_int32, ctypes.c_int32, P, P],
    "md_rescale_velocities": [P, P, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, P],
    "md_kick_drift": [P, ctypes.POINTER(c_box), P, P, P, ctypes.c_int32, ctypes.POINTER(c_nlist), ctypes.c_float, P],
    "nl_update": [P, ctypes.POINTER(c_box), P, ctypes.c_int32, ctypes.POINTER(c_nlist), P],
    "md_kick": [P, P, P, ctypes.c_int32, ctypes.c_int32, ctypes.c_float, P],
    "md_langevin_baoa": [P, ctypes.POINTER(c_box), P, P, P, ctypes.c_int32, ctypes.POINTER(c_nlist), ctypes.c_float,
                         ctypes.c_float, ctypes.c_float, ctypes.c_uint64, P, P],
    "md_brownian_step": [P, ctypes.POINTER(c_box), P, P, ctypes.c_int32, ctypes.POINTER(c_nlist), ctypes.c_float,
                         ctypes.c_float, ctypes.c_float, ctypes.c_uint64, P, P],
    "md_gradient_step": [P, ctypes.POINTER(c_box), P, P, ctypes.c_int32, ctypes.POINTER(c_nlist), ctypes.c_float, P],
    "md_nhc_half": [P, P, ctypes.c_int32, ctypes.c_int32, P, ctypes.c_double, P],
    "nl_half": [P, ctypes.POINTER(c_nlist), P, P, ctypes.c_int32, P, P],
    "flock_step": [P, ctypes.POINTER(c_box), P, P, ctypes.c_int32, ctypes.POINTER(c_nlist),
                   ctypes.POINTER(c_flock_params), ctypes.POINTER(c_flock_predators), P, P],
    "pair_force_half": [P, ctypes.POINTER(c_box), ctypes.POINTER(c_potential), P, P, ctypes.c_int32, P, P,
                        ctypes.c_int32, P, P],
    "md_rms_diff": [P, P, P, ctypes.c_int64, P, P],
    "md_copy_words": [P, P, P, ctypes.c_int64, P],
    "md_min_distance": [P, ctypes.POINTER(c_box), P, ctypes.c_int32, ctypes.POINTER(c_nlist), P, P],
    "md_flags_read": [ctypes.POINTER(c_nlist), P, P],
    "md_flags_clear": [ctypes.POINTER(c_nlist), P],
    "md_version": [],
}


_RESTYPES = {"md_version": ctypes.c_char_p, "fire_unrolled_workspace_bytes": ctypes.c_uint64}


def header_functions(path: str = HEADER):
    """Names of the functions declared in include/md.h."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:md_status|int32_t|uint64_t|const char \*)\s*\**\s*([a-z_0-9]+)\s*\(", text,
                                 flags=re.M)))


def load(path: str = LIB_PATH):
    """Load libmdcore.so and attach the C signatures.  Raises if the library is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"{path} not built: run `python -m paper_1912_04232_amd.build`")
        lib = ctypes.CDLL(path)
        for name, args in _SIGNATURES.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = _RESTYPES.get(name, ctypes.c_int)
        _lib = lib
    return _lib


def _check(fn, code):
    if code != 0:
        raise MDError(fn, code)


def _ptr(t):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev():
    if not torch.cuda.is_available():
        raise RuntimeError("the MD library needs a GPU; none is visible")
    return torch.device("cuda", torch.cuda.current_device())


# ------------------------------------------------------------------ value types

@dataclass
class Box:
    """Periodic orthorhombic box [0, L) (paper Sec. 3.2.1)."""
    L: tuple
    dim: int = 3

    def c(self) -> c_box:
        b = c_box()
        b.dim = self.dim
        for k in range(3):
            b.L[k] = float(self.L[k]) if k < len(self.L) else 0.0
        return b


@dataclass
class Potential:
    """Pair potential (paper Sec. 3.3.2): kind 'lj', 'soft_sphere', 'morse' or 'buckingham', S x S sigma / epsilon
    (Morse: sigma is the minimum position, epsilon the well depth, alpha the range; Buckingham: epsilon the
    repulsion strength A, sigma its range rho, coef the dispersion coefficient C)."""
    kind: str = "lj"
    sigma: object = ((1.0,),)
    epsilon: object = ((1.0,),)
    alpha: float = 2.0
    r_cut: float = 2.5
    shift: bool = True
    coef: object = None

    @property
    def n_species(self) -> int:
        return int(np.atleast_2d(np.asarray(self.sigma)).shape[0])

    def cutoff(self) -> float:
        if self.kind in ("lj", "morse", "buckingham"):
            return float(self.r_cut)
        return float(np.max(np.asarray(self.sigma, dtype=np.float64)))

    def c(self) -> c_potential:
        s = np.atleast_2d(np.asarray(self.sigma, dtype=np.float64))
        e = np.atleast_2d(np.asarray(self.epsilon, dtype=np.float64))
        S = s.shape[0]
        if e.shape != (S, S) or S > 8:
            raise ValueError("sigma / epsilon must be S x S with S <= 8")
        p = c_potential()
        p.kind = {"lj": MD_LJ, "soft_sphere": MD_SOFT_SPHERE, "morse": MD_MORSE,
                  "buckingham": MD_BUCKINGHAM}[self.kind]
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


@dataclass
class FireParams:
    """FIRE parameters; n_min, f_inc, f_dec, alpha_start, f_alpha are Bitzek et al.'s published values."""
    dt_start: float = 0.1
    dt_max: float = 0.4
    n_min: int = 5
    f_inc: float = 1.1
    f_dec: float = 0.5
    alpha_start: float = 0.1
    f_alpha: float = 0.99

    def c(self, sync_rebuild: bool = False) -> c_fire_params:
        return c_fire_params(self.dt_start, self.dt_max, self.f_inc, self.f_dec, self.alpha_start, self.f_alpha,
                             self.n_min, int(sync_rebuild))


class Context:
    """md_ctx: owns the library's scratch on one device."""

    def __init__(self, device: int | None = None):
        lib = load()
        dev = _dev() if device is None else torch.device("cuda", device)
        self.device = dev
        h = ctypes.c_void_p()
        _check("md_ctx_create", lib.md_ctx_create(dev.index, ctypes.byref(h)))
        self.h = h
        self.N = self.dim = self.C = self.cap = self.W = self.M = 0

    def reserve(self, N: int, dim: int, max_cells: int = 1, capacity: int = 1, lanes: int = 1,
                max_per_cell: int = 1):
        if (N > self.N or dim > self.dim or max_cells > self.C or capacity > self.cap or lanes > self.W
                or max_per_cell > self.M):
            self.N, self.dim, self.C = max(N, self.N), max(dim, self.dim), max(max_cells, self.C)
            self.cap, self.W, self.M = max(capacity, self.cap), max(lanes, self.W), max(max_per_cell, self.M)
            _check("md_ctx_reserve", load().md_ctx_reserve(self.h, self.N, self.dim, self.C, self.cap, self.W,
                                                           self.M))

    def close(self):
        if self.h:
            load().md_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cell_count(box: Box, r_list: float) -> int:
    b = box.c()
    return int(load().md_cell_count(ctypes.byref(b), ctypes.c_float(r_list)))


class NeighborList:
    """md_nlist with its arrays held as torch tensors: idx[capacity/W][N][W], count[N][W], pos_ref[N][dim], flags.

    ``lanes`` (W) is the number of GPU lanes per particle; ``max_per_cell`` is the bin size the context
    reserves for this list's cell list."""

    def __init__(self, N: int, dim: int, capacity: int, r_list: float, skin: float, device=None,
                 max_per_cell: int = 64, lanes: int = 1, segment: int = 0):
        dev = device or _dev()
        capacity = (capacity + lanes - 1) // lanes * lanes
        if segment < 0 or (segment > 0 and N % segment != 0):
            raise ValueError("segment must divide N")
        self.N, self.dim, self.capacity, self.max_per_cell, self.lanes = N, dim, capacity, max_per_cell, lanes
        self.segment = segment
        self.r_list, self.skin = float(np.float32(r_list)), float(np.float32(skin))
        self.idx = torch.empty((capacity // lanes, max(N, 1), lanes), dtype=torch.int32, device=dev)
        self.count = torch.zeros((max(N, 1), lanes), dtype=torch.int32, device=dev)
        self.pos_ref = torch.zeros((max(N, 1), dim), dtype=torch.int32, device=dev)
        self.flags = torch.zeros(NFLAGS, dtype=torch.int32, device=dev)

    def c(self) -> c_nlist:
        n = c_nlist()
        n.N, n.capacity, n.lanes, n.r_list, n.skin = self.N, self.capacity, self.lanes, self.r_list, self.skin
        n.segment = self.segment
        n.idx, n.count = self.idx.data_ptr(), self.count.data_ptr()
        n.pos_ref, n.flags = self.pos_ref.data_ptr(), self.flags.data_ptr()
        return n

    def read_flags(self) -> np.ndarray:
        out = (ctypes.c_int32 * NFLAGS)()
        n = self.c()
        _check("md_flags_read", load().md_flags_read(ctypes.byref(n), out, _stream()))
        return np.array(out[:], dtype=np.int32)

    def clear_flags(self):
        n = self.c()
        _check("md_flags_clear", load().md_flags_clear(ctypes.byref(n), _stream()))

    def rows(self) -> list:
        """Host copy of the rows (list of int arrays, sub-rows concatenated), for inspection and tests."""
        idx = self.idx.cpu().numpy()
        cnt = np.minimum(self.count.cpu().numpy(), self.capacity // self.lanes)
        return [np.concatenate([idx[: cnt[i, l], i, l] for l in range(self.lanes)]) for i in range(self.N)]

    def lengths(self) -> np.ndarray:
        return self.count.cpu().numpy()[: self.N].sum(axis=1)


# ------------------------------------------------------------ C entry points

def positions_from_float(box: Box, x: torch.Tensor) -> torch.Tensor:
    x = x.contiguous()
    u = torch.empty(x.shape, dtype=torch.int32, device=x.device)
    b = box.c()
    _check("md_positions_from_float",
           load().md_positions_from_float(ctypes.byref(b), _ptr(x), _ptr(u), x.shape[0], _stream()))
    return u


def positions_to_float(box: Box, u: torch.Tensor) -> torch.Tensor:
    x = torch.empty(u.shape, dtype=torch.float32, device=u.device)
    b = box.c()
    _check("md_positions_to_float",
           load().md_positions_to_float(ctypes.byref(b), _ptr(u), _ptr(x), u.shape[0], _stream()))
    return x


def _reserve_for(ctx: Context, box: Box, N: int, nl: NeighborList):
    systems = N // nl.segment if nl.segment else 1
    ctx.reserve(N, box.dim, max(1, cell_count(box, nl.r_list)) * systems, nl.capacity, nl.lanes, nl.max_per_cell)


def nl_build(ctx: Context, box: Box, pos: torch.Tensor, nl: NeighborList):
    N = pos.shape[0]
    _reserve_for(ctx, box, N, nl)
    b, n = box.c(), nl.c()
    _check("nl_build", load().nl_build(ctx.h, ctypes.byref(b), _ptr(pos), N, ctypes.byref(n), _stream()))


def pair_energy_force(ctx: Context, box: Box, pot: Potential, pos: torch.Tensor, species=None,
                      nl: NeighborList | None = None, force=None, energy=None, virial=None):
    N = pos.shape[0]
    ctx.reserve(N, box.dim, 1)
    b, p = box.c(), pot.c()
    n = nl.c() if nl is not None else None
    _check("pair_energy_force", load().pair_energy_force(
        ctx.h, ctypes.byref(b), ctypes.byref(p), _ptr(pos), _ptr(species), N,
        ctypes.byref(n) if n is not None else None, _ptr(force), _ptr(energy), _ptr(virial), _stream()))


def kick_drift(ctx: Context, box: Box, pos, vel, force, nl: NeighborList, dt: float):
    b, n = box.c(), nl.c()
    _check("md_kick_drift", load().md_kick_drift(ctx.h, ctypes.byref(b), _ptr(pos), _ptr(vel), _ptr(force),
                                                 pos.shape[0], ctypes.byref(n), ctypes.c_float(dt), _stream()))


def nl_update(ctx: Context, box: Box, pos, nl: NeighborList):
    N = pos.shape[0]
    _reserve_for(ctx, box, N, nl)
    b, n = box.c(), nl.c()
    _check("nl_update", load().nl_update(ctx.h, ctypes.byref(b), _ptr(pos), N, ctypes.byref(n), _stream()))


def kick(ctx: Context, vel, force, h: float):
    N, dim = vel.shape
    _check("md_kick", load().md_kick(ctx.h, _ptr(vel), _ptr(force), N, dim, ctypes.c_float(h), _stream()))


def langevin_baoa(ctx: Context, box: Box, pos, vel, force, nl: NeighborList, dt: float, gamma: float, kT: float,
                  seed: int, step: torch.Tensor):
    b, n = box.c(), nl.c()
    _check("md_langevin_baoa", load().md_langevin_baoa(
        ctx.h, ctypes.byref(b), _ptr(pos), _ptr(vel), _ptr(force), pos.shape[0], ctypes.byref(n), ctypes.c_float(dt),
        ctypes.c_float(gamma), ctypes.c_float(kT), ctypes.c_uint64(seed), _ptr(step), _stream()))


def brownian_step(ctx: Context, box: Box, pos, force, nl: NeighborList, dt: float, gamma: float, kT: float,
                  seed: int, step: torch.Tensor | None):
    b, n = box.c(), nl.c()
    _check("md_brownian_step", load().md_brownian_step(
        ctx.h, ctypes.byref(b), _ptr(pos), _ptr(force), pos.shape[0], ctypes.byref(n), ctypes.c_float(dt),
        ctypes.c_float(gamma), ctypes.c_float(kT), ctypes.c_uint64(seed), _ptr(step), _stream()))


def gradient_step(ctx: Context, box: Box, pos, force, nl: NeighborList, dt: float):
    b, n = box.c(), nl.c()
    _check("md_gradient_step", load().md_gradient_step(ctx.h, ctypes.byref(b), _ptr(pos), _ptr(force), pos.shape[0],
                                                       ctypes.byref(n), ctypes.c_float(dt), _stream()))


def nhc_state_tensor(Q, kT: float, n_dof: int, device=None) -> torch.Tensor:
    """A Nose-Hoover chain state (md_nhc_state) in device memory: masses Q (chain length len(Q) <= 8), momenta and
    positions zero."""
    Q = [float(q) for q in Q]
    if not 1 <= len(Q) <= 8 or min(Q) <= 0.0:
        raise ValueError("chain of 1..8 positive masses")
    st = c_nhc_state()
    for k, q in enumerate(Q):
        st.Q[k] = q
    st.kT, st.scale, st.M, st.n_dof = float(kT), 1.0, len(Q), int(n_dof)
    raw = np.frombuffer(bytes(st), dtype=np.uint8).copy()
    return torch.as_tensor(raw, device=device or _dev())


def nhc_state_read(state: torch.Tensor) -> dict:
    s = c_nhc_state.from_buffer_copy(state.cpu().numpy().tobytes())
    return dict(p=np.array(s.p[: s.M]), eta=np.array(s.eta[: s.M]), Q=np.array(s.Q[: s.M]), kT=s.kT, scale=s.scale,
                M=s.M, n_dof=s.n_dof)


def nhc_half(ctx: Context, vel, state: torch.Tensor, h: float):
    N, dim = vel.shape
    _check("md_nhc_half", load().md_nhc_half(ctx.h, _ptr(vel), N, dim, _ptr(state), ctypes.c_double(h), _stream()))


def flock_step(ctx: Context, box: Box, pos, theta, nl: NeighborList, fp: c_flock_params, work,
               pred: c_flock_predators | None = None):
    b, n = box.c(), nl.c()
    _check("flock_step", load().flock_step(ctx.h, ctypes.byref(b), _ptr(pos), _ptr(theta), pos.shape[0],
                                           ctypes.byref(n), ctypes.byref(fp),
                                           ctypes.byref(pred) if pred is not None else None, _ptr(work), _stream()))


class HalfList:
    """Each pair of a full list once (row i keeps j when (i < j) differs from (i + j odd)): hidx [hcap][N],
    hcount [N], for the Newton's-third-law pass."""

    def __init__(self, ctx: Context, nl: NeighborList, hcap: int | None = None):
        self.ctx, self.nl = ctx, nl
        self.hcap = int(hcap or max(8, nl.capacity // 2 + 8))
        dev = ctx.device
        self.hidx = torch.zeros((self.hcap, nl.N), dtype=torch.int32, device=dev)
        self.hcount = torch.zeros(nl.N, dtype=torch.int32, device=dev)
        self.overflow = torch.zeros(1, dtype=torch.int32, device=dev)

    def update(self):
        n = self.nl.c()
        _check("nl_half", load().nl_half(self.ctx.h, ctypes.byref(n), _ptr(self.hidx), _ptr(self.hcount), self.hcap,
                                         _ptr(self.overflow), _stream()))

    def forces(self, box: Box, pot: Potential, pos, species, force):
        b, p = box.c(), pot.c()
        _check("pair_force_half", load().pair_force_half(
            self.ctx.h, ctypes.byref(b), ctypes.byref(p), _ptr(pos), _ptr(species), pos.shape[0], _ptr(self.hidx),
            _ptr(self.hcount), self.hcap, _ptr(force), _stream()))


def min_distance(ctx: Context, box: Box, pos, nl: NeighborList) -> torch.Tensor:
    out = torch.zeros(1, dtype=torch.float64, device=pos.device)
    b, n = box.c(), nl.c()
    _check("md_min_distance", load().md_min_distance(ctx.h, ctypes.byref(b), _ptr(pos), pos.shape[0], ctypes.byref(n),
                                                     _ptr(out), _stream()))
    return out


def rms_diff(ctx: Context, a, b) -> torch.Tensor:
    out = torch.zeros(1, dtype=torch.float64, device=a.device)
    _check("md_rms_diff", load().md_rms_diff(ctx.h, _ptr(a), _ptr(b), a.numel(), _ptr(out), _stream()))
    return out


def copy_words(ctx: Context, dst: torch.Tensor, src: torch.Tensor):
    """dst <- src as 16-byte words (both contiguous, same byte size, a multiple of 16)."""
    nb = src.numel() * src.element_size()
    if nb % 16 or dst.numel() * dst.element_size() != nb:
        raise ValueError("copy_words needs equal sizes that are multiples of 16 bytes")
    _check("md_copy_words", load().md_copy_words(ctx.h, _ptr(dst), _ptr(src), nb // 16, _stream()))


def rescale_velocities(ctx: Context, vel: torch.Tensor, T: float):
    N, dim = vel.shape
    _check("md_rescale_velocities", load().md_rescale_velocities(ctx.h, _ptr(vel), N, dim, ctypes.c_double(T),
                                                                 _stream()))


def verlet_step(ctx: Context, box: Box, pot: Potential, pos, vel, force, species, nl: NeighborList, dt: float,
                n_steps: int):
    N = pos.shape[0]
    _reserve_for(ctx, box, N, nl)
    b, p, n = box.c(), pot.c(), nl.c()
    _check("verlet_step", load().verlet_step(ctx.h, ctypes.byref(b), ctypes.byref(p), _ptr(pos), _ptr(vel),
                                             _ptr(force), _ptr(species), N, ctypes.byref(n),
                                             ctypes.c_float(dt), int(n_steps), _stream()))


def langevin_run(ctx: Context, box: Box, pot: Potential, pos, vel, force, species, nl: NeighborList, dt: float,
                 gamma: float, kT: float, seed: int, step: torch.Tensor, n_steps: int):
    N = pos.shape[0]
    _reserve_for(ctx, box, N, nl)
    b, p, n = box.c(), pot.c(), nl.c()
    _check("langevin_run", load().langevin_run(ctx.h, ctypes.byref(b), ctypes.byref(p), _ptr(pos), _ptr(vel),
                                               _ptr(force), _ptr(species), N, ctypes.byref(n), ctypes.c_float(dt),
                                               ctypes.c_float(gamma), ctypes.c_float(kT), ctypes.c_uint64(seed),
                                               _ptr(step), int(n_steps), _stream()))


def fire_init(ctx: Context, box: Box, pot: Potential, pos, vel, force, species, nl: NeighborList,
              fp: FireParams, state: torch.Tensor, f_tol: float):
    N = pos.shape[0]
    _reserve_for(ctx, box, N, nl)
    b, p, n, f = box.c(), pot.c(), nl.c(), fp.c()
    _check("fire_init", load().fire_init(ctx.h, ctypes.byref(b), ctypes.byref(p), _ptr(pos), _ptr(vel),
                                         _ptr(force), _ptr(species), N, ctypes.byref(n), ctypes.byref(f),
                                         _ptr(state), ctypes.c_double(f_tol), _stream()))


def fire_step(ctx: Context, box: Box, pot: Potential, pos, vel, force, species, nl: NeighborList,
              fp: FireParams, state: torch.Tensor, n_steps: int, f_tol: float, sync_rebuild: bool = False):
    """n_steps FIRE steps; sync_rebuild selects the list upkeep (pipelined, or a full rebuild before each force
    evaluation that needs one)."""
    N = pos.shape[0]
    _reserve_for(ctx, box, N, nl)
    b, p, n, f = box.c(), pot.c(), nl.c(), fp.c(sync_rebuild)
    _check("fire_step", load().fire_step(ctx.h, ctypes.byref(b), ctypes.byref(p), _ptr(pos), _ptr(vel),
                                         _ptr(force), _ptr(species), N, ctypes.byref(n), ctypes.byref(f),
                                         _ptr(state), int(n_steps), ctypes.c_double(f_tol), _stream()))


class Batch:
    """md_batch: B independent 2D replicas of uneven size, concatenated (offset[B+1], box[B][2], pos, species)."""

    def __init__(self, replicas, device=None):
        dev = device or _dev()
        self.B = len(replicas)
        self.dim = 2
        sizes = [int(r["u"].shape[0]) for r in replicas]
        self.sizes = sizes
        off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
        self.offset = torch.as_tensor(off, device=dev)
        boxes = np.array([[r["L"][0], r["L"][1]] for r in replicas], dtype=np.float32)
        self.boxes = boxes
        self.box = torch.as_tensor(boxes, device=dev)
        u = np.concatenate([np.asarray(r["u"], dtype=np.uint32) for r in replicas]) if replicas else \
            np.zeros((0, 2), np.uint32)
        self.pos = to_device_u32(u, dev)
        sp = [r.get("species") for r in replicas]
        self.species = None if sp and sp[0] is None else torch.as_tensor(
            np.concatenate([np.asarray(x, dtype=np.int32) for x in sp]), device=dev)
        self.max_n = max(sizes) if sizes else 0

    def max_cells(self, r_range: float) -> int:
        m = 1
        for Lx, Ly in self.boxes:
            c = 1
            for L in (Lx, Ly):
                k = int(np.floor(float(L) / (r_range * (1 + 1e-6))))
                c *= k if k >= 3 else 1
            m = max(m, c)
        return m

    def c(self, r_range: float) -> c_batch:
        b = c_batch()
        b.B, b.dim, b.max_n, b.max_cells = self.B, 2, self.max_n, self.max_cells(r_range)
        b.offset, b.box, b.pos = self.offset.data_ptr(), self.box.data_ptr(), self.pos.data_ptr()
        b.species = self.species.data_ptr() if self.species is not None else None
        return b

    def replica_positions(self, b: int) -> np.ndarray:
        off = self.offset.cpu().numpy()
        return from_device_u32(self.pos)[off[b]:off[b + 1]]


def fire_batched(ctx: Context, batch: Batch, pot: Potential, fp: FireParams, max_steps: int, f_tol: float,
                 config: tuple | None = None):
    """FIRE on every replica in one launch.  Returns (energy[B] f64, fmax[B] f64, steps[B] i32, status[B] i32).
    config: (threads per replica workgroup, cell factor), e.g. from autotune_fire_batched; None for the default."""
    dev = batch.pos.device
    e = torch.zeros(max(batch.B, 1), dtype=torch.float64, device=dev)
    fm = torch.zeros_like(e)
    st = torch.zeros(max(batch.B, 1), dtype=torch.int32, device=dev)
    status = torch.zeros_like(st)
    b, p, f = batch.c(pot.cutoff()), pot.c(), fp.c()
    cfg = None
    if config is not None:
        cfg = c_batch_config()
        cfg.threads, cfg.cell_factor = int(config[0]), float(config[1])
    _check("fire_batched", load().fire_batched(ctx.h, ctypes.byref(b), ctypes.byref(p), ctypes.byref(f),
                                               None if cfg is None else ctypes.byref(cfg), int(max_steps),
                                               ctypes.c_double(f_tol), _ptr(e), _ptr(fm), _ptr(st), _ptr(status),
                                               _stream()))
    return e[: batch.B], fm[: batch.B], st[: batch.B], status[: batch.B]


BATCH_CONFIGS = ((512, 1.0), (512, 1.25), (512, 1.5), (1024, 1.0), (1024, 1.25), (1024, 1.5))


def autotune_fire_batched(ctx: Context, batch: Batch, pot: Potential, fp: FireParams | None = None,
                          trial_steps: int = 200, candidates=BATCH_CONFIGS, repeats: int = 2) -> dict:
    """Launch shape for fire_batched on this batch: each candidate (threads per replica workgroup, cell factor) runs
    `trial_steps` FIRE steps on every replica (f_tol 0, from the batch's current positions, restored afterwards),
    timed with HIP events on the launch stream; the fastest (best of `repeats`) is returned with every timing.
    Trials take the same steps as a real run, so the time per step they measure is the one that matters."""
    fp = fp or FireParams()
    saved = batch.pos.clone()
    stream = torch.cuda.current_stream()
    times = {}
    for cfg in candidates:
        best = None
        for _ in range(repeats):
            batch.pos.copy_(saved)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fire_batched(ctx, batch, pot, fp, trial_steps, 0.0, config=cfg)
            e1.record(stream)
            torch.cuda.synchronize()
            t = e0.elapsed_time(e1)
            best = t if best is None else min(best, t)
        times[cfg] = best
    batch.pos.copy_(saved)
    choice = min(times, key=times.get)
    return {"config": choice, "ms_per_trial": {f"{t}x{c}": v for (t, c), v in times.items()},
            "trial_steps": trial_steps}


def envelope_grad(ctx: Context, batch: Batch, pot: Potential):
    """dU/dsigma_ab, dU/deps_ab (each [B][S][S], per ordered species pair) and U[B] at the batch positions."""
    dev = batch.pos.device
    S = pot.n_species
    gs = torch.zeros((max(batch.B, 1), S, S), dtype=torch.float64, device=dev)
    ge = torch.zeros_like(gs)
    e = torch.zeros(max(batch.B, 1), dtype=torch.float64, device=dev)
    b, p = batch.c(pot.cutoff()), pot.c()
    _check("envelope_grad", load().envelope_grad(ctx.h, ctypes.byref(b), ctypes.byref(p), _ptr(gs), _ptr(ge),
                                                 _ptr(e), None, _stream()))
    return gs[: batch.B], ge[: batch.B], e[: batch.B]


def envelope_grad_wrt(ctx: Context, batch: Batch, pot: Potential, wrt: int, box: int = BOX_FIXED, weights=None):
    """dU_b/dtheta for one parameter family (WRT_*) at the batch positions: [B][m] (m = S*S, S or 1), or with
    weights [B] (float64 device tensor) the weighted sum over replicas [m]."""
    dev = batch.pos.device
    S = pot.n_species
    m = S * S if wrt in (WRT_SIGMA, WRT_EPSILON) else (S if wrt == WRT_DIAMETER else 1)
    out = torch.zeros((m,) if weights is not None else (max(batch.B, 1), m), dtype=torch.float64, device=dev)
    b, p = batch.c(pot.cutoff()), pot.c()
    w = None if weights is None else weights.to(dev, torch.float64).contiguous()
    _check("envelope_grad_wrt", load().envelope_grad_wrt(ctx.h, ctypes.byref(b), ctypes.byref(p), int(wrt), int(box),
                                                         _ptr(w), _ptr(out), None, None, _stream()))
    return out if weights is not None else out[: batch.B]


def diameter_grad(ctx: Context, batch: Batch, pot: Potential, g_sigma: torch.Tensor, dln=None, box: int = BOX_FIXED,
                  sigma=None, weights=None):
    """md_diameter_grad: per-species diameter derivatives [B][S] (or weighted [S]) from dU/dsigma_ab g_sigma
    [B][S][S] (float64 device), with per-replica sigma [B][S][S] or the potential's, and for BOX_PACKING the box
    derivative dln [B] (or minus the virial for soft spheres when None)."""
    dev = batch.pos.device
    S = pot.n_species
    out = torch.zeros((S,) if weights is not None else (max(batch.B, 1), S), dtype=torch.float64, device=dev)
    b, p = batch.c(pot.cutoff()), pot.c()
    sg = None if sigma is None else torch.as_tensor(sigma, dtype=torch.float64, device=dev).contiguous()
    w = None if weights is None else weights.to(dev, torch.float64).contiguous()
    _check("md_diameter_grad", load().md_diameter_grad(ctx.h, ctypes.byref(b), ctypes.byref(p), _ptr(sg),
                                                       _ptr(g_sigma.contiguous()), _ptr(dln), int(box), _ptr(w),
                                                       _ptr(out), _stream()))
    return out if weights is not None else out[: batch.B]


def fire_unrolled_grad(ctx: Context, batch: Batch, pot: Potential, fp: FireParams, K: int, rbar0: bool = False,
                       mixed: bool = False, workspace=None, sigma=None):
    """K FIRE steps on every replica, then dE_K/dtheta by reverse mode through the steps (one launch).

    Returns a dict of device tensors: energy [B] f64, g_sigma and g_eps [B][S][S] f64 (ordered entries),
    g_lnc [B] f64 (box scale at fixed fractional start), status [B] i32, and when asked rbar0 [total][2] f32
    (dE_K/dR_0, fractional) and mixed [B][K] u8 (P > 0 per step).  The batch positions end at R_K.  The
    trajectory workspace is allocated here unless a uint8 device tensor of at least
    fire_unrolled_workspace_bytes bytes is passed; it is returned as "workspace".  sigma: optional per-replica
    sigma matrices [B][S][S] (float64 device tensor); the potential's own sigma is used when it is None.
    """
    lib = load()
    dev = batch.pos.device
    total = int(sum(batch.sizes))
    need = int(lib.fire_unrolled_workspace_bytes(batch.B, total, int(K)))
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    S = pot.n_species
    B1 = max(batch.B, 1)
    out = {
        "energy": torch.zeros(B1, dtype=torch.float64, device=dev),
        "g_sigma": torch.zeros((B1, S, S), dtype=torch.float64, device=dev),
        "g_eps": torch.zeros((B1, S, S), dtype=torch.float64, device=dev),
        "g_lnc": torch.zeros(B1, dtype=torch.float64, device=dev),
        "status": torch.zeros(B1, dtype=torch.int32, device=dev),
    }
    rb = torch.zeros((max(total, 1), 2), dtype=torch.float32, device=dev) if rbar0 else None
    mx = torch.zeros((B1, max(int(K), 1)), dtype=torch.uint8, device=dev) if mixed else None
    if sigma is not None:
        sigma = torch.as_tensor(sigma, dtype=torch.float64, device=dev).contiguous()
        if tuple(sigma.shape) != (batch.B, S, S):
            raise ValueError("sigma must be [B][S][S]")
    rng = pot.cutoff() if sigma is None or pot.kind == "lj" else max(pot.cutoff(), float(sigma.max()))
    b, p, f = batch.c(rng), pot.c(), fp.c()
    _check("fire_unrolled_grad", lib.fire_unrolled_grad(
        ctx.h, ctypes.byref(b), ctypes.byref(p), _ptr(sigma), ctypes.byref(f), int(K), _ptr(workspace), workspace.numel(),
        _ptr(out["energy"]), _ptr(out["g_sigma"]), _ptr(out["g_eps"]), _ptr(out["g_lnc"]), _ptr(rb), _ptr(mx),
        _ptr(out["status"]), _stream()))
    res = {k: v[: batch.B] for k, v in out.items()}
    if rb is not None:
        res["rbar0"] = rb[:total]
    if mx is not None:
        res["mixed"] = mx[: batch.B, : int(K)]
    res["workspace"] = workspace
    return res


class NNParams:
    """Device copy of the neural pair potential: BF16 W1 [H][K], W2 [H][H]; float b1, b2, w3 [H], b3; m, s [K]."""

    def __init__(self, W1, b1, W2, b2, w3, b3, m, s, mu0=0.8, mu1=2.5, r_c=2.5, device=None, eta=0.0):
        dev = device or _dev()

        def f32(a):
            return torch.as_tensor(np.asarray(a, dtype=np.float32), device=dev).contiguous()

        self.W1 = f32(W1).to(torch.bfloat16).contiguous()
        self.W2 = f32(W2).to(torch.bfloat16).contiguous()
        self.b1, self.b2, self.w3, self.m, self.s = f32(b1), f32(b2), f32(w3), f32(m), f32(s)
        self.b3 = f32([b3])
        self.mu0, self.mu1, self.r_c, self.eta = float(mu0), float(mu1), float(r_c), float(eta)
        self.K, self.H = int(self.W1.shape[1]), int(self.W1.shape[0])

    def c(self) -> c_nn_params:
        q = c_nn_params()
        q.K, q.H, q.mu0, q.mu1, q.r_c, q.eta = self.K, self.H, self.mu0, self.mu1, self.r_c, self.eta
        q.W1, q.W2 = self.W1.data_ptr(), self.W2.data_ptr()
        q.b1, q.b2, q.w3, q.b3, q.m, q.s = (t.data_ptr() for t in (self.b1, self.b2, self.w3, self.b3, self.m,
                                                                   self.s))
        return q

    def host(self) -> dict:
        """Weights as float64 numpy arrays (W1, W2 exactly the BF16 values)."""
        return dict(W1=self.W1.float().cpu().numpy().astype(np.float64),
                    W2=self.W2.float().cpu().numpy().astype(np.float64),
                    b1=self.b1.cpu().numpy().astype(np.float64), b2=self.b2.cpu().numpy().astype(np.float64),
                    w3=self.w3.cpu().numpy().astype(np.float64), b3=float(self.b3.cpu()[0]),
                    m=self.m.cpu().numpy().astype(np.float64), s=self.s.cpu().numpy().astype(np.float64))


def nn_descriptor_stats(ctx: Context, G: torch.Tensor, mean: torch.Tensor, scale: torch.Tensor):
    """Per-basis mean and population standard deviation of G [N][K] (float32 device) into mean, scale [K]."""
    _check("nn_descriptor_stats", load().nn_descriptor_stats(ctx.h, _ptr(G), G.shape[0], _ptr(mean), _ptr(scale),
                                                             _stream()))


def nn_descriptors(ctx: Context, box: Box, nn: NNParams, pos: torch.Tensor, nl: NeighborList) -> torch.Tensor:
    N = pos.shape[0]
    G = torch.zeros((N, nn.K), dtype=torch.float32, device=pos.device)
    b, q, n = box.c(), nn.c(), nl.c()
    _check("nn_descriptors", load().nn_descriptors(ctx.h, ctypes.byref(b), ctypes.byref(q), _ptr(pos), N,
                                                   ctypes.byref(n), _ptr(G), _stream()))
    return G


def nn_mlp(ctx: Context, nn: NNParams, G: torch.Tensor):
    N = G.shape[0]
    Ei = torch.zeros(N, dtype=torch.float32, device=G.device)
    e = torch.zeros((N, nn.K), dtype=torch.float32, device=G.device)
    q = nn.c()
    _check("nn_mlp", load().nn_mlp(ctx.h, ctypes.byref(q), _ptr(G), N, _ptr(Ei), _ptr(e), _stream()))
    return Ei, e


def nn_forces(ctx: Context, box: Box, nn: NNParams, pos: torch.Tensor, nl: NeighborList, e: torch.Tensor,
              force: torch.Tensor):
    N = pos.shape[0]
    b, q, n = box.c(), nn.c(), nl.c()
    _check("nn_forces", load().nn_forces(ctx.h, ctypes.byref(b), ctypes.byref(q), _ptr(pos), N, ctypes.byref(n),
                                         _ptr(e), _ptr(force), _stream()))


def md_sum(ctx: Context, x: torch.Tensor, out: torch.Tensor):
    _check("md_sum", load().md_sum(ctx.h, _ptr(x), x.numel(), _ptr(out), _stream()))


def kinetic_energy(ctx: Context, vel: torch.Tensor, out: torch.Tensor):
    _check("md_kinetic_energy", load().md_kinetic_energy(ctx.h, _ptr(vel), vel.shape[0], vel.shape[1], _ptr(out),
                                                         _stream()))


def kinetic_energy_noalloc(vel: torch.Tensor, out: torch.Tensor):
    """md_kinetic_energy_noalloc: no context, partial sums in the library's own per-GPU array."""
    _check("md_kinetic_energy_noalloc", load().md_kinetic_energy_noalloc(_ptr(vel), vel.shape[0], vel.shape[1],
                                                                         _ptr(out), _stream()))


def fire_state_tensor(device=None) -> torch.Tensor:
    return torch.zeros(FIRE_STATE_BYTES, dtype=torch.uint8, device=device or _dev())


def fire_state_read(state: torch.Tensor) -> dict:
    raw = state.cpu().numpy().tobytes()
    s = c_fire_state.from_buffer_copy(raw)
    return dict(dt=s.dt, alpha=s.alpha, fmax=s.fmax, power=s.power, mix_v=s.mix_v, mix_f=s.mix_f, steps=s.steps,
                n_pos=s.n_pos, converged=bool(s.converged))


# --------------------------------------------------------- init / update helpers

def to_device_u32(u: np.ndarray, device=None) -> torch.Tensor:
    """uint32 torus coordinates (numpy) -> int32 tensor holding the same bits."""
    return torch.from_numpy(np.ascontiguousarray(u, dtype=np.uint32).view(np.int32)).to(device or _dev())


def from_device_u32(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy().view(np.uint32)


MAX_PER_CELL = 252  # bin capacity limit of the library


class System:
    """A periodic system on the GPU: positions, velocities, forces, species, and its neighbor list."""

    def __init__(self, box: Box, pot: Potential, u: np.ndarray, v=None, species=None, skin: float = 0.3,
                 capacity: int | None = None, ctx: Context | None = None, max_per_cell: int | None = None,
                 lanes: int | None = None):
        self.ctx = ctx or Context()
        dev = self.ctx.device
        self.box, self.pot = box, pot
        self.N, self.dim = u.shape
        self.pos = to_device_u32(u, dev)
        self.vel = torch.zeros((self.N, self.dim), dtype=torch.float32, device=dev) if v is None else \
            torch.as_tensor(np.asarray(v, dtype=np.float32), device=dev).contiguous()
        self.force = torch.zeros((self.N, self.dim), dtype=torch.float32, device=dev)
        self.species = None if species is None else torch.as_tensor(np.asarray(species, dtype=np.int32),
                                                                     device=dev).contiguous()
        if pot.n_species > 1 and self.species is None:
            raise ValueError("multi-species potential needs species")
        r_list = float(np.float32(pot.cutoff() + skin))
        vol = float(np.prod(np.asarray(box.L[: self.dim], dtype=np.float64)))
        ball = (4.0 / 3.0 * np.pi * r_list ** 3) if self.dim == 3 else (np.pi * r_list ** 2)
        mean_row = self.N / vol * ball
        if lanes is None:
            # enough lanes per particle that a lane walks ~20 entries
            lanes = 1
            while lanes < 8 and mean_row / lanes > 24:
                lanes *= 2
        if capacity is None:
            # rows are dealt round-robin over the lanes, so the capacity only covers the spread of row lengths
            capacity = int(max(16, 1.3 * mean_row + 16))
            capacity = (capacity + 7) // 8 * 8
        if max_per_cell is None:
            cells = max(1, cell_count(box, r_list))
            mean = self.N / cells
            max_per_cell = 8
            while max_per_cell < 2.5 * mean + 8 and max_per_cell < MAX_PER_CELL:
                max_per_cell = min(2 * max_per_cell, MAX_PER_CELL)
        self.nl = NeighborList(self.N, self.dim, capacity, r_list, skin, dev, max_per_cell, lanes)

    def build(self):
        """Build the neighbor list, growing its capacity or bin size if something did not fit."""
        for _ in range(6):
            self.nl.clear_flags()
            nl_build(self.ctx, self.box, self.pos, self.nl)
            f = self.nl.read_flags()
            if not (f[FLAG_OVERFLOW] or f[FLAG_CELL_OVERFLOW]):
                return
            self.grow(f)
        raise RuntimeError("neighbor list did not fit after growing")

    def grow(self, f):
        """New list sized from the flag words of a failed build or run."""
        cap, M = self.nl.capacity, self.nl.max_per_cell
        if f[FLAG_OVERFLOW]:
            cap = (int(f[FLAG_MAXCOUNT] * 1.25) + 8) // 8 * 8
        if f[FLAG_CELL_OVERFLOW]:
            if f[FLAG_MAXCELL] > MAX_PER_CELL:
                raise RuntimeError(f"a cell holds {int(f[FLAG_MAXCELL])} particles; bins hold at most {MAX_PER_CELL}")
            while M < f[FLAG_MAXCELL]:
                M = min(2 * M, MAX_PER_CELL)
        self.nl = NeighborList(self.N, self.dim, cap, self.nl.r_list, self.nl.skin, self.ctx.device, M,
                               self.nl.lanes)

    def forces(self, energy: bool = False):
        e = torch.zeros(self.N, dtype=torch.float64, device=self.ctx.device) if energy else None
        w = torch.zeros(self.N, dtype=torch.float64, device=self.ctx.device) if energy else None
        pair_energy_force(self.ctx, self.box, self.pot, self.pos, self.species, self.nl, self.force, e, w)
        return e, w

    def potential_energy(self) -> float:
        e = torch.zeros(self.N, dtype=torch.float64, device=self.ctx.device)
        pair_energy_force(self.ctx, self.box, self.pot, self.pos, self.species, self.nl, None, e, None)
        out = torch.zeros(1, dtype=torch.float64, device=self.ctx.device)
        md_sum(self.ctx, e, out)
        return float(out.item())

    def kinetic_energy(self) -> float:
        out = torch.zeros(1, dtype=torch.float64, device=self.ctx.device)
        kinetic_energy(self.ctx, self.vel, out)
        return float(out.item())


def _run_checked(system: System, saved, call, n_steps: int, on_stale=None):
    """Run call(n) and re-run from `saved` when the device reported a list that did not fit (grow it) or went
    stale: with `on_stale`, run the same steps through it (a call whose list cannot go stale); otherwise in
    shorter pieces, each starting from a fresh list (a piece of one step cannot go stale unless a single step
    moves a particle more than skin/2)."""
    for _ in range(6):
        system.nl.clear_flags()
        call(n_steps)
        f = system.nl.read_flags()
        if not (f[FLAG_OVERFLOW] or f[FLAG_CELL_OVERFLOW] or f[FLAG_STALE]):
            if f[FLAG_NONFINITE]:
                raise FloatingPointError("non-finite force")
            return f
        for t, v in zip(saved[0], saved[1]):
            t.copy_(v)
        if f[FLAG_STALE] and on_stale is not None:
            call, on_stale = on_stale, None
            continue
        if f[FLAG_STALE]:
            if n_steps == 1:
                raise RuntimeError(f"a single step left the list stale: flags {f.tolist()}")
            piece = max(1, n_steps // 8)
            done = 0
            while done < n_steps:
                k = min(piece, n_steps - done)
                sub = (saved[0], tuple(t.clone() for t in saved[0]))
                f = _run_checked(system, sub, call, k)
                done += k
            return f
        system.grow(f)
        system.build()  # a step may read the list before any rebuild (flocking does): build it for the restored state
    raise RuntimeError("neighbor list kept overflowing")


def nve(system: System, dt: float):
    """init_fn / update_fn pair for constant-energy dynamics (paper Sec. 3.3.1, ``simulate.nve``).

    ``init_fn()`` builds the list and the forces; ``update_fn(n)`` advances n velocity-Verlet steps on the
    device (one verlet_step call), re-running from a saved copy if the device reported a problem.
    """

    def init_fn():
        system.build()
        system.forces()
        return system

    def update_fn(n_steps: int = 1):
        tensors = (system.pos, system.vel, system.force)
        saved = (tensors, tuple(t.clone() for t in tensors))

        def call(n):
            verlet_step(system.ctx, system.box, system.pot, system.pos, system.vel, system.force, system.species,
                        system.nl, dt, n)

        system.last_flags = _run_checked(system, saved, call, n_steps)
        return system

    return init_fn, update_fn


def _stepper(system: System, step_once, state_tensors, chunk: int = 20):
    """update_fn(n, graph=False) for an integrator whose step is a fixed sequence of launches (step_once).  The
    device decides every rebuild (nl_update), so `chunk` steps can be captured once in a HIP graph and replayed;
    flags are read after every run, and a run that reports an overflow is re-run eagerly from its saved state."""
    graphs = {}

    def eager(n):
        for _ in range(n):
            step_once()

    def update_fn(n_steps: int = 1, graph: bool = False):
        done = 0
        while done < n_steps:
            k = min(chunk, n_steps - done) if graph else n_steps - done
            saved = (state_tensors, tuple(t.clone() for t in state_tensors))
            if graph and k == chunk:
                g = graphs.get(chunk)
                if g is None:
                    g = torch.cuda.CUDAGraph()
                    with torch.cuda.graph(g):  # records the launches; nothing runs until a replay
                        eager(chunk)
                    graphs[chunk] = g
                system.nl.clear_flags()
                g.replay()
                f = system.nl.read_flags()
                if f[FLAG_OVERFLOW] or f[FLAG_CELL_OVERFLOW] or f[FLAG_STALE]:
                    for t, v in zip(saved[0], saved[1]):
                        t.copy_(v)
                    graphs.clear()
                    if f[FLAG_OVERFLOW] or f[FLAG_CELL_OVERFLOW]:
                        system.grow(f)
                        system.build()  # the grown list must be valid for the restored positions
                    system.last_flags = _run_checked(system, saved, eager, k)
                elif f[FLAG_NONFINITE]:
                    raise FloatingPointError("non-finite force")
                else:
                    system.last_flags = f
            else:
                system.last_flags = _run_checked(system, saved, eager, k)
            done += k
        return system

    return update_fn


def _init_forces(system: System):
    def init_fn():
        system.build()
        system.forces()
        return system
    return init_fn


def nvt_langevin(system: System, dt: float, gamma: float, kT: float, seed: int = 0, fused: bool = False):
    """init_fn / update_fn for Langevin dynamics at temperature kT (Sec. 3.3.1 ``simulate.nvt_langevin``; BAOAB
    with friction gamma, unit masses).  The step counter that indexes the noise lives on the device.  fused=True
    runs the steps like ``nve`` (langevin_run: one launch per step, the list rebuilt inside the run); otherwise a
    step is the BAOA launch, the device-gated rebuild, the force pass and the closing kick."""
    step = torch.zeros(1, dtype=torch.int64, device=system.ctx.device)
    if fused:
        def update_fn(n_steps: int = 1, graph: bool = False):
            tensors = (system.pos, system.vel, system.force, step)
            saved = (tensors, tuple(t.clone() for t in tensors))

            def call(n):
                langevin_run(system.ctx, system.box, system.pot, system.pos, system.vel, system.force,
                             system.species, system.nl, dt, gamma, kT, seed, step, n)

            system.last_flags = _run_checked(system, saved, call, n_steps)
            return system

        update_fn.step = step
        return _init_forces(system), update_fn

    def once():
        langevin_baoa(system.ctx, system.box, system.pos, system.vel, system.force, system.nl, dt, gamma, kT, seed,
                      step)
        nl_update(system.ctx, system.box, system.pos, system.nl)
        system.forces()
        kick(system.ctx, system.vel, system.force, 0.5 * dt)

    return _init_forces(system), _stepper(system, once, (system.pos, system.vel, system.force, step))


def brownian(system: System, dt: float, gamma: float, kT: float, seed: int = 0):
    """init_fn / update_fn for Brownian (overdamped Langevin) dynamics at temperature kT, friction gamma
    (Sec. 3.3.1 ``simulate.brownian``; Euler-Maruyama)."""
    step = torch.zeros(1, dtype=torch.int64, device=system.ctx.device)

    def once():
        brownian_step(system.ctx, system.box, system.pos, system.force, system.nl, dt, gamma, kT, seed, step)
        nl_update(system.ctx, system.box, system.pos, system.nl)
        system.forces()

    return _init_forces(system), _stepper(system, once, (system.pos, system.force, step))


def gradient_descent(system: System, dt: float):
    """init_fn / update_fn for steepest descent x += dt F (Sec. 3.3.1 ``minimize.gradient_descent``)."""

    def once():
        gradient_step(system.ctx, system.box, system.pos, system.force, system.nl, dt)
        nl_update(system.ctx, system.box, system.pos, system.nl)
        system.forces()

    return _init_forces(system), _stepper(system, once, (system.pos, system.force))


def nvt_nose_hoover(system: System, dt: float, kT: float, Q=(1.0,)):
    """init_fn / update_fn for a Nose-Hoover chain at temperature kT with thermostat masses Q (Sec. 3.3.1
    ``simulate.nvt_nose_hoover``, Martyna et al.).  The chain state (md_nhc_state) is returned as the third
    element; nhc_state_read decodes it."""
    state = nhc_state_tensor(Q, kT, system.N * system.dim, system.ctx.device)

    def once():
        nhc_half(system.ctx, system.vel, state, 0.5 * dt)
        kick_drift(system.ctx, system.box, system.pos, system.vel, system.force, system.nl, dt)
        nl_update(system.ctx, system.box, system.pos, system.nl)
        system.forces()
        kick(system.ctx, system.vel, system.force, 0.5 * dt)
        nhc_half(system.ctx, system.vel, state, 0.5 * dt)

    return _init_forces(system), _stepper(system, once, (system.pos, system.vel, system.force, state)), state


def autotune_lanes(system: System, dt: float, candidates=(2, 4, 8), steps: int = 60, repeats: int = 2) -> dict:
    """Choose the lanes per particle (W) of a system's neighbor list by timing NVE steps with each candidate on
    a copy of its state; the system keeps its state and gets a list with the fastest W.  Returns the timings
    (us per step) and the choice."""
    saved = (system.pos.clone(), system.vel.clone(), system.force.clone())
    nl0 = system.nl
    res = {}
    for W in candidates:
        system.nl = NeighborList(system.N, system.dim, nl0.capacity, nl0.r_list, nl0.skin, system.ctx.device,
                                 nl0.max_per_cell, W, nl0.segment)
        init, update = nve(system, dt)
        best = float("inf")
        for _ in range(repeats):
            for t, v in zip((system.pos, system.vel, system.force), saved):
                t.copy_(v)
            init()
            update(5)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            update(steps)
            torch.cuda.synchronize()
            best = min(best, (time.perf_counter() - t0) / steps * 1e6)
        res[W] = best
    choice = min(res, key=res.get)
    for t, v in zip((system.pos, system.vel, system.force), saved):
        t.copy_(v)
    system.nl = NeighborList(system.N, system.dim, nl0.capacity, nl0.r_list, nl0.skin, system.ctx.device,
                             nl0.max_per_cell, choice, nl0.segment)
    system.build()
    system.forces()
    return {"us_per_step": res, "lanes": choice}


def fire_descent(system: System, fp: FireParams | None = None, f_tol: float = 1e-6):
    """init_fn / step_fn pair for FIRE minimization (paper Sec. 3.3.1, App. A ``minimize.fire_descent``)."""
    fp = fp or FireParams()
    state = fire_state_tensor(system.ctx.device)

    def init_fn():
        system.build()
        system.vel.zero_()
        fire_init(system.ctx, system.box, system.pot, system.pos, system.vel, system.force, system.species,
                  system.nl, fp, state, f_tol)
        return state

    def call(n: int, sync: bool):
        fire_step(system.ctx, system.box, system.pot, system.pos, system.vel, system.force, system.species,
                  system.nl, fp, state, n, f_tol, sync)

    def step_fn(n_steps: int = 1, sync: bool = False):
        """n_steps FIRE steps in one call: the list pipeline (sync=False) or a full rebuild before each force
        evaluation that needs one (sync=True).  A pipelined run whose list went stale (a step too long for the
        pipeline's lookahead, as in the first steps from an overlapping start) is run again synchronously."""
        tensors = (system.pos, system.vel, system.force, state)
        saved = (tensors, tuple(t.clone() for t in tensors))
        _run_checked(system, saved, lambda n: call(n, sync), n_steps, on_stale=lambda n: call(n, True))
        return fire_state_read(state)

    graphs = {}

    def minimize(max_steps: int = 100000, chunk: int = 200, graph: bool = False):
        """Run FIRE until converged or max_steps, in fire_step calls of `chunk` steps.  With graph=True the
        launches of a chunk are captured once in a HIP graph and replayed (a step's launches are all device-gated,
        so replays need no host decisions).  The flags are read after every chunk; a chunk that reports a problem
        is re-run eagerly from its saved state.  The first chunk runs with a full rebuild before each force
        evaluation that needs one (the first steps from an overlapping start are too long for the list pipeline),
        and so do the chunks after it until a chunk needs no more than one rebuild per 6 steps; then chunks use the
        pipeline, and one whose list went stale is re-run synchronously and the rule starts over.  Synchronous
        chunks are a fifth as long (at least 20 steps), so that the switch comes soon after the steps have
        shortened.  The returned state also holds "rebuilds" (list builds
        over the call: one at the start of every chunk, plus the device's) and "chunks" (how many ran each way)."""
        st = fire_state_read(state)
        rebuilds = 0
        chunks = {"pipelined": 0, "synchronous": 0, "stale_reruns": 0}
        sync = True
        while not st["converged"] and st["steps"] < max_steps:
            size = max(20, chunk // 5) if sync else chunk
            k = min(size, max_steps - st["steps"])
            tensors = (system.pos, system.vel, system.force, state)
            saved = tuple(t.clone() for t in tensors)
            system.nl.clear_flags()
            if graph and k == size:
                g = graphs.get((size, sync))
                if g is None:
                    g = torch.cuda.CUDAGraph()
                    with torch.cuda.graph(g):  # records the launches; nothing runs until a replay
                        call(size, sync)
                    graphs[(size, sync)] = g
                g.replay()
            else:
                call(k, sync)
            f = system.nl.read_flags()
            if f[FLAG_OVERFLOW] or f[FLAG_CELL_OVERFLOW] or f[FLAG_STALE] or f[FLAG_NONFINITE]:
                for t, v in zip(tensors, saved):
                    t.copy_(v)
                if f[FLAG_OVERFLOW] or f[FLAG_CELL_OVERFLOW]:
                    graphs.clear()  # the list will be regrown (new buffers): capture again afterwards
                if f[FLAG_STALE]:
                    chunks["stale_reruns"] += 1
                    sync = True
                step_fn(k, sync)
                f = system.nl.read_flags()
            rebuilds += int(f[FLAG_REBUILDS])
            chunks["synchronous" if sync else "pipelined"] += 1
            if sync and 6 * int(f[FLAG_REBUILDS]) <= k:
                sync = False
            st = fire_state_read(state)
        st["rebuilds"] = rebuilds
        st["chunks"] = chunks
        return st

    return init_fn, step_fn, minimize


FLOCK_DEFAULTS = dict(J_align=1.0, R_align=3.0, J_avoid=25.0, R_avoid=1.0, J_coh=0.05, R_coh=3.0, J_obs=10.0,
                      alpha=3.0, v=1.0, dt=0.05)
PREDATOR_DEFAULTS = dict(J_flee=10.0, R_flee=4.0, J_chase=1.0, R_chase=8.0, v=1.2)


class Flock(System):
    """Boids of the flocking model (Sec. 4.3, App. B): positions pos (uint32 torus, [N][2]), headings theta [N],
    and a full neighbor list of radius max(R_align, R_avoid, R_coh) + skin.  ``params`` overrides FLOCK_DEFAULTS;
    ``obstacles`` is a list of disks (C_x, C_y, D), at most 16; ``lanes`` GPU lanes share each boid.
    ``predators`` = (uint32 positions [P][2], headings [P]) adds the predators of App. B (``predator_params``
    overrides PREDATOR_DEFAULTS); they live in ``ppos`` and ``ptheta``."""

    def __init__(self, box: Box, u: np.ndarray, theta, params: dict | None = None, obstacles=(), skin: float = 0.5,
                 capacity: int | None = None, ctx: Context | None = None, max_per_cell: int | None = None,
                 lanes: int = 4, predators=None, predator_params: dict | None = None):
        if box.dim != 2:
            raise ValueError("the flocking model is two-dimensional")
        p = dict(FLOCK_DEFAULTS, **(params or {}))
        obstacles = np.asarray(obstacles, dtype=np.float64).reshape(-1, 3)
        if len(obstacles) > 16:
            raise ValueError("at most 16 obstacles")
        self.fp = c_flock_params(**{k: float(v) for k, v in p.items()})
        self.fp.n_obstacles = len(obstacles)
        for o, (cx, cy, D) in enumerate(obstacles):
            self.fp.obstacles[3 * o: 3 * o + 3] = (float(cx), float(cy), float(D))
        self.params = p
        r = max(p["R_align"], p["R_avoid"], p["R_coh"])
        # the list radius is r + skin; the stand-in potential only carries the range r and is never evaluated
        super().__init__(box, Potential("soft_sphere", [[r]], [[1.0]], alpha=2.0), u, None, None, skin, capacity, ctx,
                         max_per_cell, lanes)
        self.theta = torch.as_tensor(np.asarray(theta, dtype=np.float32), device=self.ctx.device).contiguous()
        self.work = torch.zeros((self.N, 8), dtype=torch.float32, device=self.ctx.device)
        self.pred = None
        if predators is not None:
            up, thp = predators
            self.ppos = to_device_u32(np.asarray(up, np.uint32).reshape(-1, 2), self.ctx.device)
            self.ptheta = torch.as_tensor(np.asarray(thp, dtype=np.float32), device=self.ctx.device).contiguous()
            q = dict(PREDATOR_DEFAULTS, **(predator_params or {}))
            self.predator_params = q
            self.pred = c_flock_predators(P=self.ppos.shape[0], **{k: float(v) for k, v in q.items()})
            self.pred.pos, self.pred.theta = self.ppos.data_ptr(), self.ptheta.data_ptr()


def flocking(flock: Flock):
    """init_fn / update_fn for the forward-Euler flocking dynamics: each step is flock_step then nl_update (the
    rebuild decided on the device), so update_fn(n, graph=True) replays chunks of 20 steps from a HIP graph."""

    def init_fn():
        flock.build()
        return flock

    def once():
        flock_step(flock.ctx, flock.box, flock.pos, flock.theta, flock.nl, flock.fp, flock.work, flock.pred)
        nl_update(flock.ctx, flock.box, flock.pos, flock.nl)

    state = (flock.pos, flock.theta) + ((flock.ppos, flock.ptheta) if flock.pred is not None else ())
    return init_fn, _stepper(flock, once, state)
