"""Neural pair potential: training on the GPU from plain-engine data, and MD with it (paper Sec. 3.2.4, 4.1).

Every numerical step runs in the library's kernels (include/md.h): descriptors, the MFMA network pass,
forces, the loss, the pair adjoint, the weight gradient and Adam.  This module holds the parameters as
device tensors and sequences the calls.

  generate_lj_data   snapshots of 3D LJ runs by the plain engine: positions, total potential energies
                     (double) and forces, with a segmented neighbor list per minibatch.
  Network            FP32 master weights theta (flat, the layout nn_param_count() describes), Adam moments,
                     the BF16 copies W1, W2, and the descriptor shift / scale.
  train              minibatch Adam on L = mean_s ((E_s - E^_s)/n)^2 + lam_F mean |F - F^|^2.
  NNSystem           NVE with network forces, plain LJ as fallback: every `check_every` steps the LJ forces
                     of the same configuration judge the network's force RMSE, and a run that exceeds the
                     threshold continues with LJ.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np
import torch

from . import inputs, md

K, H = 16, 64


class Network:
    """Parameters on the device.  theta: float32 [P]; W1, W2: BF16 copies; m, s: descriptor shift / scale."""

    def __init__(self, ctx: md.Context, weights: dict, m, s, mu0=0.8, mu1=2.5, r_c=2.5, eta=0.0):
        dev = ctx.device
        P = int(md.load().nn_param_count())
        th = np.concatenate([np.asarray(weights["W1"], np.float64).ravel(), np.asarray(weights["b1"]).ravel(),
                             np.asarray(weights["W2"], np.float64).ravel(), np.asarray(weights["b2"]).ravel(),
                             np.asarray(weights["w3"]).ravel(), [float(weights["b3"])]])
        if th.size != P:
            raise ValueError(f"parameter count {th.size} != {P}")
        self.P = P
        self.theta = torch.as_tensor(th.astype(np.float32), device=dev).contiguous()
        self.m_adam = torch.zeros(P, dtype=torch.float32, device=dev)
        self.v_adam = torch.zeros(P, dtype=torch.float32, device=dev)
        self.W1 = torch.zeros(H * K, dtype=torch.int16, device=dev)
        self.W2 = torch.zeros(H * H, dtype=torch.int16, device=dev)
        as_dev = lambda x: (x.to(dev, torch.float32) if isinstance(x, torch.Tensor)
                            else torch.as_tensor(np.asarray(x, np.float32), device=dev)).contiguous()
        self.m, self.s = as_dev(m), as_dev(s)
        self.mu0, self.mu1, self.r_c = float(mu0), float(mu1), float(r_c)
        self.eta = float(eta)   # 0: the default width 1/(2 Delta^2) of the basis
        self.step = 0
        md._check("nn_cast_weights", md.load().nn_cast_weights(ctx.h, md._ptr(self.theta),
                                                                 md._ptr(self.W1), md._ptr(self.W2), md._stream()))

    def c(self) -> md.c_nn_params:
        q = md.c_nn_params()
        q.K, q.H, q.mu0, q.mu1, q.r_c, q.eta = K, H, self.mu0, self.mu1, self.r_c, self.eta
        base = self.theta.data_ptr()
        o_b1, o_W2 = H * K, H * K + H
        o_b2 = o_W2 + H * H
        o_w3, o_b3 = o_b2 + H, o_b2 + 2 * H
        q.W1, q.W2 = self.W1.data_ptr(), self.W2.data_ptr()
        q.b1, q.b2, q.w3, q.b3 = base + 4 * o_b1, base + 4 * o_b2, base + 4 * o_w3, base + 4 * o_b3
        q.m, q.s = self.m.data_ptr(), self.s.data_ptr()
        return q

    def host(self) -> dict:
        """Parameters as float64 numpy arrays, W1 and W2 exactly the BF16 values the kernels use."""
        th = self.theta.cpu().numpy().astype(np.float64)
        bf = lambda t, shape: (t.cpu().numpy().astype(np.uint16).astype(np.uint32) << 16).view(np.float32) \
            .astype(np.float64).reshape(shape)
        o_b1, o_W2 = H * K, H * K + H
        o_b2 = o_W2 + H * H
        return dict(W1=bf(self.W1, (H, K)), b1=th[o_b1:o_W2], W2=bf(self.W2, (H, H)), b2=th[o_b2:o_b2 + H],
                    w3=th[o_b2 + H:o_b2 + 2 * H], b3=float(th[-1]), m=self.m.cpu().numpy().astype(np.float64),
                    s=self.s.cpu().numpy().astype(np.float64))

    def adam(self, ctx: md.Context, grad: torch.Tensor, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step += 1
        md._check("nn_adam", md.load().nn_adam(ctx.h, md._ptr(self.theta), md._ptr(self.m_adam),
                                               md._ptr(self.v_adam), md._ptr(grad), self.P, self.step,
                                               ctypes.c_float(lr), ctypes.c_float(beta1), ctypes.c_float(beta2),
                                               ctypes.c_float(eps), md._ptr(self.W1), md._ptr(self.W2),
                                               md._stream()))


# ------------------------------------------------------------------ calls

def descriptors(ctx, box, net, pos, nl):
    N = pos.shape[0]
    G = torch.zeros((N, K), dtype=torch.float32, device=pos.device)
    b, q, n = box.c(), net.c(), nl.c()
    md._check("nn_descriptors", md.load().nn_descriptors(ctx.h, ctypes.byref(b), ctypes.byref(q), md._ptr(pos), N,
                                                         ctypes.byref(n), md._ptr(G), md._stream()))
    return G


def mlp(ctx, net, G):
    N = G.shape[0]
    Ei = torch.zeros(N, dtype=torch.float32, device=G.device)
    e = torch.zeros((N, K), dtype=torch.float32, device=G.device)
    q = net.c()
    md._check("nn_mlp", md.load().nn_mlp(ctx.h, ctypes.byref(q), md._ptr(G), N, md._ptr(Ei), md._ptr(e),
                                         md._stream()))
    return Ei, e


def forces(ctx, box, net, pos, nl, e, out=None):
    N = pos.shape[0]
    F = torch.zeros((N, 3), dtype=torch.float32, device=pos.device) if out is None else out
    b, q, n = box.c(), net.c(), nl.c()
    md._check("nn_forces", md.load().nn_forces(ctx.h, ctypes.byref(b), ctypes.byref(q), md._ptr(pos), N,
                                               ctypes.byref(n), md._ptr(e), md._ptr(F), md._stream()))
    return F


def loss(ctx, Ei, F, E_ref, F_ref, segment, lam_F=1.0):
    N = Ei.shape[0]
    S = N // segment
    out = torch.zeros(1, dtype=torch.float64, device=Ei.device)
    gE = torch.zeros(S, dtype=torch.float32, device=Ei.device)
    lam = torch.zeros((N, 3), dtype=torch.float32, device=Ei.device)
    md._check("nn_loss", md.load().nn_loss(ctx.h, md._ptr(Ei), md._ptr(F), md._ptr(E_ref), md._ptr(F_ref), N,
                                           segment, ctypes.c_float(lam_F), md._ptr(out), md._ptr(gE), md._ptr(lam),
                                           md._stream()))
    return out, gE, lam


def pair_adjoint(ctx, box, net, pos, nl, lam):
    N = pos.shape[0]
    ebar = torch.zeros((N, K), dtype=torch.float32, device=pos.device)
    b, q, n = box.c(), net.c(), nl.c()
    md._check("nn_pair_adjoint", md.load().nn_pair_adjoint(ctx.h, ctypes.byref(b), ctypes.byref(q), md._ptr(pos),
                                                           N, ctypes.byref(n), md._ptr(lam), md._ptr(ebar),
                                                           md._stream()))
    return ebar


def mlp_grad(ctx, net, G, segment, gE, ebar):
    grad = torch.zeros(net.P, dtype=torch.float32, device=G.device)
    q = net.c()
    md._check("nn_mlp_grad", md.load().nn_mlp_grad(ctx.h, ctypes.byref(q), md._ptr(G), G.shape[0], segment,
                                                   md._ptr(gE), md._ptr(ebar), md._ptr(grad), md._stream()))
    return grad


# ------------------------------------------------------------------ data

class Batch:
    """A minibatch of S snapshots of n atoms as one segmented system: positions, list, descriptors, references."""

    def __init__(self, ctx, box, net, pos, E_ref, F_ref, n, r_list, capacity=None, lanes=2):
        self.pos, self.E_ref, self.F_ref, self.n = pos, E_ref, F_ref, n
        N = pos.shape[0]
        if capacity is None:
            rho = n / float(np.prod(np.asarray(box.L[:3], dtype=np.float64)))
            capacity = int(1.3 * 4.0 / 3.0 * math.pi * r_list ** 3 * rho + 16)
            capacity = (capacity + 7) // 8 * 8
        self.nl = md.NeighborList(N, 3, capacity, r_list, 0.0, max_per_cell=64, lanes=lanes, segment=n)
        md.nl_build(ctx, box, pos, self.nl)
        f = self.nl.read_flags()
        if f[md.FLAG_OVERFLOW] or f[md.FLAG_CELL_OVERFLOW]:
            raise RuntimeError(f"training list did not fit: {f.tolist()}")
        self.G = descriptors(ctx, box, net, pos, self.nl)


def generate_lj_data(ctx: md.Context, n_runs=20, per_run=100, equilibrate=2000, every=50, seed=5001,
                     progress=None):
    """Snapshots of plain-engine LJ runs (rc 2.5, shifted energy, skin 0.3, dt 0.005) held near temperatures
    spread over [0.5, 1.5] by velocity rescaling every 50 steps: returns the box, positions [S][N][3] (uint32,
    device), energies [S] (float64, device), forces [S][N][3] (float32, device) and the temperatures."""
    runs = inputs.lj_train_runs(n_runs=n_runs, seed=seed)
    L = runs[0]["L"]
    box = md.Box(tuple(L), 3)
    pot = md.Potential("lj", [[1.0]], [[1.0]], r_cut=2.5)
    P, E, F, T = [], [], [], []
    for k, r in enumerate(runs):
        s = md.System(box, pot, r["u"], r["v"], skin=0.3, ctx=ctx)
        init, update = md.nve(s, 0.005)
        init()
        for _ in range(max(1, equilibrate // 50)):
            update(50)
            md.rescale_velocities(ctx, s.vel, r["T"])
        for _ in range(per_run):
            for _ in range(max(1, every // 50)):
                update(min(50, every))
                md.rescale_velocities(ctx, s.vel, r["T"])
            e, _ = s.forces(energy=True)
            tot = torch.zeros(1, dtype=torch.float64, device=e.device)
            md.md_sum(ctx, e, tot)
            P.append(s.pos.clone())
            E.append(tot)
            F.append(s.force.clone())
            T.append(r["T"])
        if progress:
            progress(f"run {k + 1}/{len(runs)} (T {r['T']:.2f}) sampled")
    return box, torch.stack(P), torch.cat(E), torch.stack(F), np.array(T)


def descriptor_scale(ctx, G: torch.Tensor):
    """Per-basis mean and standard deviation of the training descriptors (nn_descriptor_stats, on the device)."""
    K = G.shape[1]
    m = torch.zeros(K, dtype=torch.float32, device=G.device)
    s = torch.ones(K, dtype=torch.float32, device=G.device)
    md.nn_descriptor_stats(ctx, G.contiguous(), m, s)
    return m, s


def make_batches(ctx, box, net, P, E, F, idx, per_batch, r_list=2.5):
    n = P.shape[1]
    out = []
    for a in range(0, len(idx), per_batch):
        sel = torch.as_tensor(np.asarray(idx[a:a + per_batch]), device=P.device)
        pos = P[sel].reshape(-1, 3).contiguous()
        out.append(Batch(ctx, box, net, pos, E[sel].contiguous(), F[sel].reshape(-1, 3).contiguous(), n, r_list))
    return out


def train_step(ctx, box, net, batch: Batch, lr, lam_F=1.0):
    """One Adam step on one minibatch; returns the loss (device tensor)."""
    Ei, e = mlp(ctx, net, batch.G)
    Fp = forces(ctx, box, net, batch.pos, batch.nl, e)
    L, gE, lam = loss(ctx, Ei, Fp, batch.E_ref, batch.F_ref, batch.n, lam_F)
    ebar = pair_adjoint(ctx, box, net, batch.pos, batch.nl, lam)
    grad = mlp_grad(ctx, net, batch.G, batch.n, gE, ebar)
    net.adam(ctx, grad, lr)
    return L


def evaluate(ctx, box, net, batches):
    """Force RMSE (per component) and energy-per-atom RMSE of the network over batches."""
    se_f, nf, se_e, ne = 0.0, 0, 0.0, 0
    for b in batches:
        Ei, e = mlp(ctx, net, b.G)
        Fp = forces(ctx, box, net, b.pos, b.nl, e)
        d = (Fp - b.F_ref).double()
        se_f += float((d * d).sum())
        nf += d.numel()
        Es = Ei.double().reshape(-1, b.n).sum(dim=1)
        de = (Es - b.E_ref) / b.n
        se_e += float((de * de).sum())
        ne += de.numel()
    return math.sqrt(se_f / nf), math.sqrt(se_e / ne)


# ------------------------------------------------------------------ molecular dynamics with the network

class NNMD:
    """NVE with network forces (velocity Verlet, Sec. 3.3.1) and plain LJ as fallback and judge.

    One step: md_kick_drift -> nl_update (rebuilds on the device only when a particle moved > skin/2) ->
    descriptors -> MLP -> network forces -> md_kick.  `chunk` steps are captured once in a HIP graph and
    replayed.  Every `check_every` steps the LJ forces of the current configuration judge the network:
    if their RMSE exceeds `max_rmse` the run continues with plain LJ (md.nve) from that state."""

    def __init__(self, ctx: md.Context, net: Network, box: md.Box, u, v, dt=0.005, skin=0.3, r_cut=2.5,
                 max_rmse=1e-2, check_every=100, chunk=20, r_min=0.8):
        self.ctx, self.net, self.box, self.dt = ctx, net, box, dt
        self.lj = md.Potential("lj", [[1.0]], [[1.0]], r_cut=r_cut)
        self.sys = md.System(box, self.lj, u, v, skin=skin, ctx=ctx)
        self.sys.build()
        self.max_rmse, self.check_every, self.chunk, self.r_min = max_rmse, check_every, chunk, r_min
        self.min_r_log = []
        self.fallback = False
        self.rmse_log = []
        self.steps = 0
        self._graph = None
        self._lj = None
        self.G = torch.zeros((self.sys.N, K), dtype=torch.float32, device=ctx.device)
        self.Ei = torch.zeros(self.sys.N, dtype=torch.float32, device=ctx.device)
        self.e = torch.zeros((self.sys.N, K), dtype=torch.float32, device=ctx.device)
        self.F_lj = torch.zeros_like(self.sys.force)
        self._bind()
        self.forces()

    def _bind(self):
        """ctypes arguments built once (the tensors behind them stay put)."""
        lib = md.load()
        s = self.sys
        self._b, self._q, self._n = s.box.c(), self.net.c(), s.nl.c()
        B, Q, Nl = ctypes.byref(self._b), ctypes.byref(self._q), ctypes.byref(self._n)
        N, st = s.N, md._stream
        P = md._ptr
        self._calls_force = [
            lambda: lib.nn_descriptors(self.ctx.h, B, Q, P(s.pos), N, Nl, P(self.G), st()),
            lambda: lib.nn_mlp(self.ctx.h, Q, P(self.G), N, P(self.Ei), P(self.e), st()),
            lambda: lib.nn_forces(self.ctx.h, B, Q, P(s.pos), N, Nl, P(self.e), P(s.force), st()),
        ]
        dt = ctypes.c_float(self.dt)
        half = ctypes.c_float(0.5 * self.dt)
        self._calls_step = [
            lambda: lib.md_kick_drift(self.ctx.h, B, P(s.pos), P(s.vel), P(s.force), N, Nl, dt, st()),
            lambda: lib.nl_update(self.ctx.h, B, P(s.pos), N, Nl, st()),
        ] + self._calls_force + [lambda: lib.md_kick(self.ctx.h, P(s.vel), P(s.force), N, 3, half, st())]

    def _run(self, calls):
        for c in calls:
            r = c()
            if r != 0:
                raise RuntimeError(f"neural-potential MD call failed with status {r}")

    def forces(self):
        self._run(self._calls_force)

    def _eager(self, n):
        for _ in range(n):
            self._run(self._calls_step)

    def _replay(self, n):
        if self._graph is None:
            self._eager(1)  # one ordinary step before capture
            n -= 1
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):  # records the launches; nothing runs until a replay
                self._eager(self.chunk)
            self._graph = g
        while n >= self.chunk:
            self._graph.replay()
            n -= self.chunk
        if n > 0:
            self._eager(n)

    def judge(self) -> float:
        """Force RMSE of the network against plain LJ at the current configuration (reads the device)."""
        s = self.sys
        md.pair_energy_force(self.ctx, self.box, self.lj, s.pos, None, s.nl, self.F_lj)
        return float(md.rms_diff(self.ctx, s.force, self.F_lj))

    def min_distance(self) -> float:
        """Closest pair distance now; below r_min the configuration has left the descriptors' training range."""
        return float(md.min_distance(self.ctx, self.box, self.sys.pos, self.sys.nl))

    def run(self, n_steps: int, graph: bool = True):
        """Advance n_steps; returns the number of steps run with the network before any fallback."""
        done_nn = 0
        while n_steps > 0 and not self.fallback:
            k = min(n_steps, self.check_every)
            (self._replay if graph else self._eager)(k)
            f = self.sys.nl.read_flags()
            if f[md.FLAG_OVERFLOW] or f[md.FLAG_CELL_OVERFLOW]:
                raise RuntimeError(f"neighbor list overflow during network MD: {f.tolist()}")
            rmse = self.judge()
            rmin = self.min_distance()
            self.rmse_log.append(rmse)
            self.min_r_log.append(rmin)
            n_steps -= k
            done_nn += k
            self.steps += k
            if not math.isfinite(rmse) or rmse > self.max_rmse or rmin < self.r_min:
                self.fallback = True
        if n_steps > 0:
            # plain LJ takes over from the current positions and velocities
            s = self.sys
            init, update = md.nve(s, self.dt)
            init()
            update(n_steps)
            self.steps += n_steps
        return done_nn


def train_network(ctx: md.Context, n_runs=20, per_run=100, steps=20000, per_batch=16, lr=3e-3, lr_end=3e-5,
                  lam_F=1.0, seed=1, progress=None, eta=0.0, data=None):
    """The learned part end to end: plain-engine LJ data (n_runs x per_run snapshots of N = 4000), 10% held out,
    descriptor scale from the training set, `steps` Adam steps on minibatches of `per_batch` snapshots with an
    exponential learning-rate decay from lr to lr_end.  Returns the network, the held-out batches and a record
    (force / energy RMSE of the untrained and trained network on the held-out set, timings)."""
    import time
    t0 = time.perf_counter()
    box, P, E, F, T = data if data is not None else generate_lj_data(ctx, n_runs=n_runs, per_run=per_run,
                                                                      progress=progress)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    S = P.shape[0]
    perm = np.random.default_rng(seed).permutation(S)
    ntest = max(1, S // 10)
    test_idx, train_idx = perm[:ntest], perm[ntest:]
    w = inputs.nn_init(seed)
    probe = Network(ctx, w, np.zeros(K), np.ones(K), eta=eta)
    G = torch.cat([b.G for b in make_batches(ctx, box, probe, P, E, F, train_idx, per_batch)])
    m, s = descriptor_scale(ctx, G)
    del G
    net = Network(ctx, w, m, s, eta=eta)
    train = make_batches(ctx, box, net, P, E, F, train_idx, per_batch)
    test = make_batches(ctx, box, net, P, E, F, test_idx, per_batch)
    f0, e0 = evaluate(ctx, box, net, test)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    decay = (lr_end / lr) ** (1.0 / max(steps - 1, 1))
    order = np.random.default_rng(seed + 1)
    for k in range(steps):
        if k % len(train) == 0:
            sched = order.permutation(len(train))
        L = train_step(ctx, box, net, train[sched[k % len(train)]], lr * decay ** k, lam_F)
        if progress and (k % 5000 == 0 or k == steps - 1):
            progress(f"step {k} loss {float(L):.4g}")
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    f1, e1 = evaluate(ctx, box, net, test)
    eta_used = eta if eta > 0 else 1.0 / (2.0 * ((net.mu1 - net.mu0) / (K - 1)) ** 2)
    rec = dict(eta=eta_used, snapshots=int(S), atoms_per_snapshot=int(P.shape[1]), test_snapshots=int(ntest), steps=steps,
               per_batch=per_batch, force_rmse_untrained=f0, energy_rmse_untrained=e0, force_rmse=f1,
               energy_rmse_per_atom=e1, data_s=t_data, train_s=t_train, train_ms_per_step=1e3 * t_train / steps,
               force_rms_reference=float(F.pow(2).mean().sqrt()))
    return net, box, test, rec
