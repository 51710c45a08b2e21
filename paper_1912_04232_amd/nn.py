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

    def __init__(self, ctx: md.Context, weights: dict, m, s, mu0=0.8, mu1=2.5, r_c=2.5):
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
        self.m = torch.as_tensor(np.asarray(m, np.float32), device=dev).contiguous()
        self.s = torch.as_tensor(np.asarray(s, np.float32), device=dev).contiguous()
        self.mu0, self.mu1, self.r_c = float(mu0), float(mu1), float(r_c)
        self.step = 0
        md._check("nn_cast_weights", md.load().nn_cast_weights(ctx.h, md._ptr(self.theta),
                                                                 md._ptr(self.W1), md._ptr(self.W2), md._stream()))

    def c(self) -> md.c_nn_params:
        q = md.c_nn_params()
        q.K, q.H, q.mu0, q.mu1, q.r_c = K, H, self.mu0, self.mu1, self.r_c
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


def descriptor_scale(G: torch.Tensor):
    """Per-basis mean and standard deviation of the training descriptors (host numpy, set-up only)."""
    g = G.cpu().numpy().astype(np.float64)
    m = g.mean(axis=0)
    s = g.std(axis=0)
    return m, np.where(s > 1e-8, s, 1.0)


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
