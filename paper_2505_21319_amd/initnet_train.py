"""Training and evaluation of the learned initialiser (efunc_initnet).

The paper fits every shape from the same starting point (scales e^7, zero
values, mean-shift offsets; Sec. 3.3, Sec. 4.3).  Here a convolution network
maps the coarse signed-distance field sampled at the lattice vertices to a
full parameter tensor.  It is trained end to end on the fitting loss: theta =
net(sdf), then efunc_loss_grad gives dL/dtheta of the shape's MSE on its
sample points, the network backward gives dL/dparams, AdamW updates.  All
arithmetic runs in the library (network, loss, gradients, optimiser); torch
holds the buffers.

Three initialisations are compared by fitting held-out shapes from each with
the batched fit step:
  paper   rho = 7, values 0, Delta by one mean-shift step (16,384 surface samples)
  sdf     the paper's, plus o = o' = coarse SDF and d = d' = its central-difference
          gradient at the vertices (a strong hand-made baseline)
  learned net(coarse SDF)
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import efunc as E

CHANNELS = [1, 32, 64, 64, 13]


def lattice(R: int) -> np.ndarray:
    return (-1.0 + 2.0 * np.arange(R) / (R - 1)).astype(np.float32).astype(np.float64)


def coarse_sdf(target_fn, R: int, device) -> torch.Tensor:
    """The shape's signed distance at the R^3 lattice vertices, [R^3] float32."""
    t = lattice(R)
    g = np.stack(np.meshgrid(t, t, t, indexing="ij"), axis=-1).reshape(-1, 3)
    return target_fn(torch.as_tensor(g, device=device)).to(torch.float32).contiguous()


def sdf_gradient(sdf: torch.Tensor, R: int) -> torch.Tensor:
    """Central differences of the lattice SDF (one-sided at the faces): [R^3, 3]."""
    h = 2.0 / (R - 1)
    s = sdf.view(R, R, R)
    out = []
    for ax in range(3):
        d = torch.empty_like(s)
        sl = [slice(None)] * 3
        lo, hi, mid = list(sl), list(sl), list(sl)
        mid[ax] = slice(1, -1)
        hi[ax] = slice(2, None)
        lo[ax] = slice(0, -2)
        d[tuple(mid)] = (s[tuple(hi)] - s[tuple(lo)]) / (2 * h)
        a, b = list(sl), list(sl)
        a[ax], b[ax] = 0, 1
        d[tuple(a)] = (s[tuple(b)] - s[tuple(a)]) / h
        a[ax], b[ax] = -1, -2
        d[tuple(a)] = (s[tuple(a)] - s[tuple(b)]) / h
        out.append(d.reshape(-1))
    return torch.stack(out, dim=1)


def initial_params(seed: int, rho0: float = 7.0) -> np.ndarray:
    """He-initialised weights, zero biases, the last layer small with the scale
    channels' bias at rho0 (so that an untrained network starts near the
    paper's initialisation)."""
    rng = np.random.default_rng(seed)
    parts = []
    L = len(CHANNELS) - 1
    for l, (ci, co) in enumerate(zip(CHANNELS[:-1], CHANNELS[1:])):
        std = np.sqrt(2.0 / (27 * ci)) * (0.1 if l == L - 1 else 1.0)
        parts.append(rng.standard_normal(co * 27 * ci) * std)
        b = np.zeros(co)
        if l == L - 1:
            b[4] = rho0
            b[12] = rho0
        parts.append(b)
    return np.concatenate(parts).astype(np.float32)


def train(net: "E.InitNet", params: torch.Tensor, shapes, steps: int, batch: int, lr: float, seed: int,
          log=None):
    """End-to-end training: shapes is a list of (sdf [R^3], q [J,3], o [J]) device tensors of
    one lattice size.  Returns the mean fitting loss per step."""
    R = net.R
    J = max(int(s[1].shape[0]) for s in shapes)
    rng = np.random.default_rng(seed)
    m, v, g = (torch.zeros_like(params) for _ in range(3))
    adam = E.efunc_default_adam()
    adam.lr = lr
    losses = []
    dev = params.device
    loss = torch.zeros(batch, 2, device=dev, dtype=torch.float64)
    with E.Engine(R, J) as eng:
        for step in range(1, steps + 1):
            idx = rng.choice(len(shapes), batch, replace=False)
            sdf = torch.stack([shapes[i][0] for i in idx])
            theta = net.forward(params, sdf)
            dtheta = torch.zeros_like(theta)
            for b, i in enumerate(idx):
                _, q, o = shapes[i]
                eng.loss_grad(theta[b], q, o, dtheta[b], loss[b])
            net.backward(dtheta, g)
            E.efunc_adam_update(params, m, v, g, step, adam)
            if step % 25 == 0 or step == 1:
                lv = float(loss[:, 0].mean())
                losses.append((step, lv))
                if log:
                    log(f"train step {step}: mean loss {lv:.5f}")
    return losses


def paper_theta(R, surf, device):
    """The paper's initialisation through the library (mean-shift offsets)."""
    th = torch.empty(R ** 3 * 13, device=device)
    with E.Engine(R, 16) as e1:
        e1.init_params(th, surf, 100.0, 7.0)
    return th


def sdf_theta(R, sdf, surf, device):
    th = paper_theta(R, surf, device).view(R ** 3, 13)
    gr = sdf_gradient(sdf, R)
    th[:, 0] = sdf
    th[:, 1:4] = gr
    th[:, 8] = sdf
    th[:, 9:12] = gr
    return th.reshape(-1).contiguous()


def fit_curves(Rs, thetas, qs, os_, steps: int, every: int):
    """Batched fits of all shapes from the given parameters; per-shape L1
    (mean |O - o|) before step 1, every `every` steps and after the last."""
    n = len(thetas)
    th = [t.clone() for t in thetas]
    ms = [torch.zeros_like(t) for t in th]
    vs = [torch.zeros_like(t) for t in th]
    dev = th[0].device
    loss = torch.zeros(n, 2, device=dev, dtype=torch.float64)
    curve = []
    t0 = time.perf_counter()
    with E.BatchEngine(Rs, [int(q.shape[0]) for q in qs]) as B:
        B.bind(th, ms, vs, qs, os_, loss)
        done = 0
        while done < steps:
            k = min(every, steps - done)
            B.fit(done + 1, 1, use_graph=False)
            curve.append((done, loss[:, 1].cpu().numpy().copy()))  # L1 of the parameters before step done+1
            if k > 1:
                B.fit(done + 2, k - 1, use_graph=True)
            done += k
        # L1 of the final parameters (the loss of one more step, before its update)
        B.fit(done + 1, 1, use_graph=False)
        curve.append((done, loss[:, 1].cpu().numpy().copy()))
        torch.cuda.synchronize()
    return curve, time.perf_counter() - t0


def steps_to(curve, thr: float):
    """First recorded step at which each shape's L1 <= thr (None if never)."""
    n = len(curve[0][1])
    out = [None] * n
    for step, l1 in curve:
        for i in range(n):
            if out[i] is None and l1[i] <= thr:
                out[i] = step
    return out
