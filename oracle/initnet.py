"""FP64 CPU oracle of the learned initialiser network -- TEST INFRASTRUCTURE ONLY.

The paper fits every shape from a fixed initialisation (Sec. 3.3, Sec. 4.3)
and leaves generative or learned initialisation to future work (Sec. 5).
The network here maps a coarse signed-distance field sampled at the R^3
lattice vertices to the R^3 x 13 parameter tensor: L layers of 3x3x3
convolutions with zero padding (stride 1), ReLU between layers, none after
the last.

Storage (shared layout, not shared code): activations channels-last
[B][R][R][R][C]; layer l has weights W_l[co][tap][ci] (tap = (dz*3 + dy)*3 +
dx over offsets -1..1, z outermost) followed by the bias b_l[co], all layers
concatenated in one flat parameter vector.

Mixed precision of the GPU path, reproduced exactly here: weights and every
layer input are rounded to bfloat16 (round to nearest even) before the
layer, products are accumulated in double (the GPU accumulates in float32,
the tolerance covers the difference), the bias is added in the accumulator
precision.  The backward rounds the incoming gradient of every layer output
to bfloat16 as well.

The convolution itself is torch.nn.functional.conv3d in float64 on the CPU (a
library primitive, pinned against direct loops in the tests).
"""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as F


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round float64/float32 values to bfloat16 (nearest even), returned as float64."""
    x = np.asarray(a, dtype=np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isfinite(x), out, x.astype(np.float64))


# Rounding applied at the GPU's bf16 points; the pins replace it by the
# identity to check the exact-arithmetic gradient against finite differences.
ROUND = bf16_round


def layer_shapes(channels):
    """(W shape [co][27][ci], bias length) per layer."""
    return [((channels[i + 1], 27, channels[i]), channels[i + 1]) for i in range(len(channels) - 1)]


def num_params(channels) -> int:
    return sum(co * 27 * ci + co for (co, _, ci), _ in layer_shapes(channels))


def unpack(params, channels):
    """Flat parameters -> list of (W [co][27][ci], b [co]) as float64."""
    p = np.asarray(params, dtype=np.float64)
    out, o = [], 0
    for (co, t, ci), nb in layer_shapes(channels):
        w = p[o:o + co * t * ci].reshape(co, t, ci)
        o += co * t * ci
        b = p[o:o + nb]
        o += nb
        out.append((w, b))
    assert o == p.size
    return out


def _conv(x, w):
    """x [B][D][D][D][ci], w [co][27][ci] -> [B][D][D][D][co] (cross-correlation,
    zero padding 1)."""
    co, _, ci = w.shape
    X = torch.from_numpy(np.ascontiguousarray(np.moveaxis(x, -1, 1)))
    K = torch.from_numpy(np.ascontiguousarray(w.reshape(co, 3, 3, 3, ci).transpose(0, 4, 1, 2, 3)))
    Y = F.conv3d(X, K, padding=1)
    return np.moveaxis(Y.numpy(), 1, -1)


def layer_forward(x_in, w, b, relu: bool):
    """One layer as the GPU computes it: bf16 input and weights, exact
    products, bias; returns (pre-activation, activation)."""
    z = _conv(ROUND(x_in), ROUND(w)) + b
    a = np.maximum(z, 0.0) if relu else z
    return z, a


def forward(params, channels, x):
    """Network output and the list of layer inputs (for the backward)."""
    layers = unpack(params, channels)
    h = np.asarray(x, dtype=np.float64)
    inputs = []
    for i, (w, b) in enumerate(layers):
        inputs.append(h)
        _, h = layer_forward(h, w, b, relu=i < len(layers) - 1)
    return h, inputs


def layer_backward(x_in, w, dz):
    """Gradients of one layer given dL/d(pre-activation) dz: (dL/dW, dL/db,
    dL/dx_in), with the GPU's bf16 rounding of dz, x_in and w."""
    Xb = torch.from_numpy(np.ascontiguousarray(np.moveaxis(ROUND(x_in), -1, 1))).requires_grad_(True)
    co, _, ci = w.shape
    Kb = torch.from_numpy(np.ascontiguousarray(
        ROUND(w).reshape(co, 3, 3, 3, ci).transpose(0, 4, 1, 2, 3))).requires_grad_(True)
    Y = F.conv3d(Xb, Kb, padding=1)
    G = torch.from_numpy(np.ascontiguousarray(np.moveaxis(ROUND(dz), -1, 1)))
    Y.backward(G)
    dW = Kb.grad.numpy().transpose(0, 2, 3, 4, 1).reshape(co, 27, ci)
    db = ROUND(dz).reshape(-1, co).sum(axis=0)
    dx = np.moveaxis(Xb.grad.numpy(), 1, -1)
    return dW, db, dx


def backward(params, channels, x, dout):
    """dL/dparams (flat) for the output gradient dout, recomputing the forward."""
    layers = unpack(params, channels)
    out, inputs = forward(params, channels, x)
    grads = []
    g = np.asarray(dout, dtype=np.float64)
    for i in range(len(layers) - 1, -1, -1):
        w, _ = layers[i]
        dW, db, dx = layer_backward(inputs[i], w, g)
        grads.append((dW, db))
        if i > 0:
            g = dx * (inputs[i] > 0)  # ReLU of the previous layer
    flat = []
    for dW, db in reversed(grads):
        flat.append(dW.reshape(-1))
        flat.append(db)
    return np.concatenate(flat)


def base_theta(sdf, R: int, rho0: float = 7.0, res=None, rho_min: float = -np.inf):
    """Starting parameters of the learned initialiser from coarse fields sdf
    [B][R^3] (float32 values at the lattice vertices), in float64: returns
    (theta [B][R^3][13], mask [B][R^3][2] of floored log-scales, grad
    [B][R^3][3]).  The definition, written out: g = central differences of
    sdf with spacing h = 2 / (R - 1), one-sided on the faces; o = sdf, d = g,
    rho = rho0; Delta = -sdf g / max(|g|^2, 1e-12), scaled down to length h
    if longer (one Newton step towards the zero set); o' = o + Delta . g,
    d' = g, rho' = rho0; then theta + res, both log-scales floored at
    rho_min."""
    s = np.asarray(sdf, dtype=np.float32).astype(np.float64).reshape(-1, R, R, R)
    B = s.shape[0]
    h = 2.0 / (R - 1)
    g = np.empty(s.shape + (3,))
    for ax in range(3):
        a = np.moveaxis(s, ax + 1, 1)
        d = np.empty_like(a)
        d[:, 1:-1] = (a[:, 2:] - a[:, :-2]) / (2.0 * h)
        d[:, 0] = (a[:, 1] - a[:, 0]) / h
        d[:, -1] = (a[:, -1] - a[:, -2]) / h
        g[..., ax] = np.moveaxis(d, 1, ax + 1)
    s = s.reshape(B, -1)
    g = g.reshape(B, -1, 3)
    gn2 = np.maximum((g * g).sum(-1), 1e-12)
    delta = -(s / gn2)[..., None] * g
    ln = np.linalg.norm(delta, axis=-1)
    delta = delta * np.minimum(h / np.maximum(ln, 1e-30), 1.0)[..., None]
    th = np.empty((B, s.shape[1], 13))
    th[..., 0] = s
    th[..., 1:4] = g
    th[..., 4] = rho0
    th[..., 5:8] = delta
    th[..., 8] = s + (delta * g).sum(-1)
    th[..., 9:12] = g
    th[..., 12] = rho0
    if res is not None:
        r32 = np.asarray(res, dtype=np.float32).reshape(th.shape)
        th = th + r32.astype(np.float64)
        # the floor decides per entry: taken, as in the kernel, on the float32
        # sum rho0 + res (a residual below half an ulp of rho0 leaves it at rho0)
        for c in (4, 12):
            th[..., c] = (np.float32(rho0) + r32[..., c]).astype(np.float64)
    mask = np.stack([th[..., 4] < rho_min, th[..., 12] < rho_min], axis=-1)
    th[..., 4] = np.maximum(th[..., 4], rho_min)
    th[..., 12] = np.maximum(th[..., 12], rho_min)
    return th, mask, g
