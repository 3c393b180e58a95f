"""Training and evaluation of the learned initialiser (efunc_initnet).

The paper fits every shape from the same starting point (scales e^7, zero
values, mean-shift offsets; Sec. 3.3, Sec. 4.3).  Here a convolution network
maps the coarse signed-distance field sampled at the lattice vertices to a
full parameter tensor.  It is trained end to end on the fitting loss: theta =
net(sdf), then efunc_loss_grad gives dL/dtheta of the shape's MSE on its
sample points, the network backward gives dL/dparams, AdamW updates.  All
arithmetic runs in the library (network, starting parameters, loss,
gradients, optimiser); torch holds the buffers and draws the minibatches.

The initialisations are compared by fitting held-out shapes from each with
the batched fit step (fresh points every step, cycled from a pool):
  paper   rho = 7, values 0, Delta by one mean-shift step (16,384 surface samples)
  sdf     the paper's, with o = coarse SDF, d = d' = its central-difference gradient
          at the vertices and o' = o + Delta . d (a strong hand-made baseline)
  newton  from the coarse SDF alone: the same values, the moved keys one Newton
          step towards the zero set (newton_theta)
  learned newton + net(coarse SDF), the network trained on the fitting loss
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import efunc as E

CHANNELS = [1, 32, 64, 64, 13]
RHO = [4, 12]      # log-scale channels of the parameter tensor
RHO_MIN = 7.0      # the paper's initial log-scale: the network may narrow a kernel, never widen it


def lattice(R: int) -> np.ndarray:
    return (-1.0 + 2.0 * np.arange(R) / (R - 1)).astype(np.float32).astype(np.float64)


def coarse_sdf(target_fn, R: int, device) -> torch.Tensor:
    """The shape's signed distance at the R^3 lattice vertices, [R^3] float32."""
    t = lattice(R)
    g = np.stack(np.meshgrid(t, t, t, indexing="ij"), axis=-1).reshape(-1, 3)
    return target_fn(torch.as_tensor(g, device=device)).to(torch.float32).contiguous()


def sdf_gradient(sdf: torch.Tensor, R: int) -> torch.Tensor:
    """Central differences of the lattice SDF (one-sided at the faces): [R^3, 3]
    (library kernel efunc_initnet_theta)."""
    return E.efunc_initnet_theta(sdf, R, theta=False, grad=True)[2].reshape(R ** 3, 3)


def newton_theta(sdf: torch.Tensor, R: int, rho0: float = 7.0) -> torch.Tensor:
    """A parameter tensor from the coarse SDF alone, [R^3, 13]: o = sdf and
    d = its central-difference gradient at each vertex; the moved key takes
    one Newton step towards the zero set, Delta = -sdf d / |d|^2 (its length
    capped at one lattice spacing), with o' = o + Delta . d and d' = d; both
    log-scales rho0 (library kernel efunc_initnet_theta)."""
    return E.efunc_initnet_theta(sdf, R, rho0=rho0)[0].reshape(R ** 3, 13)


def initial_params(seed: int) -> np.ndarray:
    """He-initialised weights, zero biases, the last layer small: an untrained
    network adds a small residual to the base parameters (newton_theta)."""
    rng = np.random.default_rng(seed)
    parts = []
    L = len(CHANNELS) - 1
    for l, (ci, co) in enumerate(zip(CHANNELS[:-1], CHANNELS[1:])):
        std = np.sqrt(2.0 / (27 * ci)) * (0.1 if l == L - 1 else 1.0)
        parts.append(rng.standard_normal(co * 27 * ci) * std)
        parts.append(np.zeros(co))
    return np.concatenate(parts).astype(np.float32)


def compose_theta(sdf: torch.Tensor, R: int, res: torch.Tensor, rho_min: float = RHO_MIN):
    """newton_theta(sdf) + res for B shapes (sdf [B, R^3], res [B, R^3, 13]),
    both log-scales floored at rho_min; returns (theta [B, R^3, 13], mask
    [B, R^3, 2] of the floored entries, whose gradient is zero).

    A smaller log-scale widens a radial basis function, and with it the window
    of keys every query must visit: the cost of a fitting step grows with the
    cube of the reach.  Trained end to end without a floor, the network lowers
    the scales and makes the fit several times slower per step."""
    th, mask, _ = E.efunc_initnet_theta(sdf, R, res=res.contiguous(), rho0=7.0, rho_min=rho_min, mask=True)
    return th, mask


def learned_theta(net: "E.InitNet", params, sdf) -> torch.Tensor:
    """The learned initialisation of one shape (flat [R^3 x 13]):
    newton_theta(sdf) plus the network's residual, log-scales floored."""
    res = net.forward(params, sdf[None]).reshape(1, -1, CHANNELS[-1])
    return compose_theta(sdf, net.R, res)[0].reshape(-1).contiguous()


def train(net: "E.InitNet", params: torch.Tensor, shapes, steps: int, batch: int, lr: float, seed: int,
          log=None):
    """End-to-end training of the residual: theta = newton_theta(sdf) +
    net(sdf).  shapes is a list of (sdf [R^3], [q [J,3]], [o [J]]) device
    tensors of one lattice size, with one or more point sets per shape (a
    random one each time the shape is drawn).  Returns the mean fitting loss
    per logged step."""
    R = net.R
    J = max(int(q.shape[0]) for s in shapes for q in s[1])
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
            res = net.forward(params, sdf).reshape(batch, -1, CHANNELS[-1])
            theta, mask = compose_theta(sdf, R, res)
            dtheta = torch.zeros_like(theta)
            for b, i in enumerate(idx):
                _, qsets, osets = shapes[i]
                k = int(rng.integers(len(qsets)))
                eng.loss_grad(theta[b].reshape(-1), qsets[k], osets[k], dtheta[b].reshape(-1), loss[b])
            E.efunc_initnet_theta_backward(mask, R, dtheta)
            net.backward(dtheta.reshape(res.shape[0], -1, CHANNELS[-1]), g)
            E.efunc_adam_update(params, m, v, g, step, adam)
            if step % 100 == 0 or step == 1:
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
    """The paper's initialisation with the values filled from the coarse SDF:
    o = sdf and d = its central-difference gradient at the vertex; the moved
    key sits at k + Delta, so o' = o + Delta . d (first order) and d' = d."""
    th = paper_theta(R, surf, device).view(R ** 3, 13)
    gr = sdf_gradient(sdf, R)
    th[:, 0] = sdf
    th[:, 1:4] = gr
    th[:, 8] = sdf + (th[:, 5:8] * gr).sum(dim=1)
    th[:, 9:12] = gr
    return th.reshape(-1).contiguous()


def heldout_l1(eng: "E.Engine", theta, qh, oh):
    """(L1, volume L1, near-surface L1) of theta on a held-out point set whose
    first half is uniform in the box and second half near the surface."""
    O = eng.eval(theta, qh, with_lse=False)[0]
    err = (O.double() - oh.double()).abs()
    h = qh.shape[0] // 2
    return float(err.mean()), float(err[:h].mean()), float(err[h:].mean())


def next_checkpoint(done: int) -> int:
    """Scoring schedule of fit_curves: every 10 steps up to 200, then every 50."""
    return done + (10 if done < 200 else 50)


def fit_curves(Rs, thetas, qpool, opool, steps: int, heldout, log=None):
    """Batched fits of all shapes from the given parameters.  qpool [P][S][J][3]
    and opool [P][S][J] hold P point sets per shape; step t trains on set
    (t - 1) mod P, copied into the bound buffers before the step (one device
    copy; the captured iteration is replayed unchanged).  Before the first
    step and at every checkpoint of next_checkpoint each shape's parameters
    are scored on its held-out points.  Returns (checkpoints, fit seconds): checkpoints = [(step, L1 [S],
    volume L1 [S], near L1 [S], L1 on the last step's points [S])]; the fit
    seconds include the point copies and exclude the scoring."""
    n = len(thetas)
    P = qpool.shape[0]
    th = [t.clone() for t in thetas]
    ms = [torch.zeros_like(t) for t in th]
    vs = [torch.zeros_like(t) for t in th]
    dev = th[0].device
    Q = qpool[0].clone()
    Ob = opool[0].clone()
    qs = [Q[i] for i in range(n)]
    os_ = [Ob[i] for i in range(n)]
    loss = torch.zeros(n, 2, device=dev, dtype=torch.float64)
    Jh = max(int(q.shape[0]) for q, _ in heldout)
    engs = {R: E.Engine(R, Jh) for R in set(Rs)}
    curve = []
    fit_s = 0.0

    def score(step):
        res = [heldout_l1(engs[Rs[i]], th[i], *heldout[i]) for i in range(n)]
        a = np.array(res)
        curve.append((step, a[:, 0], a[:, 1], a[:, 2], loss[:, 1].cpu().numpy().copy()))

    with E.BatchEngine(Rs, [int(q.shape[0]) for q in qs]) as B:
        B.bind(th, ms, vs, qs, os_, loss)
        done = 0
        score(0)
        while done < steps:
            k = min(next_checkpoint(done), steps) - done
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for t in range(done + 1, done + k + 1):
                Q.copy_(qpool[(t - 1) % P])
                Ob.copy_(opool[(t - 1) % P])
                B.fit(t, 1, use_graph=True)
            torch.cuda.synchronize()
            fit_s += time.perf_counter() - t0
            done += k
            score(done)
            if log and (done % 250 == 0 or done == 10):
                log(f"fit step {done}: mean held-out L1 {float(curve[-1][1].mean()):.5f}, "
                    f"{fit_s / done * 1e3:.2f} ms per batched step")
    for e in engs.values():
        e.close()
    return curve, fit_s


def choose_init(R, learned, fallback, q, o):
    """The learned parameters unless the fitting loss (mean squared error on
    the shape's own training points) of the fallback is lower."""
    with E.Engine(R, int(q.shape[0])) as eng:
        ls = []
        for th in (learned, fallback):
            O = eng.eval(th, q, with_lse=False)[0]
            ls.append(float(((O.double() - o.double()) ** 2).mean()))
    return (learned, False) if ls[0] <= ls[1] else (fallback, True)


def steps_to(curve, thr: float):
    """First checkpoint step at which each shape's held-out L1 <= thr (None if never)."""
    n = len(curve[0][1])
    out = [None] * n
    for step, l1, *_ in curve:
        for i in range(n):
            if out[i] is None and l1[i] <= thr:
                out[i] = step
    return out
