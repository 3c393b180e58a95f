"""Pins for the FP64 oracle against facts the paper and mathematics fix.

Nothing here re-types an oracle formula and compares it with itself: each
test checks a closed form, an invariant, a special case computed by an
independent library routine, finite differences of the oracle's own
evaluation, or a count printed in the paper.
"""
import json
import os

import numpy as np
import pytest
import scipy.special as sps
import scipy.stats as sst
from scipy.spatial import cKDTree

import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def rand_q(rng, J, lo=-1.0, hi=1.0):
    return rng.uniform(lo, hi, size=(J, 3))


# ---------------------------------------------------------------- layout pins
def test_param_counts_match_paper(orc):
    """Tab. main / Tab. ablation: R^3 x channels; the default model is 13 floats
    per vertex = 5 (grid key) + 8 (moved key)."""
    gold = json.load(open(os.path.join(GOLD, "paper_param_counts.json")))
    for e in gold["entries"]:
        assert e["R"] ** 3 * e["channels"] == e["params"], e["cite"]
    b = gold["channel_budget"]
    assert sum(v for k, v in b["grid_key"].items() if k != "cite") + \
        sum(v for k, v in b["moved_key"].items() if k != "cite") == orc.NCH == 13
    g = orc.Grid(R=4)
    assert orc.num_keys(g) == 2 * 4 ** 3
    assert orc.num_keys(orc.Grid(R=4, offsets=0)) == 4 ** 3


def test_every_channel_enters_the_model(orc):
    """Each of the 13 channels changes the output somewhere (no dead channel)."""
    rng = np.random.default_rng(0)
    g = orc.Grid(R=3)
    th = W.perturbed_theta(3, 5)
    q = rand_q(rng, 64)
    O0, _, _ = orc.eval_global(orc.build_keys(g, th), q)
    for ch in range(13):
        t2 = th.copy()
        t2[..., ch] += 0.05
        O1, _, _ = orc.eval_global(orc.build_keys(g, t2), q)
        assert np.abs(O1 - O0).max() > 1e-6, ch


def test_lattice_is_float32_rounded_uniform(orc):
    g = orc.Grid(R=7, lo=-1.0, hi=1.0)
    t = orc.lattice(g)
    ref = np.linspace(-1.0, 1.0, 7).astype(np.float32).astype(np.float64)
    assert np.array_equal(t, ref)


# ------------------------------------------------------ forward special cases
def test_one_key_returns_its_polynomial(orc):
    """A single key: softmax weight 1, so O = f(q - c) and lse = s."""
    rng = np.random.default_rng(1)
    key = np.array([[0.1, -0.2, 0.3, 50.0, 0.7, 1.5, -2.0, 0.25]])
    q = rand_q(rng, 20)
    O, lse, _ = orc.eval_global(key, q)
    x = q - key[0, :3]
    assert np.allclose(O, 0.7 + x @ key[0, 5:], rtol=0, atol=1e-14)
    assert np.allclose(lse, -50.0 * (x * x).sum(1), rtol=1e-14, atol=1e-14)


def test_two_keys_logistic_blend(orc):
    """Two keys: the softmax is the logistic function of the logit gap."""
    rng = np.random.default_rng(2)
    keys = np.array([[0.0, 0.0, 0.0, 30.0, 1.0, 0.5, 0.0, 0.0],
                     [0.4, 0.1, -0.2, 80.0, -1.0, 0.0, 2.0, -1.0]])
    q = rand_q(rng, 50, -0.5, 0.7)
    O, _, _ = orc.eval_global(keys, q)
    s = [-k[3] * ((q - k[:3]) ** 2).sum(1) for k in keys]
    f = [k[4] + (q - k[:3]) @ k[5:] for k in keys]
    w0 = sps.expit(s[0] - s[1])
    assert np.allclose(O, w0 * f[0] + (1 - w0) * f[1], rtol=1e-12, atol=1e-13)


def test_order0_fixed_grid_is_nadaraya_watson(orc):
    """f^0 on fixed grid keys with one common beta is Gaussian-kernel
    Nadaraya-Watson regression (Sec. 3.1): compare with the estimator built
    from scipy's multivariate normal density of covariance 1/(2 beta) I."""
    rng = np.random.default_rng(3)
    R, beta = 4, 9.0
    g = orc.Grid(R=R, offsets=0)
    th = np.zeros((R, R, R, 13), np.float32)
    th[..., 0] = rng.uniform(0.2, 2.0, size=(R, R, R))
    th[..., 4] = np.float32(np.log(beta))
    keys = orc.build_keys(g, th)
    beta_used = keys[0, 3]
    q = rand_q(rng, 40, -0.9, 0.9)
    O, _, _ = orc.eval_global(keys, q)
    v = keys[:, 4]
    cov = np.eye(3) / (2.0 * beta_used)
    K = np.stack([sst.multivariate_normal(mean=k, cov=cov).pdf(q) for k in keys[:, :3]], 1)
    nw = (K @ v) / K.sum(1)
    assert np.allclose(O, nw, rtol=1e-10, atol=1e-12)


def test_lse_separates_over_axes_on_the_lattice(orc):
    """Equal betas on the fixed lattice: sum over vertices of
    exp(-beta ||q - k||^2) factorises into three 1-D sums."""
    rng = np.random.default_rng(4)
    R = 5
    g = orc.Grid(R=R, offsets=0)
    th = W.plain_theta(R, rho0=2.5)
    keys = orc.build_keys(g, th)
    t = orc.lattice(g)
    beta = keys[0, 3]
    q = rand_q(rng, 30)
    _, lse, _ = orc.eval_global(keys, q)
    ref = sum(sps.logsumexp(-beta * (q[:, d:d + 1] - t[None, :]) ** 2, axis=1) for d in range(3))
    assert np.allclose(lse, ref, rtol=1e-13, atol=1e-12)


def test_large_beta_selects_nearest_key(orc):
    """beta -> infinity: the output is the polynomial of the nearest centre
    (found with a k-d tree)."""
    rng = np.random.default_rng(5)
    R = 4
    g = orc.Grid(R=R)
    th = W.perturbed_theta(R, 7, rho0=9.0, rho_spread=0.0, offset_cells=0.4)
    th[..., 4] = 11.0
    th[..., 12] = 11.0
    keys = orc.build_keys(g, th)
    q = rand_q(rng, 300, -0.95, 0.95)
    d, idx = cKDTree(keys[:, :3]).query(q, k=2)
    ok = (d[:, 1] ** 2 - d[:, 0] ** 2) > 0.02   # clear winner: gap x beta ~ 1200
    O, _, _ = orc.eval_global(keys, q)
    k = keys[idx[:, 0]]
    f = k[:, 4] + ((q - k[:, :3]) * k[:, 5:]).sum(1)
    assert ok.sum() > 100
    assert np.allclose(O[ok], f[ok], rtol=0, atol=1e-9)


def test_convexity_and_constant_reproduction(orc):
    """Softmax weights are a convex combination (Sec. 3.1): with f^0 the output
    lies within [min v, max v]; equal values are reproduced to rounding."""
    rng = np.random.default_rng(6)
    g = orc.Grid(R=3)
    th = W.perturbed_theta(3, 8)
    th[..., 1:4] = 0
    th[..., 9:12] = 0
    keys = orc.build_keys(g, th)
    q = rand_q(rng, 100)
    O, _, _ = orc.eval_global(keys, q)
    assert O.min() >= keys[:, 4].min() - 1e-12 and O.max() <= keys[:, 4].max() + 1e-12
    th[..., 0] = 0.375
    th[..., 8] = 0.375
    O, _, _ = orc.eval_global(orc.build_keys(g, th), q)
    assert np.allclose(O, 0.375, rtol=4e-16, atol=0)


def linear_theta(R, alpha, b, seed=0, lo=-1.0, hi=1.0):
    """Every key (grid and moved, any beta, any offset) carries the same
    linear function alpha + b.q written around its own centre."""
    rng = np.random.default_rng(seed)
    th = W.perturbed_theta(R, seed)
    t = np.linspace(lo, hi, R).astype(np.float32).astype(np.float64)
    K = np.stack(np.meshgrid(t, t, t, indexing="ij"), -1)
    C = K + th[..., 5:8].astype(np.float64)
    th = th.astype(np.float64)
    th[..., 0] = alpha + K @ b
    th[..., 1:4] = b
    th[..., 8] = alpha + C @ b
    th[..., 9:12] = b
    del rng
    return th.astype(np.float32)


def test_linear_field_reproduction(orc):
    """If every key carries alpha + b.(c + x) then f_a(q) = alpha + b.q for all a,
    so O(q) = alpha + b.q for any scales and offsets (Sec. 3.2 shift
    invariance + convexity); dO/dq = b (Eq. func-normal)."""
    rng = np.random.default_rng(7)
    R = 4
    g = orc.Grid(R=R)
    alpha, b = 0.3, np.array([0.5, -1.25, 2.0])
    th = linear_theta(R, alpha, b, seed=3)
    keys = orc.build_keys(g, th)
    # the float32 storage rounds alpha + b.c; compare against the stored values
    q = rand_q(rng, 200)
    O, _, sig = orc.eval_global(keys, q)
    assert np.allclose(O, alpha + q @ b, rtol=0, atol=2e-6 * sig.max())
    Ot, _, _ = orc.eval_trunc(g, keys, q, 20.0)
    assert np.allclose(Ot, alpha + q @ b, rtol=0, atol=2e-6 * sig.max())
    # exact double-precision values remove the float32 rounding of alpha + b.c
    keys[:, 4] = alpha + keys[:, :3] @ b
    dq = orc.eval_qgrad(keys, q)
    assert np.allclose(dq, b[None, :], rtol=0, atol=1e-12)


def test_shift_invariance(orc):
    """Translating lattice and queries together leaves O unchanged (f depends
    on q - k only, Sec. 3.2)."""
    rng = np.random.default_rng(8)
    th = W.perturbed_theta(5, 9)
    q = rand_q(rng, 50)
    # R = 5 on [-1, 1] and on [-0.75, 1.25]: both lattices are exact in float32
    O0, l0, _ = orc.eval_global(orc.build_keys(orc.Grid(R=5, lo=-1, hi=1), th), q)
    O1, l1, _ = orc.eval_global(orc.build_keys(orc.Grid(R=5, lo=-0.75, hi=1.25), th), q + 0.25)
    assert np.allclose(O0, O1, rtol=0, atol=1e-10)
    assert np.allclose(l0, l1, rtol=1e-12, atol=1e-9)


# ------------------------------------------------------------- query gradient
def test_query_gradient_matches_central_differences(orc):
    rng = np.random.default_rng(9)
    g = orc.Grid(R=3)
    keys = orc.build_keys(g, W.perturbed_theta(3, 10, rho0=2.0))
    q = rand_q(rng, 25, -0.8, 0.8)
    G = orc.eval_qgrad(keys, q)
    h = 1e-6
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        fd = (orc.eval_global(keys, q + e)[0] - orc.eval_global(keys, q - e)[0]) / (2 * h)
        assert np.allclose(G[:, d], fd, rtol=1e-6, atol=1e-7)


# ----------------------------------------------------------------- gradients
def _loss(orc, keys, q, dl):
    return float(dl @ orc.eval_global(keys, q)[0])


def test_key_gradients_match_central_differences(orc):
    """Sec. 3.6 closed forms (every entry of every key, both key kinds)
    against central differences of sum_j dL/dO_j O(q_j)."""
    rng = np.random.default_rng(11)
    g = orc.Grid(R=3)
    keys = orc.build_keys(g, W.perturbed_theta(3, 12, rho0=2.0, rho_spread=1.0))
    q = rand_q(rng, 40, -0.9, 0.9)
    dl = rng.standard_normal(40)
    gk, ak = orc.grad_global(keys, q, dl)
    # central-difference rounding noise: ~ eps * sum_j |dl_j O_j| / h
    Lmag = float(np.abs(dl) @ np.abs(orc.eval_global(keys, q)[0]))
    worst = 0.0
    for a in range(keys.shape[0]):
        for c in range(8):
            h = 1e-6 * max(1.0, abs(keys[a, c]))
            kp, km = keys.copy(), keys.copy()
            kp[a, c] += h
            km[a, c] -= h
            fd = (_loss(orc, kp, q, dl) - _loss(orc, km, q, dl)) / (2 * h)
            noise = 50 * np.finfo(float).eps * Lmag / h
            err = abs(fd - gk[a, c]) / (1e-6 * ak[a, c] + noise)
            worst = max(worst, err)
    assert worst < 1.0, worst


def _theta_loss(orc, g, th, q, dl):
    return _loss(orc, orc.build_keys(g, th), q, dl)


def test_theta_channel_gradients_match_central_differences(orc):
    """The 13-channel mapping (rho = ln beta chain rule, dL/dDelta = dL/dc,
    fixed grid centres) against Richardson-extrapolated central differences
    in the stored float32 parameters."""
    rng = np.random.default_rng(13)
    R = 3
    g = orc.Grid(R=R)
    th = W.perturbed_theta(R, 14, rho0=2.0, rho_spread=0.5)
    q = rand_q(rng, 40, -0.9, 0.9)
    dl = rng.standard_normal(40)
    keys = orc.build_keys(g, th)
    gk, ak = orc.grad_global(keys, q, dl)
    gt = orc.grad_theta(g, th, gk)
    at = orc.grad_theta(g, th, ak)
    for trial in range(40):
        i = tuple(rng.integers(0, R, size=3))
        ch = int(rng.integers(0, 13))

        def D(h):
            tp, tm = th.copy(), th.copy()
            tp[i + (ch,)] = np.float32(th[i + (ch,)] + h)
            tm[i + (ch,)] = np.float32(th[i + (ch,)] - h)
            span = float(tp[i + (ch,)]) - float(tm[i + (ch,)])
            return (_theta_loss(orc, g, tp, q, dl) - _theta_loss(orc, g, tm, q, dl)) / span

        h = 2.0 ** -8
        fd = (4 * D(h / 2) - D(h)) / 3
        scale = at[i + (ch,)] * (np.exp(th[i + (4,)]) if ch == 4 else 1.0) + 1e-6
        if ch == 12:
            scale = at[i + (ch,)] * np.exp(th[i + (12,)]) + 1e-6
        assert abs(fd - gt[i + (ch,)]) <= 2e-5 * scale + 1e-9, (i, ch, fd, gt[i + (ch,)])


def test_gradients_match_torch_autograd(orc):
    """The same gradients from torch autograd (FP64) through an independently
    written forward on a tiny problem."""
    import torch
    rng = np.random.default_rng(15)
    R = 2
    g = orc.Grid(R=R)
    th = W.perturbed_theta(R, 16, rho0=1.5)
    q = rand_q(rng, 30)
    dl = rng.standard_normal(30)
    gt = orc.grad_theta(g, th, orc.grad_global(orc.build_keys(g, th), q, dl)[0])

    T = torch.tensor(th.astype(np.float64), requires_grad=True)
    t = torch.tensor(orc.lattice(g))
    K = torch.stack(torch.meshgrid(t, t, t, indexing="ij"), -1).reshape(-1, 3)
    P = T.reshape(-1, 13)
    Q = torch.tensor(q)
    centres = torch.cat([K, K + P[:, 5:8]])
    betas = torch.cat([P[:, 4].exp(), P[:, 12].exp()])
    vals = torch.cat([P[:, 0], P[:, 8]])
    slopes = torch.cat([P[:, 1:4], P[:, 9:12]])
    X = Q[:, None, :] - centres[None]
    logits = -betas[None] * (X * X).sum(-1)
    F = vals[None] + (X * slopes[None]).sum(-1)
    O = (torch.softmax(logits, dim=1) * F).sum(1)
    (O * torch.tensor(dl)).sum().backward()
    ref = T.grad.numpy()
    ref[..., 5:8] = ref[..., 5:8]  # moved centres: dL/dDelta
    assert np.allclose(gt, ref, rtol=1e-9, atol=1e-11)


def test_linear_field_gradient_invariants(orc):
    """With a linear field, f_a - O = 0 for every pair, so dO/dbeta = 0 and
    dO/dc_a = -w_a b; summed: dL/dc_a = -b dL/do_a (Sec. 3.6)."""
    rng = np.random.default_rng(17)
    R = 3
    g = orc.Grid(R=R)
    b = np.array([0.25, -0.5, 1.0])
    keys = orc.build_keys(g, linear_theta(R, -0.1, b, seed=4))
    # rebuild values exactly in double so f_a - O vanishes to rounding
    keys[:, 4] = -0.1 + keys[:, :3] @ b
    keys[:, 5:] = b
    q = rand_q(rng, 50)
    dl = rng.standard_normal(50)
    gk, ak = orc.grad_global(keys, q, dl)
    assert np.abs(gk[:, 3]).max() <= 1e-12 * (1 + ak[:, 3].max())
    assert np.allclose(gk[:, 0:3], -gk[:, 4:5] * b[None], rtol=0, atol=1e-12)


# ----------------------------------------------------------------- truncation
def test_truncation_error_within_bound(orc):
    """Dropping only keys with s < M - T changes O by at most the dropped
    mass (<= nkeys e^-T) times 2 max |f|; large T recovers the global sum."""
    rng = np.random.default_rng(19)
    R = 6
    g = orc.Grid(R=R)
    th = W.perturbed_theta(R, 20, rho0=3.0, rho_spread=1.0, offset_cells=1.0)
    keys = orc.build_keys(g, th)
    q = rand_q(rng, 400)
    O, lse, sig = orc.eval_global(keys, q)
    fmax = np.abs(keys[:, 4]).max() + 4 * np.abs(keys[:, 5:]).max()
    for T in (6.0, 10.0):
        Ot, lt, _ = orc.eval_trunc(g, keys, q, T)
        eps = keys.shape[0] * np.exp(-T)
        assert np.all(np.abs(Ot - O) <= 2 * eps * fmax / (1 - min(eps, 0.5)))
        assert np.all(lt <= lse + 1e-12) and np.all(lse - lt <= eps / (1 - min(eps, 0.5)))
        assert np.abs(Ot - O).max() > 0  # the truncation really dropped something
    Ot, lt, _ = orc.eval_trunc(g, keys, q, 1e4)
    assert np.allclose(Ot, O, rtol=0, atol=1e-12) and np.allclose(lt, lse, atol=1e-12)


def test_truncated_gradient_limits(orc):
    rng = np.random.default_rng(21)
    R = 4
    g = orc.Grid(R=R)
    keys = orc.build_keys(g, W.perturbed_theta(R, 22, rho0=3.0))
    q = rand_q(rng, 100)
    dl = rng.standard_normal(100)
    gk, ak = orc.grad_global(keys, q, dl)
    gt, at = orc.grad_trunc(g, keys, q, dl, 1e4)
    assert np.allclose(gt, gk, rtol=1e-10, atol=1e-12)
    gt, at = orc.grad_trunc(g, keys, q, dl, 20.0)
    assert np.all(np.abs(gt - gk) <= 1e-4 * ak + 1e-6 * ak.max(axis=0))


def test_truncated_mode_keeps_points_outside_domain_correct(orc):
    rng = np.random.default_rng(23)
    g = orc.Grid(R=5)
    keys = orc.build_keys(g, W.perturbed_theta(5, 24, rho0=4.0))
    q = rand_q(rng, 100, -1.6, 1.6)
    O, _, _ = orc.eval_global(keys, q)
    Ot, _, _ = orc.eval_trunc(g, keys, q, 30.0)
    assert np.allclose(Ot, O, rtol=0, atol=1e-9)


# ---------------------------------------------------------------------- Adam
@pytest.mark.parametrize("wd", [0.0, 0.01])
def test_adamw_matches_torch(orc, wd):
    import torch
    rng = np.random.default_rng(25)
    n = 64
    p0 = rng.standard_normal(n)
    grads = [rng.standard_normal(n) for _ in range(4)]
    P = torch.tensor(p0, requires_grad=True)
    opt = torch.optim.AdamW([P], lr=6e-4, betas=(0.9, 0.999), eps=1e-8, weight_decay=wd)
    th, m, v = p0.copy(), np.zeros(n), np.zeros(n)
    for s, gr in enumerate(grads, start=1):
        P.grad = torch.tensor(gr)
        opt.step()
        th, m, v = orc.adam(th, m, v, gr, s, lr=6e-4, wd=wd)
    assert np.allclose(th, P.detach().numpy(), rtol=0, atol=1e-15)


# ---------------------------------------------------------------- mean-shift
def test_meanshift_single_point_moves_every_key_onto_it(orc):
    g = orc.Grid(R=3)
    s = np.array([[0.123, -0.456, 0.789]])
    D = orc.meanshift(g, s, 100.0)
    t = orc.lattice(g)
    K = np.stack(np.meshgrid(t, t, t, indexing="ij"), -1).reshape(-1, 3)
    assert np.allclose(K + D, s, rtol=0, atol=1e-15)


def test_meanshift_symmetric_set_keeps_centre_key(orc):
    g = orc.Grid(R=3)  # vertex 13 sits at the origin
    s = np.array([[0.1, 0, 0], [-0.1, 0, 0], [0, 0.2, 0], [0, -0.2, 0], [0, 0, 0.3], [0, 0, -0.3]])
    D = orc.meanshift(g, s, 100.0)
    assert np.allclose(D[13], 0.0, atol=1e-15)


def test_meanshift_matches_library_softmax_and_survives_far_keys(orc):
    """Sec. 3.3 mean-shift = softmax(-bw ||k - s||^2)-weighted mean minus k;
    keys ~10 away would underflow exp(-100 d^2) without the common factor."""
    rng = np.random.default_rng(27)
    g = orc.Grid(R=3, lo=-10.0, hi=10.0)
    s = rng.standard_normal((300, 3)) * 0.3
    D = orc.meanshift(g, s, 100.0)
    t = orc.lattice(g)
    K = np.stack(np.meshgrid(t, t, t, indexing="ij"), -1).reshape(-1, 3)
    d2 = ((K[:, None, :] - s[None]) ** 2).sum(-1)
    ref = sps.softmax(-100.0 * d2, axis=1) @ s - K
    assert np.all(np.isfinite(D))
    assert np.allclose(D, ref, rtol=0, atol=1e-9)


# ------------------------------------------------------------------ fit step
def test_fit_step_composes_loss_gradient_and_adam(orc):
    rng = np.random.default_rng(29)
    R = 3
    g = orc.Grid(R=R)
    th = W.perturbed_theta(R, 30)
    q = rand_q(rng, 200)
    o = np.linalg.norm(q, axis=1) - 0.5
    n = R ** 3 * 13
    out = orc.fit_step(g, th, np.zeros(n), np.zeros(n), 1, q, o)
    O, _, _ = orc.eval_global(orc.build_keys(g, th), q)
    assert np.isclose(out["loss"], np.mean((O - o) ** 2), rtol=1e-14)
    assert np.isclose(out["l1"], np.mean(np.abs(O - o)), rtol=1e-14)
    gk, _ = orc.grad_global(orc.build_keys(g, th), q, 2 * (O - o) / len(q))
    gt = orc.grad_theta(g, th, gk)
    assert np.allclose(out["grad"], gt, rtol=1e-12, atol=1e-15)
    # step 1 of Adam moves each parameter by lr * g / (|g| + eps)
    step = out["theta"] - th.astype(np.float64)
    assert np.allclose(step, -6e-4 * gt / (np.abs(gt) + 1e-8), rtol=1e-9, atol=1e-13)
    tr = orc.fit_step(g, th, np.zeros(n), np.zeros(n), 1, q, o, mode=1, T=1e4)
    assert np.allclose(tr["grad"], out["grad"], rtol=1e-10, atol=1e-14)


def test_fit_step_on_exact_linear_target_is_stationary(orc):
    rng = np.random.default_rng(31)
    R = 3
    g = orc.Grid(R=R)
    b = np.array([0.5, 0.25, -0.75])
    th = linear_theta(R, 0.125, b, seed=5)
    keys = orc.build_keys(g, th)
    q = rand_q(rng, 100)
    O, _, _ = orc.eval_global(keys, q)
    n = R ** 3 * 13
    out = orc.fit_step(g, th, np.zeros(n), np.zeros(n), 1, q, O)
    assert out["loss"] == 0.0
    assert np.array_equal(out["theta"], th.astype(np.float64).reshape(out["theta"].shape))


def test_logit_conditioning_scale(orc):
    """kappa = sum_a w_a |s_a| |f_a - O| vanishes for a constant field and for
    a single key, and is non-negative."""
    rng = np.random.default_rng(33)
    g = orc.Grid(R=3)
    th = W.perturbed_theta(3, 34)
    q = rand_q(rng, 50)
    k = orc.eval_cond(orc.build_keys(g, th), q)
    assert np.all(k >= 0) and k.max() > 0
    th[..., [1, 2, 3, 9, 10, 11]] = 0
    th[..., 0] = 0.25
    th[..., 8] = 0.25
    assert np.all(orc.eval_cond(orc.build_keys(g, th), q) <= 1e-14)
    one = np.array([[0.1, 0.2, 0.3, 40.0, 0.5, 1.0, 2.0, 3.0]])
    assert np.all(orc.eval_cond(one, q) == 0.0)


def test_truncation_tail_scales(orc):
    """The below-threshold parts of the error scales: nothing for T -> inf,
    everything for T -> -inf, monotone in between."""
    rng = np.random.default_rng(35)
    g = orc.Grid(R=4)
    keys = orc.build_keys(g, W.perturbed_theta(4, 36, rho0=3.0))
    q = rand_q(rng, 40)
    dl = rng.standard_normal(40)
    gk, ak, b_hi = orc.grad_global(keys, q, dl, T=1e9)
    _, _, b_lo = orc.grad_global(keys, q, dl, T=-1e9)
    _, _, b_mid = orc.grad_global(keys, q, dl, T=10.0)
    assert np.all(b_hi == 0) and np.allclose(b_lo, ak, rtol=1e-12, atol=0)
    assert np.all(b_mid <= ak * (1 + 1e-12)) and 0 < b_mid.sum() < ak.sum()
    k, t_hi = orc.eval_cond(keys, q, 1e9, with_tail=True)
    _, t_lo = orc.eval_cond(keys, q, -1e9, with_tail=True)
    _, t_mid = orc.eval_cond(keys, q, 10.0, with_tail=True)
    O, _, _ = orc.eval_global(keys, q)
    assert np.all(t_hi == 0) and np.all(t_mid <= t_lo) and np.all(t_mid >= 0)
    # all keys: sum_a w_a |f_a - O| >= |sum_a w_a (f_a - O)| = 0, and <= 2 max |f|
    assert np.all(t_lo <= 2 * (np.abs(keys[:, 4]).max() + 4 * np.abs(keys[:, 5:]).max()))


# ------------------------------------------------------------ tolerance scales
# The parity tolerances rest on these scales, so each is tied to something the
# oracle does not compute itself: the pinned value or gradient in a case where
# every contribution has one sign (a sum of magnitudes then equals the sum),
# closed forms of the two-key logistic blend (Sec. 3.1, Eq. nrbf), or finite
# differences of the pinned evaluation.

def _below_keys(rng, n, lo=-1.0, hi=-0.6, beta=(5.0, 40.0)):
    """Keys centred in [lo, hi]^3 with non-negative values and slopes: for
    queries in [0, 1]^3 every x = q - c is positive, so every term of
    f_a = o_a + x . d_a is non-negative."""
    keys = np.empty((n, 8))
    keys[:, :3] = rng.uniform(lo, hi, (n, 3))
    keys[:, 3] = rng.uniform(*beta, n)
    keys[:, 4] = rng.uniform(0.0, 1.0, n)
    keys[:, 5:] = rng.uniform(0.0, 1.0, (n, 3))
    return keys


def _two_key_parts(keys, q):
    """Logits, polynomial values and logistic weights of a two-key set."""
    s = [-k[3] * ((q - k[:3]) ** 2).sum(1) for k in keys]
    f = [k[4] + (q - k[:3]) @ k[5:] for k in keys]
    return s, f, sps.expit(s[0] - s[1]), sps.expit(s[1] - s[0])


def _cancel(s, f):
    """Absolute rounding allowance of |f_a - O| (computed as a difference of
    numbers of size |f|) times the logit magnitudes."""
    return 1e-14 * (np.abs(s[0]) + np.abs(s[1]) + 1.0) * (np.abs(f[0]) + np.abs(f[1]))


TWO_KEYS = np.array([[-0.3, -0.2, -0.25, 12.0, 0.8, 0.5, -0.3, 0.2],
                     [0.35, 0.3, 0.2, 20.0, -0.6, -0.4, 0.7, 0.1]])


def test_sigma_equals_value_when_every_term_is_nonnegative(orc):
    """sigma = sum_a w_a (|o_a| + sum_k |x_k| |d_ak|) equals O when no term is
    negative, and is unchanged by flipping the signs of values and slopes."""
    rng = np.random.default_rng(41)
    keys = _below_keys(rng, 40)
    q = rng.uniform(0.0, 1.0, (60, 3))
    O, _, sig = orc.eval_global(keys, q)
    assert np.allclose(sig, O, rtol=1e-13, atol=0)
    mixed = keys.copy()
    mixed[:, 4:] *= rng.choice([-1.0, 1.0], size=(40, 4))
    Om, _, sm = orc.eval_global(mixed, q)
    assert np.allclose(sm, O, rtol=1e-13, atol=0)
    assert np.all(sm >= np.abs(Om)) and np.any(sm > 1.5 * np.abs(Om))


def test_truncated_scales_equal_global_ones_when_nothing_is_dropped(orc):
    """With a threshold no pair falls below, the truncated mode's value scale
    and gradient scales are the (pinned) global ones."""
    rng = np.random.default_rng(43)
    R = 4
    g = orc.Grid(R=R)
    keys = orc.build_keys(g, W.perturbed_theta(R, 44, rho0=3.0))
    q = rand_q(rng, 80)
    dl = rng.standard_normal(80)
    _, _, sig = orc.eval_global(keys, q)
    _, _, sig_t = orc.eval_trunc(g, keys, q, 1e4)
    assert np.allclose(sig_t, sig, rtol=1e-12, atol=0)
    _, ak = orc.grad_global(keys, q, dl)
    _, ak_t = orc.grad_trunc(g, keys, q, dl, 1e4)
    assert np.allclose(ak_t, ak, rtol=1e-10, atol=1e-300)


def test_kappa_two_key_closed_form(orc):
    """Two keys: f_1 - O = w_2 (f_1 - f_2) and f_2 - O = w_1 (f_2 - f_1), so
    kappa = w_1 w_2 |f_1 - f_2| (|s_1| + |s_2|)."""
    rng = np.random.default_rng(45)
    q = rand_q(rng, 80, -0.8, 0.8)
    kap = orc.eval_cond(TWO_KEYS, q)
    s, f, w1, w2 = _two_key_parts(TWO_KEYS, q)
    ref = w1 * w2 * np.abs(f[0] - f[1]) * (np.abs(s[0]) + np.abs(s[1]))
    assert np.all(np.abs(kap - ref) <= 1e-11 * ref + _cancel(s, f))


def test_kappa_is_the_worst_case_logit_sensitivity(orc):
    """Moving every logit by eps |s_a| towards the sign of f_a - O changes O by
    eps kappa to first order; with f^1 values that move is a scaling of
    beta_a by 1 - eps sign(f_a - O) (beta enters O only through the logits).
    Each f_a is the pinned one-key output."""
    rng = np.random.default_rng(47)
    g = orc.Grid(R=3)
    keys = orc.build_keys(g, W.perturbed_theta(3, 48, rho0=1.5, rho_spread=1.0))
    for q in rand_q(rng, 6, -0.9, 0.9):
        q = q[None, :]
        O, _, _ = orc.eval_global(keys, q)
        f = np.array([orc.eval_global(keys[a:a + 1], q)[0][0] for a in range(len(keys))])
        sgn = np.sign(f - O[0])
        eps = 1e-6

        def O_at(e):
            k2 = keys.copy()
            k2[:, 3] *= 1.0 - e * sgn
            return orc.eval_global(k2, q)[0][0]

        fd = (O_at(eps) - O_at(-eps)) / (2 * eps)
        kap = orc.eval_cond(keys, q)[0]
        assert abs(fd - kap) <= 1e-6 * kap + 1e-9, (fd, kap)


def test_tail_two_key_closed_form(orc):
    """Two keys: a key whose weight is below e^-T contributes
    w_a |f_a - O| = w_1 w_2 |f_1 - f_2| to the tail."""
    rng = np.random.default_rng(49)
    q = rand_q(rng, 200, -0.9, 0.9)
    s, f, w1, w2 = _two_key_parts(TWO_KEYS, q)
    T = 4.0
    _, tail = orc.eval_cond(TWO_KEYS, q, T, with_tail=True)
    n_light = (w1 < np.exp(-T)).astype(float) + (w2 < np.exp(-T)).astype(float)
    ref = n_light * w1 * w2 * np.abs(f[0] - f[1])
    assert 0 < (n_light > 0).sum() < len(q)
    assert np.all(np.abs(tail - ref) <= 1e-11 * ref + _cancel(s, f))


def _one_sign_setup(rng):
    """f^1 keys around the cube, plus key 0 below every query with the largest
    values (r = f_0 - O > 0, x > 0, slopes <= 0) and key 1 above every query
    with the smallest values and zero slopes (r < 0, x < 0)."""
    n = 30
    keys = np.empty((n, 8))
    keys[:, :3] = rng.uniform(-1, 1, (n, 3))
    keys[:, 3] = rng.uniform(1.0, 4.0, n)
    keys[:, 4] = rng.uniform(-1, 1, n)
    keys[:, 5:] = 0.2 * rng.standard_normal((n, 3))
    keys[0] = [-1.2, -1.2, -1.2, 2.0, 6.0, -0.1, -0.2, -0.15]
    keys[1] = [1.2, 1.2, 1.2, 2.0, -6.0, 0.0, 0.0, 0.0]
    q = rand_q(rng, 70, -1.0, 1.0)
    dl = rng.standard_normal(70)
    return keys, q, dl


def test_gradient_scale_is_the_gradient_of_magnitudes(orc):
    """A = sum_j |term| per entry.  The value channel's term is dl_j w_aj, so
    A_o(dl) = G_o(|dl|) for every key.  Keys 0 and 1 of the set-up have
    terms of one sign in every channel, so there A equals |G(|dl|)|; the
    gradient G is pinned by finite differences."""
    rng = np.random.default_rng(51)
    keys, q, dl = _one_sign_setup(rng)
    _, ak = orc.grad_global(keys, q, dl)
    gabs, _ = orc.grad_global(keys, q, np.abs(dl))
    assert np.allclose(ak[:, 4], gabs[:, 4], rtol=1e-12, atol=0)
    for a in (0, 1):
        assert np.allclose(ak[a], np.abs(gabs[a]), rtol=1e-11, atol=1e-300), a
    # the sign of dL/dO does not enter A; A is additive over queries
    _, ak_neg = orc.grad_global(keys, q, -dl)
    _, ak1 = orc.grad_global(keys, q[:30], dl[:30])
    _, ak2 = orc.grad_global(keys, q[30:], dl[30:])
    assert np.array_equal(ak, ak_neg)
    assert np.allclose(ak, ak1 + ak2, rtol=1e-12, atol=1e-300)


def test_subthreshold_gradient_scale_sums_the_light_pairs(orc):
    """B is A restricted to the pairs whose weight is below e^-T: the sum of
    the single-query scales over the queries where that key is light (weights
    from scipy's softmax of the Eq. nrbf logits)."""
    rng = np.random.default_rng(53)
    g = orc.Grid(R=3)
    keys = orc.build_keys(g, W.perturbed_theta(3, 54, rho0=2.0, rho_spread=1.0))
    q = rand_q(rng, 25)
    dl = rng.standard_normal(25)
    T = 5.0
    _, _, bk = orc.grad_global(keys, q, dl, T=T)
    logits = -keys[None, :, 3] * ((q[:, None, :] - keys[None, :, :3]) ** 2).sum(-1)
    w = sps.softmax(logits, axis=1)
    ref = np.zeros_like(bk)
    for j in range(len(q)):
        _, aj = orc.grad_global(keys, q[j:j + 1], dl[j:j + 1])
        ref += aj * (w[j] < np.exp(-T))[:, None]
    assert 0 < (w < np.exp(-T)).sum() < w.size
    assert np.allclose(bk, ref, rtol=1e-11, atol=1e-300)


def _two_key_qgrad_parts(keys, q):
    s, f, w1, w2 = _two_key_parts(keys, q)
    O = w1 * f[0] + w2 * f[1]
    g1 = keys[0, 5:] + 2 * keys[0, 3] * (q - keys[0, :3]) * (w2 * (f[1] - f[0]))[:, None]
    g2 = keys[1, 5:] + 2 * keys[1, 3] * (q - keys[1, :3]) * (w1 * (f[0] - f[1]))[:, None]
    return s, f, w1, w2, O, g1, g2


def test_query_gradient_scales_two_key_closed_forms(orc):
    """Two keys, with O - f_1 = w_2 (f_2 - f_1), O - f_2 = w_1 (f_1 - f_2) and
    g_a = d_a + 2 beta_a x_a (O - f_a) (Eq. func-normal):
      qsig  = w_1 (|d_1| + 2 beta_1 |x_1| |O - f_1|) + (same for key 2);
      qkap  = w_1 w_2 (|s_1| + |s_2|) |g_1 - g_2|
              + 2 (beta_1 w_1 |x_1| sigma_1 + beta_2 w_2 |x_2| sigma_2);
      qtail = for each key lighter than e^-T: w_a (|g_a| + |G|);
      qbx   = 2 (beta_1 w_1 |x_1| + beta_2 w_2 |x_2|), and dG/dO at fixed
              weights, 2 (beta_1 w_1 x_1 + beta_2 w_2 x_2), is within it;
    the query gradient G itself is pinned by central differences."""
    rng = np.random.default_rng(55)
    q = rand_q(rng, 150, -0.9, 0.9)
    k = TWO_KEYS
    T = 4.0
    qs, qk, qt, qb = orc.eval_qgrad_scales(k, q, T)
    s, f, w1, w2, O, g1, g2 = _two_key_qgrad_parts(k, q)
    x1, x2 = q - k[0, :3], q - k[1, :3]
    b1 = 2 * k[0, 3] * w1[:, None] * np.abs(x1)
    b2 = 2 * k[1, 3] * w2[:, None] * np.abs(x2)
    allow = _cancel(s, f)[:, None] * (b1 + b2)
    ref_s = (w1[:, None] * np.abs(k[0, 5:]) + b1 * np.abs(O - f[0])[:, None]
             + w2[:, None] * np.abs(k[1, 5:]) + b2 * np.abs(O - f[1])[:, None])
    assert np.all(np.abs(qs - ref_s) <= 1e-11 * ref_s + allow)
    sig1 = np.abs(k[0, 4]) + np.abs(x1) @ np.abs(k[0, 5:])
    sig2 = np.abs(k[1, 4]) + np.abs(x2) @ np.abs(k[1, 5:])
    ref_k = ((w1 * w2 * (np.abs(s[0]) + np.abs(s[1])))[:, None] * np.abs(g1 - g2)
             + b1 * sig1[:, None] + b2 * sig2[:, None])
    assert np.allclose(qk, ref_k, rtol=1e-11, atol=1e-300)
    G = w1[:, None] * g1 + w2[:, None] * g2
    light1 = (w1 < np.exp(-T))[:, None]
    light2 = (w2 < np.exp(-T))[:, None]
    ref_t = (light1 * w1[:, None] * (np.abs(g1) + np.abs(G))
             + light2 * w2[:, None] * (np.abs(g2) + np.abs(G)))
    assert 0 < (light1 | light2).sum() < len(q)
    assert np.allclose(qt, ref_t, rtol=1e-11, atol=1e-300)
    assert np.allclose(qb, b1 + b2, rtol=1e-12, atol=0)
    assert np.allclose(orc.eval_qgrad(k, q), G, rtol=1e-12, atol=1e-14)


def test_query_gradient_scale_bounds_its_change_with_O(orc):
    """Two keys: raising the constant term of key 2 by c leaves the weights
    alone, moves O by w_2 c and moves dO/dq by 2 w_1 w_2 (beta_1 x_1 -
    beta_2 x_2) c (central differences of the pinned oracle), which qbx
    bounds per unit change of O."""
    rng = np.random.default_rng(59)
    q = rand_q(rng, 60, -0.5, 0.5)
    k = TWO_KEYS.copy()
    qs, _, _, qb = orc.eval_qgrad_scales(k, q)
    c = 1e-6
    kp, km = k.copy(), k.copy()
    kp[1, 4] += c
    km[1, 4] -= c
    dG = (orc.eval_qgrad(kp, q) - orc.eval_qgrad(km, q)) / (2 * c)
    dO = (orc.eval_global(kp, q)[0] - orc.eval_global(km, q)[0]) / (2 * c)
    s, f, w1, w2 = _two_key_parts(k, q)
    assert np.allclose(dO, w2, rtol=1e-6, atol=1e-9)
    # dG/dc = 2 beta_1 w_1 x_1 w_2 - 2 beta_2 w_2 x_2 w_1 (the weights do not
    # depend on the values), i.e. exactly qbx's terms with signs
    x1, x2 = q - k[0, :3], q - k[1, :3]
    ref = 2 * k[0, 3] * (w1 * w2)[:, None] * x1 - 2 * k[1, 3] * (w1 * w2)[:, None] * x2
    assert np.allclose(dG, ref, rtol=1e-5, atol=1e-8)
    assert np.all(np.abs(dG) <= qb + 1e-8)


def test_query_gradient_scale_equals_gradient_when_terms_share_a_sign(orc):
    """Key 1 below the query and key 2 above it on every axis, zero slopes
    and f_2 > f_1: every term 2 beta_a x_a (O - f_a) is positive, so qsig
    equals dO/dq, which is pinned by central differences."""
    rng = np.random.default_rng(57)
    q = rng.uniform(-0.2, 0.2, (50, 3))
    k = np.array([[-0.5, -0.45, -0.55, 6.0, -0.7, 0.0, 0.0, 0.0],
                  [0.5, 0.6, 0.45, 9.0, 0.9, 0.0, 0.0, 0.0]])
    qs = orc.eval_qgrad_scales(k, q)[0]
    G = orc.eval_qgrad(k, q)
    assert np.all(G > 0)
    assert np.allclose(qs, G, rtol=1e-12, atol=0)


def test_truncated_band_scale_is_the_global_subthreshold_scale(orc):
    """The truncated gradient's band scale (pairs below e^-Tb, searched down to
    M_j - T2) equals the global B when T2 reaches every pair, and it bounds
    how far the truncation at T moves the gradient from the definition."""
    rng = np.random.default_rng(57)
    R = 4
    g = orc.Grid(R=R)
    keys = orc.build_keys(g, W.perturbed_theta(R, 58, rho0=3.0))
    q = rand_q(rng, 120)
    dl = rng.standard_normal(120)
    gk, ak, bk = orc.grad_global(keys, q, dl, T=5.0)
    _, _, bt = orc.grad_trunc(g, keys, q, dl, 1e4, Tb=5.0, T2=1e4)
    assert 0 < (bk > 0).sum() and np.any(bk < ak)
    assert np.allclose(bt, bk, rtol=1e-10, atol=1e-300)
    # truncating at T = 20 drops only pairs below e^-20, which B at Tb = 20 covers
    _, _, b20 = orc.grad_global(keys, q, dl, T=20.0)
    gt, at, bt = orc.grad_trunc(g, keys, q, dl, 20.0, Tb=20.0, T2=60.0)
    # weights from the truncated lse, which is within K e^-20 of the global one
    assert np.allclose(bt, b20, rtol=1e-6, atol=1e-300)
    assert np.all(np.abs(gt - gk) <= bt + 1e-6 * at + 1e-300)
    assert np.abs(gt - gk).max() > 0
