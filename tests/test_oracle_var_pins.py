"""Pins of the FP64 variant oracle (oracle/efunc_oracle_var.c) against facts
that do not come from the oracle itself: the paper's channel counts, the
pinned first-order oracle, exact reproduction of quadratics by f^2
(partition of unity), the two-key logistic closed form, central differences
and torch autograd."""
import json
import os

import numpy as np
import pytest
import scipy.special as sps

import oracle as O1
from oracle import variants as V

GOLD = os.path.join(os.path.dirname(__file__), "golden")

MODELS = [
    dict(degree=0, grid_keys=1, moved_keys=0, learn_scale=1),
    dict(degree=0, grid_keys=1, moved_keys=1, learn_scale=0, rho_fixed=4.5),
    dict(degree=1, grid_keys=0, moved_keys=1, learn_scale=1),
    dict(degree=2, grid_keys=1, moved_keys=0, learn_scale=1),
    dict(degree=2, grid_keys=1, moved_keys=1, learn_scale=1),
    dict(degree=2, grid_keys=0, moved_keys=1, learn_scale=0, rho_fixed=4.5),
]


@pytest.fixture(scope="module")
def var():
    V.build_var_oracle(force=False)
    V.load()
    return V


def random_theta(m, seed, rho=(4.0, 5.0), offset=0.3):
    """Seeded theta in the model's channel layout: values U[-1,1], slopes and
    curvatures N(0,1), log-scales U[rho], offsets N(0, (offset h)^2)."""
    rng = np.random.default_rng(seed)
    L = V.layout(m)
    nch, nv = L["nch"], V.num_values(m.degree)
    h = (m.hi - m.lo) / (m.R - 1)
    th = np.zeros((m.I, nch))
    for vo in (L["grid_values"], L["moved_values"]):
        if vo >= 0:
            th[:, vo] = rng.uniform(-1, 1, m.I)
            if nv > 1:
                th[:, vo + 1:vo + nv] = rng.standard_normal((m.I, nv - 1))
    for ro in (L["grid_rho"], L["moved_rho"]):
        if ro >= 0:
            th[:, ro] = rng.uniform(*rho, m.I)
    if L["moved_delta"] >= 0:
        th[:, L["moved_delta"]:L["moved_delta"] + 3] = offset * h * rng.standard_normal((m.I, 3))
    return th.astype(np.float32)


def queries(n, seed, span=1.1):
    return np.random.default_rng(seed).uniform(-span, span, (n, 3))


def test_channel_counts_match_paper(var):
    d = json.load(open(os.path.join(GOLD, "paper_param_counts.json")))
    for e in d["variants"]:
        m = V.Model(R=e["R"], degree=e["degree"], grid_keys=e["grid_keys"],
                    moved_keys=e["moved_keys"], learn_scale=e["learn_scale"])
        assert V.channels(m) == e["channels"], e["config"]
        assert V.channels(m) * m.I == e["params"], e["config"]


def test_degree1_default_matches_first_order_oracle(var):
    """The default model (degree 1, both key sets, learnable scales) against
    the separately pinned 13-channel oracle: keys, values, gradients."""
    m = V.Model(R=4)
    th = random_theta(m, 1)
    q = queries(300, 2)
    kv = V.build_keys(m, th)
    k1 = O1.build_keys(O1.Grid(R=4), th.reshape(4, 4, 4, 13))
    assert np.array_equal(kv[:, :8], k1)
    Ov, lv, _ = V.eval_global(kv, 1, q)
    O1v, l1v, _ = O1.eval_global(k1, q)
    assert np.allclose(Ov, O1v, rtol=0, atol=1e-13) and np.allclose(lv, l1v, rtol=0, atol=1e-12)
    dl = np.random.default_rng(3).standard_normal(len(q))
    gv, _ = V.grad_global(kv, 1, q, dl)
    g1, _ = O1.grad_global(k1, q, dl)
    assert np.allclose(gv[:, :8], g1, rtol=1e-12, atol=1e-12)
    assert np.all(gv[:, 8:] == 0)
    tv = V.grad_theta(m, th, gv)
    t1 = O1.grad_theta(O1.Grid(R=4), th.reshape(4, 4, 4, 13), g1)
    assert np.allclose(tv, t1.reshape(-1), rtol=1e-12, atol=1e-12)
    assert np.allclose(V.eval_qgrad(kv, 1, q), O1.eval_qgrad(k1, q), rtol=0, atol=1e-11)


def test_moved_keys_only_matches_first_order_oracle(var):
    """O^Delta (Eq. func-with-offset): the moved keys alone, against the
    first-order oracle evaluated on the moved half of its key list."""
    R = 4
    m = V.Model(R=R, degree=1, grid_keys=0)
    th8 = random_theta(m, 4)
    th13 = np.zeros((m.I, 13), np.float32)
    th13[:, 5:13] = th8
    th13[:, 4] = 1.0
    k1 = O1.build_keys(O1.Grid(R=R), th13.reshape(R, R, R, 13))[m.I:]
    kv = V.build_keys(m, th8)
    assert np.array_equal(kv[:, :8], k1)
    q = queries(200, 5)
    assert np.allclose(V.eval_global(kv, 1, q)[0], O1.eval_global(k1, q)[0], rtol=0, atol=1e-13)


def _taylor_keys(m, seed):
    """Keys whose polynomials are all the Taylor expansion, at the key's own
    centre, of one random quadratic Q(x) = a + b.x + 1/2 x^T A x."""
    rng = np.random.default_rng(seed)
    th = random_theta(m, seed)
    keys = V.build_keys(m, th)
    a = rng.standard_normal()
    b = rng.standard_normal(3)
    A = rng.standard_normal((3, 3))
    A = A + A.T
    c = keys[:, :3]
    keys[:, 4] = a + c @ b + 0.5 * np.einsum("ni,ij,nj->n", c, A, c)
    keys[:, 5:8] = b + c @ A
    keys[:, 8:14] = [A[0, 0], A[1, 1], A[2, 2], A[0, 1], A[0, 2], A[1, 2]]
    Q = lambda q: a + q @ b + 0.5 * np.einsum("ni,ij,nj->n", q, A, q)  # noqa: E731
    dQ = lambda q: b + q @ A  # noqa: E731
    return keys, Q, dQ


@pytest.mark.parametrize("moved", [0, 1])
def test_degree2_reproduces_quadratics(var, moved):
    """With every key carrying Q's Taylor coefficients, every f_a(q) = Q(q)
    and the softmax weights sum to one, so O = Q and dO/dq = grad Q exactly."""
    m = V.Model(R=4, degree=2, moved_keys=moved)
    keys, Q, dQ = _taylor_keys(m, 7 + moved)
    q = queries(400, 8)
    O, _, _ = V.eval_global(keys, 2, q)
    scale = np.abs(Q(q)).max() + 1.0
    assert np.abs(O - Q(q)).max() <= 1e-12 * scale
    g = V.eval_qgrad(keys, 2, q)
    assert np.abs(g - dQ(q)).max() <= 1e-11 * (np.abs(dQ(q)).max() + 1.0)


def test_degree2_gradient_of_reproduced_quadratic(var):
    """At an exactly reproduced quadratic every r = f - O vanishes, so the
    scale gradients vanish and the centre gradient is -(d + S x) summed with
    the weights: the key-level closed forms reduce to sums of Q's gradient."""
    m = V.Model(R=3, degree=2)
    keys, Q, dQ = _taylor_keys(m, 11)
    q = queries(120, 12, span=0.9)
    dl = np.random.default_rng(13).standard_normal(len(q))
    gk, _ = V.grad_global(keys, 2, q, dl)
    assert np.abs(gk[:, 3]).max() <= 1e-10
    # sum over keys of dL/dc = -sum_j dl_j sum_a w_a grad f_a = -sum_j dl_j grad Q(q_j)
    tot = gk[:, :3].sum(axis=0)
    assert np.allclose(tot, -(dl[:, None] * dQ(q)).sum(axis=0), rtol=1e-10, atol=1e-10)


def test_degree0_two_keys_logistic(var):
    """f^0 with two keys: O = o1 expit(s1 - s2) + o2 expit(s2 - s1)."""
    m = V.Model(R=2, degree=0, moved_keys=0)
    keys = V.build_keys(m, random_theta(m, 21))[:2].copy()
    keys[:, 3] = [3.0, 5.0]
    keys[:, 4] = [0.7, -1.3]
    q = queries(100, 22)
    s = -keys[:, 3][None, :] * ((q[:, None, :] - keys[None, :, :3]) ** 2).sum(-1)
    ref = keys[0, 4] * sps.expit(s[:, 0] - s[:, 1]) + keys[1, 4] * sps.expit(s[:, 1] - s[:, 0])
    assert np.allclose(V.eval_global(keys, 0, q)[0], ref, rtol=0, atol=1e-14)


def test_fixed_scale_uses_rho_fixed(var):
    """learn_scale = 0: every key has beta = exp(rho_fixed) and no scale
    channel; values equal those of the learnable model with all rho equal."""
    mf = V.Model(R=3, degree=2, learn_scale=0, rho_fixed=4.5)
    ml = V.Model(R=3, degree=2, learn_scale=1)
    thf = random_theta(mf, 31)
    Lf, Ll = V.layout(mf), V.layout(ml)
    thl = np.zeros((ml.I, Ll["nch"]), np.float32)
    thl[:, Ll["grid_values"]:Ll["grid_values"] + 10] = thf[:, Lf["grid_values"]:Lf["grid_values"] + 10]
    thl[:, Ll["moved_delta"]:Ll["moved_delta"] + 3] = thf[:, Lf["moved_delta"]:Lf["moved_delta"] + 3]
    thl[:, Ll["moved_values"]:Ll["moved_values"] + 10] = thf[:, Lf["moved_values"]:Lf["moved_values"] + 10]
    thl[:, Ll["grid_rho"]] = np.float32(4.5)
    thl[:, Ll["moved_rho"]] = np.float32(4.5)
    kf, kl = V.build_keys(mf, thf), V.build_keys(ml, thl)
    assert np.allclose(kf[:, 3], np.exp(4.5), rtol=1e-15)
    q = queries(150, 32)
    assert np.allclose(V.eval_global(kf, 2, q)[0], V.eval_global(kl, 2, q)[0], rtol=0, atol=1e-6)


@pytest.mark.parametrize("mi", range(len(MODELS)))
def test_key_gradients_match_central_differences(var, mi):
    """Every key-record gradient entry (centre, beta, coefficients) against
    central differences of sum_j dl_j O(q_j) in double precision."""
    m = V.Model(R=3, **MODELS[mi])
    keys = V.build_keys(m, random_theta(m, 40 + mi))
    q = queries(60, 41 + mi, span=1.0)
    dl = np.random.default_rng(42 + mi).standard_normal(len(q))
    gk, _ = V.grad_global(keys, m.degree, q, dl)
    nv = V.num_values(m.degree)
    rng = np.random.default_rng(43 + mi)
    for a in rng.choice(len(keys), 6, replace=False):
        for c in list(range(4)) + list(range(4, 4 + nv)):
            col = c if c < 4 else c
            h = 1e-6 * max(1.0, abs(keys[a, col]))

            def L(delta):
                k2 = keys.copy()
                k2[a, col] += delta
                return dl @ V.eval_global(k2, m.degree, q)[0]
            fd = (L(h) - L(-h)) / (2 * h)
            assert abs(fd - gk[a, c]) <= 1e-6 * (abs(gk[a, c]) + np.abs(dl).sum() * 1e-3), (a, c)


@pytest.mark.parametrize("mi", range(len(MODELS)))
def test_theta_gradients_match_central_differences(var, mi):
    """The channel mapping (rho chain rule, Delta = centre gradient) against
    Richardson-extrapolated central differences in theta."""
    m = V.Model(R=3, **MODELS[mi])
    th = random_theta(m, 50 + mi)
    q = queries(50, 51 + mi, span=1.0)
    dl = np.random.default_rng(52 + mi).standard_normal(len(q))
    gk, _ = V.grad_global(V.build_keys(m, th), m.degree, q, dl)
    gt = V.grad_theta(m, th, gk)
    flat = th.reshape(-1)
    rng = np.random.default_rng(53 + mi)
    for i in rng.choice(flat.size, 25, replace=False):
        def L(h):
            t2 = flat.copy()
            t2[i] = np.float32(flat[i] + h)
            return dl @ V.eval_global(V.build_keys(m, t2), m.degree, q)[0], float(t2[i]) - float(flat[i])

        def D(h):
            (lp, sp), (lm, sm) = L(h), L(-h)
            return (lp - lm) / (sp - sm)
        h = 2.0 ** -8
        est = (4 * D(h / 2) - D(h)) / 3
        assert abs(est - gt[i]) <= 2e-4 * (abs(gt[i]) + 1e-2 * np.abs(dl).sum() / len(dl)), i


def test_gradients_match_torch_autograd(var):
    """Degree 2 with both key sets: the oracle's closed forms against torch
    autograd of the same definition written with torch primitives."""
    import torch
    m = V.Model(R=3, degree=2)
    keys = V.build_keys(m, random_theta(m, 61))
    q = queries(80, 62)
    dl = np.random.default_rng(63).standard_normal(len(q))
    K = torch.tensor(keys[:, :14], dtype=torch.float64, requires_grad=True)
    Q = torch.tensor(q, dtype=torch.float64)
    x = Q[:, None, :] - K[None, :, :3]
    s = -K[None, :, 3] * (x * x).sum(-1)
    S = K[:, 8:14]
    quad = 0.5 * (S[None, :, 0] * x[..., 0] ** 2 + S[None, :, 1] * x[..., 1] ** 2 + S[None, :, 2] * x[..., 2] ** 2) \
        + S[None, :, 3] * x[..., 0] * x[..., 1] + S[None, :, 4] * x[..., 0] * x[..., 2] \
        + S[None, :, 5] * x[..., 1] * x[..., 2]
    f = K[None, :, 4] + (x * K[None, :, 5:8]).sum(-1) + quad
    O = (torch.softmax(s, dim=1) * f).sum(1)
    (O * torch.tensor(dl)).sum().backward()
    gk, _ = V.grad_global(keys, 2, q, dl)
    assert np.allclose(K.grad.numpy(), gk, rtol=1e-10, atol=1e-12)


def test_fit_step_composes_loss_gradient_and_adam(var):
    m = V.Model(R=3, degree=2, grid_keys=1, moved_keys=1, learn_scale=1)
    th = random_theta(m, 71)
    q = queries(90, 72)
    o = np.sin(q.sum(1))
    n = th.size
    r = V.fit_step(m, th, np.zeros(n), np.zeros(n), 1, q, o)
    keys = V.build_keys(m, th)
    Oe, _, _ = V.eval_global(keys, 2, q)
    assert np.isclose(r["loss"], np.mean((Oe - o) ** 2), rtol=1e-14)
    gk, _ = V.grad_global(keys, 2, q, 2 * (Oe - o) / len(q))
    g = V.grad_theta(m, th, gk)
    assert np.allclose(r["grad"], g, rtol=1e-13, atol=1e-15)
    t_ref, _, _ = O1.adam(th.reshape(-1).astype(np.float64), np.zeros(n), np.zeros(n), g, 1)
    assert np.allclose(r["theta"], t_ref, rtol=1e-14, atol=1e-15)


# ------------------------------------------------------------ tolerance scales
# Each scale the variant parity tolerances use is tied to the separately
# pinned first-order oracle (degree 1), to the pinned value or gradient where
# every contribution has one sign, or to a two-key closed form.

def test_degree1_scales_match_first_order_oracle(var):
    """Default model: sigma, kappa, tail, the gradient scales A and B and the
    query-gradient scales agree with the first-order oracle's (pinned by
    tests/test_oracle_pins.py)."""
    m = V.Model(R=4)
    th = random_theta(m, 61)
    q = queries(150, 62)
    kv = V.build_keys(m, th)
    k1 = O1.build_keys(O1.Grid(R=4), th.reshape(4, 4, 4, 13))
    T = 6.0
    assert np.allclose(V.eval_global(kv, 1, q)[2], O1.eval_global(k1, q)[2], rtol=1e-13, atol=0)
    kv_k, kv_t = V.eval_cond(kv, 1, q, T, with_tail=True)
    k1_k, k1_t = O1.eval_cond(k1, q, T, with_tail=True)
    assert np.allclose(kv_k, k1_k, rtol=1e-12, atol=1e-300)
    assert np.allclose(kv_t, k1_t, rtol=1e-12, atol=1e-300)
    dl = np.random.default_rng(63).standard_normal(len(q))
    _, av, bv = V.grad_global(kv, 1, q, dl, T=T)
    _, a1, b1 = O1.grad_global(k1, q, dl, T=T)
    assert np.allclose(av[:, :8], a1, rtol=1e-12, atol=1e-300)
    assert np.allclose(bv[:, :8], b1, rtol=1e-12, atol=1e-300)
    for sv, s1 in zip(V.eval_qgrad_scales(kv, 1, q, T), O1.eval_qgrad_scales(k1, q, T)):
        assert np.allclose(sv, s1, rtol=1e-12, atol=1e-300)


def _below_keys2(rng, n):
    """Degree-2 keys centred in [-1, -0.6]^3 with non-negative coefficients:
    every monomial term is non-negative for queries in [0, 1]^3."""
    keys = np.zeros((n, V.KEYW))
    keys[:, :3] = rng.uniform(-1.0, -0.6, (n, 3))
    keys[:, 3] = rng.uniform(5.0, 40.0, n)
    keys[:, 4:14] = rng.uniform(0.0, 1.0, (n, 10))
    return keys


def test_degree2_sigma_equals_value_when_every_term_is_nonnegative(var):
    rng = np.random.default_rng(65)
    keys = _below_keys2(rng, 30)
    q = rng.uniform(0.0, 1.0, (50, 3))
    O, _, sig = V.eval_global(keys, 2, q)
    assert np.allclose(sig, O, rtol=1e-13, atol=0)
    mixed = keys.copy()
    mixed[:, 4:14] *= rng.choice([-1.0, 1.0], size=(30, 10))
    Om, _, sm = V.eval_global(mixed, 2, q)
    assert np.allclose(sm, O, rtol=1e-13, atol=0)
    assert np.all(sm >= np.abs(Om)) and np.any(sm > 1.5 * np.abs(Om))


def test_degree2_gradient_scale_is_the_gradient_of_magnitudes(var):
    """A = sum_j |term|: the monomials 1, x^2/2, y^2/2, z^2/2 are never
    negative, so for those coefficients A(dl) = G(|dl|) for every key; for a
    key below every query all monomials are non-negative."""
    m = V.Model(R=3, degree=2)
    keys = V.build_keys(m, random_theta(m, 67))
    keys[0, :3] = [-1.3, -1.3, -1.3]
    q = queries(70, 68, span=1.0)
    dl = np.random.default_rng(69).standard_normal(len(q))
    _, ak = V.grad_global(keys, 2, q, dl)
    gabs, _ = V.grad_global(keys, 2, q, np.abs(dl))
    for c in (4, 8, 9, 10):
        assert np.allclose(ak[:, c], gabs[:, c], rtol=1e-12, atol=1e-300), c
    assert np.allclose(ak[0, 4:14], gabs[0, 4:14], rtol=1e-12, atol=1e-300)
    _, ak_neg = V.grad_global(keys, 2, q, -dl)
    assert np.array_equal(ak, ak_neg)


def test_degree2_subthreshold_scale_sums_the_light_pairs(var):
    m = V.Model(R=3, degree=2)
    keys = V.build_keys(m, random_theta(m, 71, rho=(1.5, 3.0)))
    q = queries(20, 72, span=1.0)
    dl = np.random.default_rng(73).standard_normal(len(q))
    T = 5.0
    _, _, bk = V.grad_global(keys, 2, q, dl, T=T)
    logits = -keys[None, :, 3] * ((q[:, None, :] - keys[None, :, :3]) ** 2).sum(-1)
    w = sps.softmax(logits, axis=1)
    ref = np.zeros_like(bk)
    for j in range(len(q)):
        _, aj = V.grad_global(keys, 2, q[j:j + 1], dl[j:j + 1])
        ref += aj * (w[j] < np.exp(-T))[:, None]
    assert 0 < (w < np.exp(-T)).sum() < w.size
    assert np.allclose(bk, ref, rtol=1e-11, atol=1e-300)


def test_degree0_kappa_and_tail_two_key_closed_forms(var):
    """f^0, two keys: kappa = w1 w2 |o1 - o2| (|s1| + |s2|); a key lighter
    than e^-T adds w1 w2 |o1 - o2| to the tail."""
    keys = np.zeros((2, 16))
    keys[0, :5] = [-0.3, 0.1, 0.2, 6.0, 0.7]
    keys[1, :5] = [0.4, -0.2, 0.1, 11.0, -1.3]
    q = queries(200, 74, span=0.9)
    s = -keys[:, 3][None, :] * ((q[:, None, :] - keys[None, :, :3]) ** 2).sum(-1)
    w1, w2 = sps.expit(s[:, 0] - s[:, 1]), sps.expit(s[:, 1] - s[:, 0])
    T = 4.0
    kap, tail = V.eval_cond(keys, 0, q, T, with_tail=True)
    d = abs(keys[0, 4] - keys[1, 4])
    allow = 1e-14 * (np.abs(s).sum(1) + 1.0) * 2.0
    assert np.all(np.abs(kap - w1 * w2 * d * np.abs(s).sum(1)) <= 1e-11 * kap + allow)
    n_light = (w1 < np.exp(-T)).astype(float) + (w2 < np.exp(-T)).astype(float)
    assert 0 < (n_light > 0).sum() < len(q)
    assert np.all(np.abs(tail - n_light * w1 * w2 * d) <= 1e-11 * tail + allow)


def test_degree2_query_gradient_scale_one_key(var):
    """One key: w = 1 and O = f, so dO/dq = d + S x and qsig is the sum of
    the magnitudes of its terms; with d, S and x all non-negative that is
    dO/dq itself, which the quadratic-reproduction pin fixes."""
    rng = np.random.default_rng(75)
    keys = _below_keys2(rng, 1)
    q = rng.uniform(0.0, 1.0, (40, 3))
    qs = V.eval_qgrad_scales(keys, 2, q)[0]
    G = V.eval_qgrad(keys, 2, q)
    assert np.all(G > 0)
    assert np.allclose(qs, G, rtol=1e-13, atol=0)
    mixed = keys.copy()
    mixed[0, 5:14] *= rng.choice([-1.0, 1.0], size=9)
    qm = V.eval_qgrad_scales(mixed, 2, q)[0]
    assert np.allclose(qm, G, rtol=1e-13, atol=0)
