"""GPU parity of the model variants (degree 0/1/2 value polynomials, grid
keys only, moved keys only, fixed scales) against the FP64 variant oracle:
values, lse and query gradients of efunc_eval, parameter gradients of
efunc_grad, and one efunc_fit_step, under the global definition with the
tolerances of tests/parity.py."""
import numpy as np
import pytest
import torch

from oracle import variants as V
import workloads as W
from tests import parity as PT
from tests.test_oracle_var_pins import random_theta

pytestmark = pytest.mark.gpu

# (name, degree, grid_keys, moved_keys, learn_scale, R)
VARIANTS = [
    ("f0_grid_learned_G5", 0, 1, 0, 1, 9),
    ("f0_grid_fixed_G1", 0, 1, 0, 0, 9),
    ("f1_grid_fixed_G2", 1, 1, 0, 0, 9),
    ("f2_grid_learned_G7", 2, 1, 0, 1, 9),
    ("f2_grid_fixed_G3", 2, 1, 0, 0, 8),
    ("f0_both", 0, 1, 1, 1, 8),
    ("f2_both", 2, 1, 1, 1, 8),
    ("f1_moved_only_Full1", 1, 0, 1, 1, 7),
    ("f2_moved_only", 2, 0, 1, 1, 6),
]
RHO_FIXED = 5.0


@pytest.fixture(scope="module")
def E():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2505_21319_amd import efunc
    efunc.lib()
    V.build_var_oracle(force=False)
    return efunc


def setup(v, seed, J=6000):
    name, deg, grid, moved, learn, R = v
    m = V.Model(R=R, degree=deg, grid_keys=grid, moved_keys=moved, learn_scale=learn,
                rho_fixed=RHO_FIXED)
    th = random_theta(m, seed, rho=(4.5, 5.5), offset=0.35)
    w = W.get("sphere_r8")
    q, o = W.make_batch(w, seed % 7, J=J)
    cfg = dict(degree=deg, grid_keys=grid, offsets=moved, learn_scale=learn, rho_fixed=RHO_FIXED)
    return m, th, q.astype(np.float32), o, cfg


def reference(m, th, q):
    keys = V.build_keys(m, th)
    O, lse, sig = V.eval_global(keys, m.degree, q)
    kap, tail = V.eval_cond(keys, m.degree, q, PT.T_TAIL, with_tail=True)
    return keys, dict(O=O, lse=lse, sigma=sig, kappa=kap, tail=tail)


@pytest.mark.parametrize("v", VARIANTS, ids=[v[0] for v in VARIANTS])
def test_variant_eval_and_query_gradient(E, v):
    m, th, q, _, cfg = setup(v, 101)
    with E.Engine(m.R, len(q), **cfg) as eng:
        assert eng.nch == V.channels(m)
        O, lse, dq, nu = eng.eval(PT.to_dev(th), PT.to_dev(q), with_qgrad=True)
        torch.cuda.synchronize()
        O, lse, dq = O.cpu().numpy(), lse.cpu().numpy(), dq.cpu().numpy()
    keys, ref = reference(m, th, q)
    PT.check_eval(O, lse, ref)
    worst = PT.check_qgrad(dq, PT.qgrad_reference(keys, q, degree=m.degree))
    print(f"{v[0]}: dO/dq worst err / tolerance {worst:.3g}")


@pytest.mark.parametrize("v", VARIANTS, ids=[v[0] for v in VARIANTS])
def test_variant_grad(E, v):
    m, th, q, _, cfg = setup(v, 202)
    keys, ref = reference(m, th, q)
    dl = np.random.default_rng(203).standard_normal(len(q)) / len(q)
    with E.Engine(m.R, len(q), **cfg) as eng:
        G = eng.grad(PT.to_dev(th), PT.to_dev(q), PT.to_dev(ref["O"]), PT.to_dev(ref["lse"]),
                     PT.to_dev(dl))
        torch.cuda.synchronize()
        G = G.cpu().numpy()
    gk, ak, bk = V.grad_global(keys, m.degree, q, dl, T=PT.T_TAIL)
    nch = V.channels(m)
    PT.check_grad(G, V.grad_theta(m, th, gk), V.grad_theta(m, th, ak), V.grad_theta(m, th, bk), nch=nch)


@pytest.mark.parametrize("v", [VARIANTS[3], VARIANTS[6], VARIANTS[7]], ids=["f2_grid", "f2_both", "f1_moved"])
def test_variant_fit_step(E, v):
    m, th, q, o, cfg = setup(v, 303)
    n = th.size
    with E.Engine(m.R, len(q), **cfg) as eng:
        tth = PT.to_dev(th)
        mm = torch.zeros(n, device=PT.DEV)
        vv = torch.zeros(n, device=PT.DEV)
        loss = torch.zeros(2, device=PT.DEV, dtype=torch.float64)
        eng.fit_step(tth, mm, vv, 1, PT.to_dev(q), PT.to_dev(o), loss)
        torch.cuda.synchronize()
        m1, loss = mm.cpu().numpy(), loss.cpu().numpy()
    ref = V.fit_step(m, th, np.zeros(n), np.zeros(n), 1, q, o)
    assert abs(loss[0] - ref["loss"]) <= 1e-5 * ref["loss"]
    keys = V.build_keys(m, th)
    _, ak, bk = V.grad_global(keys, m.degree, q, 2 * (ref["O"] - o) / len(q), T=PT.T_TAIL)
    g_gpu = m1.astype(np.float64) / (1.0 - np.float32(0.9))
    PT.check_grad(g_gpu, ref["grad"], V.grad_theta(m, th, ak), V.grad_theta(m, th, bk),
                  nch=V.channels(m))


def test_variant_init_params_layout(E):
    """init_params on a degree-2, moved-only model: rho channels, zero values,
    mean-shift offsets in the moved Delta channels."""
    from oracle import meanshift, Grid
    R = 6
    m = V.Model(R=R, degree=2, grid_keys=0, moved_keys=1, learn_scale=1)
    L = V.layout(m)
    surf = W.surface_points(W.get("sphere_r8"), 512, seed=5)
    with E.Engine(R, 16, degree=2, grid_keys=0, offsets=1) as eng:
        th = torch.full((m.I * L["nch"],), 9.0, device=PT.DEV)
        eng.init_params(th, PT.to_dev(surf.astype(np.float32)), 100.0, 6.5)
        torch.cuda.synchronize()
        th = th.cpu().numpy().reshape(m.I, L["nch"])
    ref = meanshift(Grid(R=R), surf, 100.0).reshape(m.I, 3)
    d0 = L["moved_delta"]
    assert np.allclose(th[:, d0:d0 + 3], ref, rtol=0, atol=2e-5)
    assert np.all(th[:, L["moved_rho"]] == np.float32(6.5))
    vals = th[:, L["moved_values"]:L["moved_values"] + 10]
    assert not vals.any()


def test_batch_rejects_mixed_degrees(E):
    c1 = E.efunc_default_config(6)
    c2 = E.efunc_default_config(6)
    c2.degree = 2
    with pytest.raises(E.EfuncError) as ei:
        E.efunc_batch_create([c1, c2], [10, 10])
    assert ei.value.code == E.EFUNC_EUNSUPPORTED


def test_batch_degree2_matches_single_shape(E):
    """A batch of degree-2 shapes against single-shape fit steps."""
    shapes = [(6, 3000), (8, 5000)]
    data = []
    for i, (R, J) in enumerate(shapes):
        m = V.Model(R=R, degree=2)
        th = random_theta(m, 400 + i, rho=(4.5, 5.5), offset=0.35)
        q, o = W.make_batch(W.get("sphere_r8"), i, J=J)
        data.append((m, th, q, o))
    ths = [PT.to_dev(d[1]).reshape(-1).clone() for d in data]
    ms = [torch.zeros_like(t) for t in ths]
    vs = [torch.zeros_like(t) for t in ths]
    loss = torch.zeros(len(data), 2, device=PT.DEV, dtype=torch.float64)
    with E.BatchEngine([R for R, _ in shapes], [J for _, J in shapes], degree=2) as B:
        B.bind(ths, ms, vs, [PT.to_dev(d[2]) for d in data], [PT.to_dev(d[3]) for d in data], loss)
        B.fit(1, 1)
        torch.cuda.synchronize()
    for i, (m, th, q, o) in enumerate(data):
        ts = PT.to_dev(th).reshape(-1).clone()
        m1, v1 = torch.zeros_like(ts), torch.zeros_like(ts)
        ls = torch.zeros(2, device=PT.DEV, dtype=torch.float64)
        with E.Engine(m.R, len(q), degree=2) as eng:
            eng.fit_step(ts, m1, v1, 1, PT.to_dev(q), PT.to_dev(o), ls)
            torch.cuda.synchronize()
        assert np.allclose(loss[i].cpu().numpy(), ls.cpu().numpy(), rtol=1e-5, atol=0)
        a, b = ms[i].cpu().numpy(), m1.cpu().numpy()
        scale = np.abs(b).reshape(-1, V.channels(m)).max(axis=0)
        err = np.abs(a - b).reshape(-1, V.channels(m))
        assert np.all(err <= 1e-4 * np.abs(b.reshape(-1, V.channels(m))) + 1e-5 * scale)
