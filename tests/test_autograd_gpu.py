"""The torch.autograd.Function wrapper: gradients against the FP64 oracle
and against finite differences of the engine's own forward, including 1000
sampled parameters on the 128^3 lattice."""
import numpy as np
import pytest
import torch

import oracle as orc
import workloads as W
from tests import parity as PT

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def E():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2505_21319_amd import efunc
    efunc.lib()
    return efunc


def test_autograd_matches_oracle(E):
    from paper_2505_21319_amd.autograd import efunc_apply
    R = 8
    w = W.get("sphere_r8")
    q, o = W.make_batch(w, 7, J=20000)
    th = W.perturbed_theta(R, 61)
    with E.Engine(R, len(q)) as eng:
        T = PT.to_dev(th).requires_grad_(True)
        Q = PT.to_dev(q)
        O = efunc_apply(T, Q, eng)
        loss = ((O - PT.to_dev(o)) ** 2).mean()
        loss.backward()
        G = T.grad.cpu().numpy()
        Ov = O.detach().cpu().numpy()
    ref = PT.reference(R, th, q)
    PT.check_eval(Ov, None, ref)
    gr, ar, br = PT.oracle_grad(R, th, q, 2 * (ref["O"] - o) / len(q))
    PT.check_grad(G, gr, ar, br)


def test_autograd_query_gradient(E):
    from paper_2505_21319_amd.autograd import efunc_apply
    R = 6
    w = W.get("sphere_r8")
    q, _ = W.make_batch(w, 8, J=3000)
    th = W.perturbed_theta(R, 62, rho0=5.0)
    with E.Engine(R, len(q)) as eng:
        Q = PT.to_dev(q).requires_grad_(True)
        O = efunc_apply(PT.to_dev(th), Q, eng)
        O.sum().backward()
        gq = Q.grad.cpu().numpy().astype(np.float64)
    worst = PT.check_qgrad(gq, PT.qgrad_reference(orc.build_keys(orc.Grid(R=R), th), q))
    print(f"dL/dq worst err / tolerance {worst:.3g}")


def _key_centre(th, R, i):
    """Centre of the key that parameter index i belongs to (vertex or moved)."""
    v, ch = divmod(int(i), 13)
    t = np.linspace(-1, 1, R).astype(np.float32).astype(np.float64)
    ix, iy, iz = v // (R * R), (v // R) % R, v % R
    c = np.array([t[ix], t[iy], t[iz]])
    if ch >= 5:
        c = c + th.reshape(-1, 13)[v, 5:8].astype(np.float64)
    return c


def _fd_check(R, th, q, gO, idx, eng, W):
    """Central differences (Richardson-extrapolated) of sum_j gO_j O_j(theta)
    in each parameter of idx, from per-query differences of the engine's
    float32 outputs summed in FP64 over the queries the key can reach; every
    other query's output does not depend on the parameter.  Returns the
    estimates and their rounding-noise scale."""
    tth = PT.to_dev(th)
    tq = PT.to_dev(q)
    flat = tth.view(-1)
    reach = (W + 2) * (2.0 / (R - 1)) * np.sqrt(3.0)
    out, noise = [], []
    for i in idx:
        ch = int(i) % 13
        h = 1e-2 if ch in (0, 1, 2, 3, 8, 9, 10, 11) else (1e-3 if ch in (4, 12) else 2e-4)
        near = np.flatnonzero(np.linalg.norm(q - _key_centre(th, R, i), axis=1) <= reach + 4 * h)
        v0 = float(flat[i])

        def D(hh):
            flat[i] = v0 + hh
            Op, _, _, _ = eng.eval(tth, tq, with_lse=False)
            flat[i] = v0 - hh
            Om, _, _, _ = eng.eval(tth, tq, with_lse=False)
            flat[i] = v0
            span = float(np.float32(v0 + hh)) - float(np.float32(v0 - hh))
            d = (Op.double() - Om.double()).cpu().numpy()[near]
            return float(gO[near] @ d) / span, (Op.double().cpu().numpy()[near], span)

        d1, (O1, s1) = D(h)
        d2, (O2, s2) = D(h / 2)
        out.append((4 * d2 - d1) / 3)
        ulp = np.spacing(np.abs(O2).astype(np.float32)).astype(np.float64)
        noise.append(float(np.abs(gO[near]) @ (8 * ulp)) / s2)
    return np.array(out), np.array(noise)


@pytest.mark.parametrize("R,J,n_params", [(16, 20000, 200), (128, 65536, 1000)])
def test_autograd_finite_differences_sampled_params(E, R, J, n_params):
    """1000 sampled parameters at 128^3 (and 200 at 16^3): the backward
    against central differences of the forward."""
    from paper_2505_21319_amd.autograd import efunc_apply
    w = W.get("csg256_r128" if R == 128 else "csg16_r32")
    q, o = W.make_batch(w, 3, J=J, device=PT.DEV)
    rng = np.random.default_rng(R)
    th = W.perturbed_theta(R, 63, rho0=7.0, rho_spread=0.3, offset_cells=0.4)
    gO = rng.standard_normal(J)
    with E.Engine(R, J) as eng:
        T = PT.to_dev(th).requires_grad_(True)
        O = efunc_apply(T, PT.to_dev(q), eng)
        O.backward(PT.to_dev(gO))
        G = T.grad.cpu().numpy().reshape(-1)
        Wn = eng.stats()["W"]
        # parameters whose key lies near some query (others have ~zero gradient)
        cand = np.flatnonzero(np.abs(G) > 1e-3 * np.abs(G).max())
        idx = rng.choice(cand, size=min(n_params, len(cand)), replace=False)
        fd, noise = _fd_check(R, th, q, gO, idx, eng, Wn)
    ch = idx % 13
    err = np.abs(fd - G[idx])
    tol = 1e-3 * np.abs(G[idx]) + 4 * noise
    bad = err > tol
    assert not bad.any(), (f"{bad.sum()} of {len(idx)} FD checks off; channels "
                           f"{np.bincount(ch[bad], minlength=13)}; worst ratio "
                           f"{(err / tol).max():.2f}")
