"""Batched multi-shape fitting (efunc_batch_*): every shape's iteration
against the oracle (small shapes) and against the single-shape
efunc_fit_step (the same arithmetic up to the order of float additions),
HIP-graph replays against direct launches, tuning invariance and the
autotuner, and the argument errors of the batch ABI."""
import numpy as np
import pytest
import torch

import oracle as orc
import workloads as W
from tests import parity as PT

pytestmark = pytest.mark.gpu

LR = 6e-4


@pytest.fixture(scope="module")
def E():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2505_21319_amd import efunc
    efunc.lib()
    return efunc


def _shapes(name, n, seed, R_range, J_range):
    ws = W.batch_set(name, n, seed, R_range, J_range, prims_range=(2, 12))
    data = []
    for i, w in enumerate(ws):
        q, o = W.make_batch(w, 0, device=PT.DEV)
        th = W.perturbed_theta(w.R, 500 + i, rho0=6.0 + 0.25 * i, offset_cells=0.4)
        data.append((w, q, o, th))
    return data


@pytest.fixture(scope="module")
def small():
    # R from 5 to 12, J from 2,000 to 20,000: the oracle's global fit is cheap
    return _shapes("bsmall", 4, 7, (5, 12), (2000, 20000))


@pytest.fixture(scope="module")
def medium():
    # R from 12 to 33, J from 2^14 to 2^17
    return _shapes("bmed", 6, 11, (12, 33), (1 << 14, 1 << 17))


def _state(data):
    th = [PT.to_dev(d[3]).reshape(-1).clone() for d in data]
    m = [torch.zeros_like(t) for t in th]
    v = [torch.zeros_like(t) for t in th]
    q = [PT.to_dev(d[1]) for d in data]
    o = [PT.to_dev(d[2]) for d in data]
    loss = torch.zeros(len(data), 2, device=PT.DEV, dtype=torch.float64)
    return th, m, v, q, o, loss


def _grad_tol_check(g, gr, label):
    """Two float32 sums of the same terms in different orders."""
    scale = np.abs(gr).reshape(-1, 13).max(axis=0)
    err = np.abs(g.reshape(-1, 13) - gr.reshape(-1, 13))
    ok = err <= 1e-4 * np.abs(gr.reshape(-1, 13)) + 1e-5 * scale
    assert ok.all(), f"{label}: {(~ok).sum()} gradient entries differ"


def _theta_check(a, b, label, steps=1):
    """AdamW moves every parameter by about lr per step; parameters whose
    gradient is at rounding level may move differently (its sign is not
    determined), so beyond a tiny absolute bound at most 1 % may differ, and
    none by more than 2 lr per step."""
    d = np.abs(a - b)
    assert d.max() <= 2 * LR * steps + 1e-6, f"{label}: max theta difference {d.max()}"
    frac = np.mean(d > 4 * np.spacing(np.abs(b).astype(np.float32)) + 1e-7)
    assert frac <= 0.01, f"{label}: {frac:.4f} of the parameters differ"


def test_batch_fit_step_matches_oracle(E, small):
    """One batched iteration of four small shapes (R 5..12): each shape's
    loss and gradient against the oracle's global fit, AdamW on the GPU's
    own gradient against the oracle's AdamW."""
    th, m, v, q, o, loss = _state(small)
    with E.BatchEngine([d[0].R for d in small], [d[0].J for d in small]) as B:
        B.bind(th, m, v, q, o, loss)
        B.fit(1, 1)
        torch.cuda.synchronize()
    for i, (w, qn, on, th0) in enumerate(small):
        R, n = w.R, th0.size
        ref = orc.fit_step(orc.Grid(R=R), th0, np.zeros(n), np.zeros(n), 1, qn, on)
        L = loss[i].cpu().numpy()
        assert abs(L[0] - ref["loss"]) <= 1e-5 * ref["loss"], f"shape {i} loss"
        assert abs(L[1] - ref["l1"]) <= 1e-5 * ref["l1"], f"shape {i} L1"
        g_gpu = m[i].cpu().numpy().astype(np.float64) / (1.0 - np.float32(0.9))
        O, _, _ = PT.oracle_values(R, th0, qn)
        _, ar, br = PT.oracle_grad(R, th0, qn, 2 * (O - on) / len(qn))
        PT.check_grad(g_gpu, ref["grad"], ar, br)
        th_ref, _, _ = orc.adam(th0.reshape(-1), np.zeros(n), np.zeros(n), g_gpu, 1)
        assert np.all(np.abs(th[i].cpu().numpy() - th_ref) <= 4 * PT.ulp32(th_ref) + 1e-6 * LR)


def test_batch_matches_single_shape_fit_steps(E, medium):
    """Three batched iterations against three efunc_fit_step calls per shape
    (R 12..33, J 2^14..2^17): losses of every step, moments and parameters."""
    th, m, v, q, o, loss = _state(medium)
    losses = []
    with E.BatchEngine([d[0].R for d in medium], [d[0].J for d in medium]) as B:
        B.bind(th, m, v, q, o, loss)
        for t in range(1, 4):
            B.fit(t, 1)
            losses.append(loss.cpu().numpy().copy())
        torch.cuda.synchronize()
    for i, (w, qn, on, th0) in enumerate(medium):
        ts = PT.to_dev(th0).reshape(-1).clone()
        ms = torch.zeros_like(ts)
        vs = torch.zeros_like(ts)
        ls = torch.zeros(2, device=PT.DEV, dtype=torch.float64)
        with E.Engine(w.R, w.J) as eng:
            for t in range(1, 4):
                eng.fit_step(ts, ms, vs, t, q[i], o[i], ls)
                Ls = ls.cpu().numpy()
                Lb = losses[t - 1][i]
                assert np.allclose(Lb, Ls, rtol=1e-5, atol=0), f"shape {i} step {t}: {Lb} vs {Ls}"
            torch.cuda.synchronize()
        _grad_tol_check(m[i].cpu().numpy(), ms.cpu().numpy(), f"shape {i} first moment")
        _theta_check(th[i].cpu().numpy(), ts.cpu().numpy(), f"shape {i}", steps=3)


def test_batch_graph_replays_match_direct_launches(E, medium):
    """A captured iteration replayed step by step, with eager torch work and
    synchronisations between the replays, against directly launched steps
    from the same start: every replay's losses and parameters."""
    ref_th, ref_loss = [], []
    th, m, v, q, o, loss = _state(medium)
    Rs, Js = [d[0].R for d in medium], [d[0].J for d in medium]
    with E.BatchEngine(Rs, Js) as B:
        B.bind(th, m, v, q, o, loss)
        for t in range(1, 5):
            B.fit(t, 1, use_graph=False)
            ref_loss.append(loss.cpu().numpy().copy())
            ref_th.append([x.cpu().numpy().copy() for x in th])
    th, m, v, q, o, loss = _state(medium)
    with E.BatchEngine(Rs, Js) as B:
        B.bind(th, m, v, q, o, loss)
        junk = torch.randn(1 << 20, device=PT.DEV)
        for t in range(1, 5):
            B.fit(t, 1, use_graph=True)
            torch.cuda.synchronize()
            s = float(junk.sum()) + float((junk * junk).sum())  # eager work between replays
            assert np.isfinite(s)
            L = loss.cpu().numpy()
            assert np.allclose(L, ref_loss[t - 1], rtol=1e-5, atol=0), f"replay {t}"
            for i in range(len(medium)):
                _theta_check(th[i].cpu().numpy(), ref_th[t - 1][i], f"replay {t} shape {i}", steps=t)
        # several steps in one call replay the same graph
        B.fit(5, 3, use_graph=True)
        torch.cuda.synchronize()
        assert np.all(np.isfinite(loss.cpu().numpy()))


def test_batch_tuning_does_not_change_results(E, medium):
    """Every tuning candidate gives the same first step (gradient from the
    first moment) as the default, up to the order of float additions."""
    Rs, Js = [d[0].R for d in medium], [d[0].J for d in medium]
    base = None
    for cap, grp, bpc in [(512, 2, 8), (128, 0, 4), (256, 1, 2), (128, 1, 8), (512, 0, 1), (256, 2, 4)]:
        th, m, v, q, o, loss = _state(medium)
        with E.BatchEngine(Rs, Js) as B:
            B.set_tuning(cap, grp, bpc)
            assert B.tuning() == {"tile_cap": cap, "group_cells": grp, "blocks_per_cu": bpc}
            B.bind(th, m, v, q, o, loss)
            B.fit(1, 1)
            torch.cuda.synchronize()
            got = ([x.cpu().numpy() for x in m], loss.cpu().numpy())
        if base is None:
            base = got
            continue
        assert np.allclose(got[1], base[1], rtol=1e-5, atol=0)
        for i in range(len(medium)):
            _grad_tol_check(got[0][i], base[0][i], f"tuning {cap},{grp},{bpc} shape {i}")


def test_batch_autotune_restores_state(E, medium):
    th, m, v, q, o, loss = _state(medium)
    Rs, Js = [d[0].R for d in medium], [d[0].J for d in medium]
    th0 = [x.clone() for x in th]
    with E.BatchEngine(Rs, Js) as B:
        B.bind(th, m, v, q, o, loss)
        best, ms = B.autotune(reps=1)
        assert best["tile_cap"] in (128, 256, 512) and best["group_cells"] in (0, 2)
        assert best["blocks_per_cu"] in (4, 8) and ms > 0
        assert B.tuning() == best
        for a, b in zip(th, th0):
            assert torch.equal(a, b)
        assert not any(x.any() for x in m) and not any(x.any() for x in v)
        B.fit(1, 1)
        torch.cuda.synchronize()
        assert np.all(np.isfinite(loss.cpu().numpy()))


def test_single_context_tuning_eval_parity(E):
    """The single-shape entry points under non-default tunings."""
    R = 12
    w = W.get("sphere_r8")
    q, _ = W.make_batch(w, 4, J=30000)
    th = W.perturbed_theta(R, 71, rho0=6.5)
    ref = PT.reference(R, th, q)
    for cap, grp, bpc in [(128, 0, 4), (256, 1, 1), (128, 2, 8)]:
        with E.Engine(R, len(q)) as eng:
            eng.set_tuning(cap, grp, bpc)
            O, lse, _, nu = eng.eval(PT.to_dev(th), PT.to_dev(q))
            torch.cuda.synchronize()
            PT.check_eval(O.cpu().numpy(), lse.cpu().numpy(), ref)


def test_batch_argument_errors(E):
    from paper_2505_21319_amd.efunc import EfuncError
    with E.BatchEngine([6, 7], [100, 200]) as B:
        with pytest.raises(EfuncError) as ei:
            B.fit(1, 1)
        assert ei.value.code == E.EFUNC_EINVAL
        th = [torch.zeros(6 ** 3 * 13, device=PT.DEV), torch.zeros(7 ** 3 * 13, device=PT.DEV)]
        m = [torch.zeros_like(t) for t in th]
        v = [torch.zeros_like(t) for t in th]
        q = [torch.zeros(100, 3, device=PT.DEV), torch.zeros(201, 3, device=PT.DEV)]
        o = [torch.zeros(100, device=PT.DEV), torch.zeros(201, device=PT.DEV)]
        with pytest.raises(EfuncError) as ei:
            B.bind(th, m, v, q, o)
        assert ei.value.code == E.EFUNC_ESIZE
        with pytest.raises(EfuncError) as ei:
            B.set_tuning(100, 1, 8)
        assert ei.value.code == E.EFUNC_EINVAL
        with pytest.raises(EfuncError) as ei:
            B.set_tuning(512, 1, 9)
        assert ei.value.code == E.EFUNC_EINVAL
        with pytest.raises(EfuncError) as ei:
            B.set_tuning(512, 3, 8)
        assert ei.value.code == E.EFUNC_EINVAL
    cfg = E.efunc_default_config(6)
    cfg.check_finite = 1
    with pytest.raises(EfuncError) as ei:
        E.efunc_batch_create([cfg], [10])
    assert ei.value.code == E.EFUNC_EUNSUPPORTED
