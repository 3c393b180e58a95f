"""The allocation-free fit step (efunc_fit_step_static) against
efunc_fit_step on a context, through the C ABI.

Two calls in a row share the library's fixed per-GPU scratch array: the
tiny sphere workload (8^3 lattice, 65,536 points) and then a smaller one
(6^3 lattice, 4,097 points, a ragged last tile), so the second call runs on
what the first left in the array.  Each call's loss, gradient and AdamW
update are compared with those of the context entry point on the same
inputs and with the FP64 oracle (global definition) to the parity
tolerances.
"""
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


def _step_ctx(E, R, th, q, o):
    n = th.size
    with E.Engine(R, len(q)) as eng:
        tth = PT.to_dev(th)
        m = torch.zeros(n, device=PT.DEV)
        v = torch.zeros(n, device=PT.DEV)
        loss = torch.zeros(2, device=PT.DEV, dtype=torch.float64)
        eng.fit_step(tth, m, v, 1, PT.to_dev(q), PT.to_dev(o), loss)
        torch.cuda.synchronize()
        return tuple(x.cpu().numpy() for x in (tth, m, v, loss))


def _step_static(E, R, th, q, o):
    n = th.size
    cfg = E.efunc_default_config(R)
    tth = PT.to_dev(th)
    m = torch.zeros(n, device=PT.DEV)
    v = torch.zeros(n, device=PT.DEV)
    loss = torch.zeros(2, device=PT.DEV, dtype=torch.float64)
    E.efunc_fit_step_static(cfg, tth, m, v, 1, PT.to_dev(q), PT.to_dev(o), loss)
    torch.cuda.synchronize()
    return tuple(x.cpu().numpy() for x in (tth, m, v, loss))


def _check_pair(R, th, q, o, got, ctx):
    n = th.size
    th1, m1, v1, loss = got
    th_c, m_c, _, loss_c = ctx
    ref = orc.fit_step(orc.Grid(R=R), th, np.zeros(n), np.zeros(n), 1, q, o)
    for lv, k in ((loss, "loss"), (loss_c, "loss")):
        assert abs(lv[0] - ref[k]) <= 1e-5 * ref[k]
        assert abs(lv[1] - ref["l1"]) <= 1e-5 * ref["l1"]
    assert abs(loss[0] - loss_c[0]) <= 1e-5 * loss_c[0]
    assert abs(loss[1] - loss_c[1]) <= 1e-5 * loss_c[1]
    g = m1.astype(np.float64) / (1.0 - np.float32(0.9))
    g_c = m_c.astype(np.float64) / (1.0 - np.float32(0.9))
    O, _, _ = PT.oracle_values(R, th, q)
    _, ar, br = PT.oracle_grad(R, th, q, 2 * (O - o) / len(q))
    PT.check_grad(g, ref["grad"], ar, br)
    PT.check_grad(g_c, ref["grad"], ar, br)
    # the two entry points: each within the tolerance of the definition
    PT.check_grad(g, g_c, 2 * ar, 2 * br, rtol=1e-4)
    th_ref, _, _ = orc.adam(th.reshape(-1), np.zeros(n), np.zeros(n), g.reshape(-1), 1)
    assert np.all(np.abs(th1.reshape(-1) - th_ref) <= 4 * PT.ulp32(th_ref) + 1e-6 * 6e-4)
    b2 = float(np.float32(0.999))
    assert np.allclose(v1.reshape(-1), (1 - b2) * g.reshape(-1) ** 2, rtol=1e-5, atol=1e-37)
    # where the gradient is far from zero, both steps move theta the same way
    big = np.abs(g_c.reshape(-1)) > 1e-3 * np.abs(g_c).max()
    assert np.array_equal(np.sign(th1.reshape(-1) - th.reshape(-1))[big],
                          np.sign(th_c.reshape(-1) - th.reshape(-1))[big])


def test_static_fit_step_matches_context_twice_then_smaller(E):
    w = W.get("sphere_r8")
    # first call: the tiny sphere workload at full size
    R1 = 8
    q1, o1 = W.make_batch(w, 0)
    th1 = W.perturbed_theta(R1, 16)
    got1 = _step_static(E, R1, th1, q1, o1)
    ctx1 = _step_ctx(E, R1, th1, q1, o1)
    _check_pair(R1, th1, q1, o1, got1, ctx1)
    # second call: smaller lattice and fewer points in the same scratch array
    R2, J2 = 6, 4097
    q2, o2 = W.make_batch(w, 5, J=J2)
    th2 = W.perturbed_theta(R2, 9)
    got2 = _step_static(E, R2, th2, q2, o2)
    ctx2 = _step_ctx(E, R2, th2, q2, o2)
    _check_pair(R2, th2, q2, o2, got2, ctx2)


def test_static_fit_step_limits(E):
    """Sizes beyond the scratch array are refused before any launch; J = 0
    only sets up the device."""
    R = 32
    cfg = E.efunc_default_config(R)
    n = R ** 3 * 13
    th = torch.zeros(n, device=PT.DEV)
    m = torch.zeros(n, device=PT.DEV)
    v = torch.zeros(n, device=PT.DEV)
    q = torch.zeros(1 << 21, 3, device=PT.DEV)
    o = torch.zeros(1 << 21, device=PT.DEV)
    with pytest.raises(E.EfuncError) as ei:
        E.efunc_fit_step_static(cfg, th, m, v, 1, q, o)
    assert ei.value.code == E.EFUNC_ESIZE
    E.efunc_fit_step_static(cfg, th, m, v, 1, q[:0], o[:0])
    cfg.check_finite = 1
    with pytest.raises(E.EfuncError) as ei:
        E.efunc_fit_step_static(cfg, th, m, v, 1, q[:16], o[:16])
    assert ei.value.code == E.EFUNC_EUNSUPPORTED
    torch.cuda.synchronize()
    assert not th.any() and not m.any() and not v.any()
