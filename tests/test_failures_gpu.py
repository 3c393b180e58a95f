"""Failure detection at the C ABI on the GPU.  Every case here is rejected
on the host before a kernel is enqueued: non-finite inputs under
check_finite, a minibatch beyond the context's max_points, misaligned
pointers, and parameter tensors sized for another lattice (checked by the
binding, since a C pointer carries no extent)."""
import ctypes as C

import numpy as np
import pytest
import torch

import workloads as W
from tests import parity as PT

pytestmark = pytest.mark.gpu

R, J = 6, 2000


@pytest.fixture(scope="module")
def E():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2505_21319_amd import efunc
    efunc.lib()
    return efunc


def _inputs(seed=0):
    q, o = W.make_batch(W.get("sphere_r8"), seed, J=J)
    th = W.perturbed_theta(R, 3 + seed)
    return PT.to_dev(th), PT.to_dev(q), PT.to_dev(o)


def _calls(E, eng, th, q, o, O, lse, dl):
    n = th.numel()
    m = torch.zeros(n, device=PT.DEV)
    v = torch.zeros(n, device=PT.DEV)
    g = torch.zeros(n, device=PT.DEV)
    return {
        "eval": lambda: eng.eval(th, q),
        "grad": lambda: eng.grad(th, q, O, lse, dl, g),
        "fit_step": lambda: eng.fit_step(th, m, v, 1, q, o),
        "loss_grad": lambda: eng.loss_grad(th, q, o, g),
    }


@pytest.mark.parametrize("bad", [float("nan"), float("inf"), -float("inf")], ids=["nan", "inf", "-inf"])
@pytest.mark.parametrize("where", ["theta", "q"])
def test_check_finite_rejects_nonfinite_inputs_before_launch(E, where, bad):
    th, q, o = _inputs()
    with E.Engine(R, J, check_finite=1) as eng:
        O, lse, _, _ = eng.eval(th, q)
        dl = torch.full((J,), 1.0 / J, device=PT.DEV)
        torch.cuda.synchronize()
        if where == "theta":
            th.view(-1)[4 * 13 + 9] = bad
        else:
            q.view(-1)[3 * 777 + 1] = bad
        before = th.clone()
        for name, call in _calls(E, eng, th, q, o, O, lse, dl).items():
            with pytest.raises(E.EfuncError) as ei:
                call()
            assert ei.value.code == E.EFUNC_ENONFINITE, name
            assert where in str(ei.value), (name, str(ei.value))
        torch.cuda.synchronize()
        # the rejected fit step launched nothing: theta is untouched
        assert torch.equal(th.isnan(), before.isnan())
        assert torch.equal(torch.nan_to_num(th), torch.nan_to_num(before))


@pytest.mark.parametrize("which", ["dLdO", "lse", "O"])
def test_check_finite_scans_grad_inputs(E, which):
    th, q, _ = _inputs(1)
    with E.Engine(R, J, check_finite=1) as eng:
        O, lse, _, _ = eng.eval(th, q)
        dl = torch.full((J,), 1.0 / J, device=PT.DEV)
        arr = {"dLdO": dl, "lse": lse, "O": O}[which]
        arr[123] = float("nan")
        g = torch.zeros_like(th)
        with pytest.raises(E.EfuncError) as ei:
            eng.grad(th, q, O, lse, dl, g)
        assert ei.value.code == E.EFUNC_ENONFINITE and which in str(ei.value)
        torch.cuda.synchronize()
        assert torch.count_nonzero(g) == 0


def test_check_finite_scans_targets_and_moments(E):
    th, q, o = _inputs(2)
    n = th.numel()
    with E.Engine(R, J, check_finite=1) as eng:
        m = torch.zeros(n, device=PT.DEV)
        v = torch.zeros(n, device=PT.DEV)
        o[5] = float("inf")
        with pytest.raises(E.EfuncError) as ei:
            eng.fit_step(th, m, v, 1, q, o)
        assert ei.value.code == E.EFUNC_ENONFINITE and "o[" in str(ei.value)
        o[5] = 0.0
        v[17] = float("nan")
        with pytest.raises(E.EfuncError) as ei:
            eng.fit_step(th, m, v, 1, q, o)
        assert ei.value.code == E.EFUNC_ENONFINITE and "v[" in str(ei.value)


def test_check_finite_passes_clean_inputs_and_matches_unchecked(E):
    th, q, o = _inputs(3)
    with E.Engine(R, J, check_finite=1) as a, E.Engine(R, J) as b:
        Oa, la, _, _ = a.eval(th, q)
        Ob, lb, _, _ = b.eval(th, q)
        torch.cuda.synchronize()
        ref = PT.reference(R, th.cpu().numpy(), q.cpu().numpy())
        PT.check_eval(Oa.cpu().numpy(), la.cpu().numpy(), ref)
        PT.check_eval(Ob.cpu().numpy(), lb.cpu().numpy(), ref)
        assert a.stats()["n_nonfinite"] == 0


def test_minibatch_beyond_max_points_is_rejected(E):
    th, q, o = _inputs(4)
    with E.Engine(R, J - 1) as eng:
        n = th.numel()
        for call in (lambda: eng.eval(th, q),
                     lambda: eng.fit_step(th, torch.zeros(n, device=PT.DEV), torch.zeros(n, device=PT.DEV),
                                          1, q, o),
                     lambda: eng.loss_grad(th, q, o, torch.zeros(n, device=PT.DEV))):
            with pytest.raises(E.EfuncError) as ei:
                call()
            assert ei.value.code == E.EFUNC_ESIZE and "max_points" in str(ei.value)
        # exactly max_points is accepted
        O, _, _, _ = eng.eval(th, q[:J - 1].contiguous())
        torch.cuda.synchronize()
        assert torch.isfinite(O).all()


def test_misaligned_pointers_are_rejected(E):
    th, q, _ = _inputs(5)
    L = E.lib()
    O = torch.empty(J + 1, device=PT.DEV)
    lse = torch.empty(J + 1, device=PT.DEV)
    nu = torch.zeros(2, device=PT.DEV, dtype=torch.int64)
    qq = torch.empty(3 * J + 1, device=PT.DEV)
    qq[:3 * J] = q.view(-1)
    s = torch.cuda.current_stream().cuda_stream
    with E.Engine(R, J) as eng:
        ok = L.efunc_eval(eng.ctx, th.data_ptr(), qq.data_ptr(), J, O.data_ptr(), lse.data_ptr(), None,
                          nu.data_ptr(), s)
        assert ok == E.EFUNC_OK
        torch.cuda.synchronize()
        cases = [
            (th.data_ptr() + 2, qq.data_ptr(), O.data_ptr(), lse.data_ptr(), nu.data_ptr(), b"theta"),
            (th.data_ptr(), qq.data_ptr() + 2, O.data_ptr(), lse.data_ptr(), nu.data_ptr(), b"q"),
            (th.data_ptr(), qq.data_ptr(), O.data_ptr() + 1, lse.data_ptr(), nu.data_ptr(), b"O"),
            (th.data_ptr(), qq.data_ptr(), O.data_ptr(), lse.data_ptr() + 2, nu.data_ptr(), b"lse"),
            (th.data_ptr(), qq.data_ptr(), O.data_ptr(), lse.data_ptr(), nu.data_ptr() + 4, b"n_uncertified"),
        ]
        for t, qp, op, lp, np_, name in cases:
            rc = L.efunc_eval(eng.ctx, t, qp, J, op, lp, None, np_, s)
            assert rc == E.EFUNC_EINVAL, name
            msg = L.efunc_last_error()
            assert name in msg and b"aligned" in msg, msg
        torch.cuda.synchronize()


def test_parameters_of_another_lattice_are_rejected_by_the_binding(E):
    th, q, o = _inputs(6)
    small = PT.to_dev(W.perturbed_theta(R - 1, 7))
    n = small.numel()
    with E.Engine(R, J) as eng:
        for call in (lambda: eng.eval(small, q),
                     lambda: eng.grad(small, q, q[:, 0].contiguous(), q[:, 0].contiguous(),
                                      q[:, 0].contiguous()),
                     lambda: eng.fit_step(small, torch.zeros(n, device=PT.DEV), torch.zeros(n, device=PT.DEV),
                                          1, q, o),
                     lambda: eng.loss_grad(small, q, o, torch.zeros(n, device=PT.DEV))):
            with pytest.raises(ValueError, match="theta has"):
                call()
    with E.BatchEngine([R, R], [J, J]) as b:
        ths = [th.clone(), small]
        ms = [torch.zeros_like(t) for t in ths]
        vs = [torch.zeros_like(t) for t in ths]
        with pytest.raises(ValueError, match="theta"):
            b.bind(ths, ms, vs, [q, q], [o, o])
