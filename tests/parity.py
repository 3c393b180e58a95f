"""Shared helpers of the GPU parity tests: device transfer, the oracle
reference for a problem, and the tolerances.

Tolerances (FP32 GPU against the FP64 oracle):
  values     |O_gpu - O_ref| <= 1e-5 * sigma_j + 8 u kappa_j, with
             sigma_j = sum_a w_a |f_a| (the running-error scale of the blended
             polynomials; plain relative error is meaningless where O ~ 0 on
             the surface) and kappa_j = sum_a w_a |s_a| |f_a - O_j| (a float32
             logit carries a few ulps u = 2^-24 of |s_a|; only coarse lattices
             with large beta, |s| ~ 100, make this term matter).
  lse        |lse_gpu - lse_ref| <= 1e-5 * (1 + |lse_ref|).
  gradients  |g_gpu - g_ref| <= 1e-4 * A + B + 1e-6 * max_channel(A), A the
             sum of |contributions| per entry and B its part from pairs with
             weight below e^-T (T = 20), which the engine may omit.
  truncation the engine drops pairs whose weight is below e^-T relative to
             the query's normaliser, so values also allow
             tail_j = sum over such keys of w_a |f_a - O_j|.
  Adam       theta from the GPU's own gradient through the oracle's AdamW
             agrees within 4 float32 ulps of theta plus 1e-6 lr.
  dO/dq      per query and component |G_gpu - G_ref| <= 1e-4 qsig + 8 u qkap
             + qtail (oracle_eval_qgrad_scales): qsig the magnitudes of the
             terms of Eq. func-normal, qkap their first-order change under
             float32 rounding of logits, values and O, qtail the most that
             omitting pairs below e^-T can change the sum.
"""
from __future__ import annotations

import numpy as np
import torch

import oracle as orc

DEV = "cuda:0"


def to_dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).to(DEV)


U32 = 2.0 ** -24


T_CUT = 20.0
# the allowance is taken at e^-(T - 0.1): the engine decides "below e^-T" from
# its float32 lse, which agrees with the FP64 one to ~1e-5 in the exponent
T_TAIL = T_CUT - 0.1


def check_values(O, O_ref, sigma, rtol=1e-5, what="O", kappa=None, tail=None):
    O = np.asarray(O, dtype=np.float64)
    err = np.abs(O - O_ref)
    tol = rtol * sigma + 1e-30
    if kappa is not None:
        tol = tol + 8 * U32 * kappa
    if tail is not None:
        tol = tol + tail
    bad = err > tol
    if bad.any():
        k = int(np.argmax(err / tol))
        raise AssertionError(f"{what}: {bad.sum()} of {len(O)} outside {rtol} sigma; worst j={k} "
                             f"gpu={O[k]!r} ref={O_ref[k]!r} sigma={sigma[k]!r}")
    return float((err / np.maximum(sigma, 1e-300)).max()) if len(O) else 0.0


def check_lse(lse, lse_ref, rtol=1e-5):
    lse = np.asarray(lse, dtype=np.float64)
    err = np.abs(lse - lse_ref)
    tol = rtol * (1.0 + np.abs(lse_ref))
    assert np.all(err <= tol), f"lse: worst {np.max(err / tol)} x tolerance"


def check_grad(g, g_ref, A, B=None, rtol=1e-4, floor=1e-6, nch=13):
    g = np.asarray(g, dtype=np.float64).reshape(-1, nch)
    g_ref = g_ref.reshape(-1, nch)
    A = A.reshape(-1, nch)
    tol = rtol * A + floor * A.max(axis=0, keepdims=True) + 1e-30
    if B is not None:
        tol = tol + B.reshape(-1, nch)
    err = np.abs(g - g_ref)
    bad = err > tol
    if bad.any():
        i, c = np.unravel_index(np.argmax(err / tol), err.shape)
        raise AssertionError(f"grad: {bad.sum()} entries out of tolerance; worst vertex {i} ch {c}: "
                             f"gpu={g[i, c]!r} ref={g_ref[i, c]!r} A={A[i, c]!r}")
    return float((err / (A + 1e-300)).max())


def oracle_values(R, theta, q, offsets=1):
    g = orc.Grid(R=R, offsets=offsets)
    keys = orc.build_keys(g, theta)
    return orc.eval_global(keys, q)


def oracle_kappa(R, theta, q, offsets=1):
    g = orc.Grid(R=R, offsets=offsets)
    return orc.eval_cond(orc.build_keys(g, theta), q)


def reference(R, theta, q, offsets=1):
    """Oracle values, lse and both error scales under the global definition."""
    g = orc.Grid(R=R, offsets=offsets)
    keys = orc.build_keys(g, theta)
    O, lse, sig = orc.eval_global(keys, q)
    kap, tail = orc.eval_cond(keys, q, T_TAIL, with_tail=True)
    return dict(O=O, lse=lse, sigma=sig, kappa=kap, tail=tail)


def check_eval(O, lse, ref):
    """Values and lse against reference() with the tolerances above; returns
    the worst |err| / (1e-5 sigma + 8 u kappa)."""
    worst = check_values(O, ref["O"], ref["sigma"], kappa=ref["kappa"], tail=ref["tail"])
    if lse is not None:
        check_lse(lse, ref["lse"])
    return worst


def oracle_grad(R, theta, q, dLdO, offsets=1):
    """(gradient, A, B) in theta layout under the global definition."""
    g = orc.Grid(R=R, offsets=offsets)
    keys = orc.build_keys(g, theta)
    gk, ak, bk = orc.grad_global(keys, q, dLdO, T=T_TAIL)
    return (orc.grad_theta(g, theta, gk), orc.grad_theta(g, theta, ak),
            orc.grad_theta(g, theta, bk))


def qgrad_reference(keys, q, degree=None):
    """dO/dq of the global definition with its tolerance scales, and the value
    reference whose tolerance the O in Eq. func-normal carries over; degree
    selects the variant oracle (None: the first-order 13-channel oracle)."""
    if degree is None:
        G = orc.eval_qgrad(keys, q)
        qs, qk, qt, qb = orc.eval_qgrad_scales(keys, q, T_TAIL)
        _, _, sig = orc.eval_global(keys, q)
        kap, tail = orc.eval_cond(keys, q, T_TAIL, with_tail=True)
    else:
        from oracle import variants as V
        G = V.eval_qgrad(keys, degree, q)
        qs, qk, qt, qb = V.eval_qgrad_scales(keys, degree, q, T_TAIL)
        _, _, sig = V.eval_global(keys, degree, q)
        kap, tail = V.eval_cond(keys, degree, q, T_TAIL, with_tail=True)
    return dict(G=G, qsig=qs, qkap=qk, qtail=qt, qbx=qb, sigma=sig, kappa=kap, tail=tail)


def check_qgrad(G, ref, rtol=1e-4):
    """Element-wise query-gradient check against qgrad_reference():
    |G - G_ref| <= 1e-4 qsig + 8 u qkap + qtail + qbx tol_O, with tol_O the
    value tolerance of check_values (an error of O moves G by at most qbx
    times it).  Returns the worst |err| / tolerance."""
    G = np.asarray(G, dtype=np.float64).reshape(-1, 3)
    err = np.abs(G - ref["G"])
    tol_O = 1e-5 * ref["sigma"] + 8 * U32 * ref["kappa"] + ref["tail"]
    tol = rtol * ref["qsig"] + 8 * U32 * ref["qkap"] + ref["qtail"] + ref["qbx"] * tol_O[:, None] + 1e-30
    bad = err > tol
    if bad.any():
        j, c = np.unravel_index(np.argmax(err / tol), err.shape)
        raise AssertionError(f"dO/dq: {bad.sum()} of {err.size} components out of tolerance; worst "
                             f"query {j} axis {c}: gpu={G[j, c]!r} ref={ref['G'][j, c]!r} "
                             f"qsig={ref['qsig'][j, c]!r} tol={tol[j, c]!r}")
    return float((err / tol).max()) if err.size else 0.0


def ulp32(x):
    x = np.abs(np.asarray(x, dtype=np.float32))
    return np.spacing(x).astype(np.float64)
