"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Workloads are the seeded synthetic ones of the workloads package: the tiny
sphere fit (8^3 grid, 65,536 points) at full size under the global
definition, plus ragged, degenerate and out-of-domain cases.
"""
import numpy as np
import pytest
import torch

import oracle as orc
import workloads as W
from tests import parity as PT

pytestmark = pytest.mark.gpu

MERGE = 2  # group_cells value that lets z-adjacent sparse blocks share a tile


@pytest.fixture(scope="module")
def E():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2505_21319_amd import efunc
    efunc.lib()  # fail loudly if the HIP library is missing
    return efunc


def meanshift_theta(R, w, seed=0):
    """Paper initialisation computed by the oracle: zero values, rho = 7,
    mean-shift offsets towards 16,384 surface samples."""
    th = W.plain_theta(R)
    surf = W.surface_points(w, 16384, seed=seed)
    D = orc.meanshift(orc.Grid(R=R), surf, 100.0)
    th[..., 5:8] = D.reshape(R, R, R, 3).astype(np.float32)
    return th, surf


def run_eval(E, R, th, q, max_points=None, **cfg):
    with E.Engine(R, max_points or max(len(q), 1), **cfg) as eng:
        O, lse, _, nu = eng.eval(PT.to_dev(th), PT.to_dev(q))
        torch.cuda.synchronize()
        st = eng.stats()
    return O.cpu().numpy(), lse.cpu().numpy(), int(nu.item()), st


# ------------------------------------------------------------------ init
def test_init_params_meanshift_matches_oracle(E):
    R = 8
    w = W.get("sphere_r8")
    surf = W.surface_points(w, 16384, seed=0)
    with E.Engine(R, 16) as eng:
        th = torch.empty(R, R, R, 13, device=PT.DEV)
        eng.init_params(th, PT.to_dev(surf), 100.0, 7.0)
        torch.cuda.synchronize()
        th = th.cpu().numpy()
    D = orc.meanshift(orc.Grid(R=R), surf, 100.0).reshape(R, R, R, 3)
    assert np.all(th[..., [0, 1, 2, 3, 8, 9, 10, 11]] == 0.0)
    assert np.all(th[..., [4, 12]] == 7.0)
    assert np.allclose(th[..., 5:8], D, rtol=0, atol=2e-6)


# ------------------------------------------------------------------ eval
@pytest.mark.parametrize("init", ["paper", "perturbed"])
def test_eval_sphere_r8_full(E, init):
    R = 8
    w = W.get("sphere_r8")
    q, o = W.make_batch(w, 0)
    th = meanshift_theta(R, w)[0] if init == "paper" else W.perturbed_theta(R, 3)
    O, lse, nu, st = run_eval(E, R, th, q)
    ref = PT.reference(R, th, q)
    worst = PT.check_eval(O, lse, ref)
    assert nu == 0
    print(f"worst err/sigma {worst:.2e}, W={st['W']}, tiles={st['n_tiles']}, pairs={st['pairs']}")


@pytest.mark.parametrize("J", [1, 7, 255, 257, 1000])
def test_eval_ragged_sizes(E, J):
    R = 5
    w = W.get("sphere_r8")
    q, _ = W.make_batch(w, 11, J=J)
    th = W.perturbed_theta(R, 4, rho0=5.0)
    O, lse, nu, _ = run_eval(E, R, th, q, max_points=1024)
    ref = PT.reference(R, th, q)
    PT.check_eval(O, lse, ref)


@pytest.mark.parametrize("J", [4097, 12293, 64 * 4096 + 3])
def test_eval_binning_chunk_edges(E, J):
    """Queries binned by several workgroups on a lattice whose sort keys fit
    in LDS: chunks that do not divide J (a shorter last chunk), and 65
    chunks' worth of queries folded into the 64-workgroup limit (uneven
    chunk size)."""
    R = 6
    w = W.get("sphere_r8")
    q, _ = W.make_batch(w, 12, J=J)
    th = W.perturbed_theta(R, 5, rho0=5.0)
    O, lse, nu, _ = run_eval(E, R, th, q)
    ref = PT.reference(R, th, q)
    PT.check_eval(O, lse, ref)


def test_fit_step_binning_chunk_edges(E):
    """Fit step with a ragged last binning chunk (12,293 queries, four
    workgroups): every query's target travels with it through the scatter,
    so loss and gradient match the oracle."""
    R, J = 6, 12293
    w = W.get("sphere_r8")
    q, o = W.make_batch(w, 13, J=J)
    th = W.perturbed_theta(R, 6)
    n = th.size
    with E.Engine(R, J) as eng:
        tth = PT.to_dev(th)
        m = torch.zeros(n, device=PT.DEV)
        v = torch.zeros(n, device=PT.DEV)
        loss = torch.zeros(2, device=PT.DEV, dtype=torch.float64)
        eng.fit_step(tth, m, v, 1, PT.to_dev(q), PT.to_dev(o), loss)
        torch.cuda.synchronize()
        m1, loss = m.cpu().numpy(), loss.cpu().numpy()
    ref = orc.fit_step(orc.Grid(R=R), th, np.zeros(n), np.zeros(n), 1, q, o)
    assert abs(loss[0] - ref["loss"]) <= 1e-5 * ref["loss"]
    assert abs(loss[1] - ref["l1"]) <= 1e-5 * ref["l1"]
    g_gpu = m1.astype(np.float64) / (1.0 - np.float32(0.9))
    O, _, _ = PT.oracle_values(R, th, q)
    _, ar, br = PT.oracle_grad(R, th, q, 2 * (O - o) / len(q))
    PT.check_grad(g_gpu, ref["grad"], ar, br)


def test_eval_j0_is_noop(E):
    R = 4
    with E.Engine(R, 8) as eng:
        th = PT.to_dev(W.perturbed_theta(R, 0))
        q = torch.empty(0, 3, device=PT.DEV)
        O = torch.empty(0, device=PT.DEV)
        E.efunc_eval(eng.ctx, th, q, O)
        g = torch.zeros_like(th)
        E.efunc_grad(eng.ctx, th, q, O, O, O, g)
        m, v = torch.zeros_like(th), torch.zeros_like(th)
        th0 = th.clone()
        E.efunc_fit_step(eng.ctx, th, m, v, 1, q, O)
        torch.cuda.synchronize()
        assert torch.equal(th, th0) and not g.any()


def test_eval_outside_domain_uses_fallback(E):
    """Queries far outside the lattice fail the window certificate and are
    evaluated against every key; results still match the definition."""
    R = 6
    rng = np.random.default_rng(5)
    q = rng.uniform(-1.8, 1.8, size=(3000, 3)).astype(np.float32)
    th = W.perturbed_theta(R, 6, rho0=4.0)
    O, lse, nu, _ = run_eval(E, R, th, q)
    ref = PT.reference(R, th, q)
    PT.check_eval(O, lse, ref)
    assert nu > 0


def test_eval_forced_small_window_falls_back(E):
    """A forced window of one cell cannot certify most queries at R = 16;
    the fallback must still reproduce the global result."""
    R = 16
    w = W.get("sphere_r8")
    q, _ = W.make_batch(w, 2, J=4096)
    th = W.perturbed_theta(R, 7, rho0=7.0)
    O, lse, nu, st = run_eval(E, R, th, q, window=1)
    ref = PT.reference(R, th, q)
    PT.check_eval(O, lse, ref)
    assert st["W"] == 1 and nu > 100


def test_eval_coarse_lattice_exact_max_path(E):
    """R = 4 with beta = exp(7): every logit is below -300 nats away from the
    vertices, so the kernel takes the exact-maximum pass."""
    R = 4
    w = W.get("sphere_r8")
    q, _ = W.make_batch(w, 3, J=5000)
    th = W.perturbed_theta(R, 8, rho0=7.0, rho_spread=0.3)
    O, lse, nu, _ = run_eval(E, R, th, q)
    ref = PT.reference(R, th, q)
    PT.check_eval(O, lse, ref)


def test_wide_window_beyond_one_row_group(E):
    """Small scales widen the window past 15 cells: at R = 40 with rho in
    [2.5, 3.5] the certificate needs W = 26, so a tile's
    moved-key rows (up to 39 x 39 cells) span two row groups.  Every query
    inside the lattice must still be certified by its window (none falls back
    to all keys), and values, gradient and a fit step match the global
    definition."""
    R, J = 40, 2048
    w = W.get("sphere_r8")
    q, o = W.make_batch(w, 21, J=J)
    th = W.perturbed_theta(R, 22, rho0=3.0)
    O, lse, nu, st = run_eval(E, R, th, q)
    assert st["W"] == 26, st["W"]
    assert nu == 0
    ref = PT.reference(R, th, q)
    PT.check_eval(O, lse, ref)
    rng = np.random.default_rng(23)
    dl = rng.standard_normal(J) / J
    with E.Engine(R, J) as eng:
        G = eng.grad(PT.to_dev(th), PT.to_dev(q), PT.to_dev(ref["O"]), PT.to_dev(ref["lse"]), PT.to_dev(dl))
        torch.cuda.synchronize()
        assert eng.stats()["n_uncertified"] == 0
        G = G.cpu().numpy()
    gr, ar, br = PT.oracle_grad(R, th, q, dl)
    PT.check_grad(G, gr, ar, br)


def test_eval_grid_keys_only(E):
    """offsets = 0 (Eq. func-interp, the ablation's G-6): theta holds only the
    five grid channels per vertex (value, slope, scale)."""
    R = 8
    w = W.get("sphere_r8")
    q, _ = W.make_batch(w, 4, J=8192)
    th = W.perturbed_theta(R, 9)
    th5 = np.ascontiguousarray(th.reshape(-1, 13)[:, :5])
    O, lse, nu, _ = run_eval(E, R, th5, q, offsets=0)
    ref = PT.reference(R, th, q, offsets=0)
    PT.check_eval(O, lse, ref)


def test_eval_queries_on_lattice_vertices_and_faces(E):
    R = 7
    t = np.linspace(-1, 1, R).astype(np.float32)
    V = np.stack(np.meshgrid(t, t, t, indexing="ij"), -1).reshape(-1, 3)
    F = V.copy()
    F[:, 0] = np.clip(F[:, 0] + (t[1] - t[0]) / 2, -1, 1)
    q = np.concatenate([V, F]).astype(np.float32)
    th = W.perturbed_theta(R, 10)
    O, lse, nu, _ = run_eval(E, R, th, q)
    ref = PT.reference(R, th, q)
    PT.check_eval(O, None, ref)


def test_query_gradient_matches_oracle(E):
    R = 6
    w = W.get("sphere_r8")
    q, _ = W.make_batch(w, 5, J=3000)
    th = W.perturbed_theta(R, 11, rho0=5.0)
    with E.Engine(R, len(q)) as eng:
        _, _, dq, _ = eng.eval(PT.to_dev(th), PT.to_dev(q), with_qgrad=True)
        torch.cuda.synchronize()
        dq = dq.cpu().numpy().astype(np.float64)
    keys = orc.build_keys(orc.Grid(R=R), th)
    worst = PT.check_qgrad(dq, PT.qgrad_reference(keys, q))
    print(f"dO/dq worst err / tolerance {worst:.3g}")


# ------------------------------------------------------------------ grad
@pytest.mark.parametrize("init", ["paper", "perturbed"])
def test_grad_sphere_r8_full(E, init):
    R = 8
    w = W.get("sphere_r8")
    q, o = W.make_batch(w, 1)
    th = meanshift_theta(R, w)[0] if init == "paper" else W.perturbed_theta(R, 12)
    Or, lr, _ = PT.oracle_values(R, th, q)
    rng = np.random.default_rng(13)
    dl = rng.standard_normal(len(q)) / len(q)
    with E.Engine(R, len(q)) as eng:
        tth = PT.to_dev(th)
        G = eng.grad(tth, PT.to_dev(q), PT.to_dev(Or), PT.to_dev(lr), PT.to_dev(dl))
        torch.cuda.synchronize()
        G = G.cpu().numpy()
    gr, ar, br = PT.oracle_grad(R, th, q, dl)
    PT.check_grad(G, gr, ar, br)


def test_grad_accumulates_into_caller_buffer(E):
    R = 5
    w = W.get("sphere_r8")
    q, _ = W.make_batch(w, 6, J=2000)
    th = W.perturbed_theta(R, 14, rho0=5.0)
    Or, lr, _ = PT.oracle_values(R, th, q)
    dl = np.random.default_rng(1).standard_normal(len(q))
    with E.Engine(R, len(q)) as eng:
        tth = PT.to_dev(th)
        base = torch.full_like(tth, 0.5)
        G = eng.grad(tth, PT.to_dev(q), PT.to_dev(Or), PT.to_dev(lr), PT.to_dev(dl), grad=base)
        torch.cuda.synchronize()
        G = G.cpu().numpy()
    gr, ar, br = PT.oracle_grad(R, th, q, dl)
    PT.check_grad(G - 0.5, gr, ar + 1e-7, br)


def test_grad_outside_domain_fallback(E):
    R = 6
    rng = np.random.default_rng(7)
    q = rng.uniform(-1.8, 1.8, size=(2000, 3)).astype(np.float32)
    th = W.perturbed_theta(R, 15, rho0=4.0)
    Or, lr, _ = PT.oracle_values(R, th, q)
    dl = rng.standard_normal(len(q))
    with E.Engine(R, len(q)) as eng:
        G = eng.grad(PT.to_dev(th), PT.to_dev(q), PT.to_dev(Or), PT.to_dev(lr), PT.to_dev(dl))
        torch.cuda.synchronize()
        st = eng.stats()
        G = G.cpu().numpy()
    gr, ar, br = PT.oracle_grad(R, th, q, dl)
    PT.check_grad(G, gr, ar, br)
    assert st["n_uncertified"] > 0


# --------------------------------------------------------------- fit step
@pytest.mark.parametrize("init", ["paper", "perturbed"])
def test_fit_step_sphere_r8_full(E, init):
    """One forward + backward + AdamW step on the full tiny workload against
    the oracle under the global definition."""
    R = 8
    w = W.get("sphere_r8")
    q, o = W.make_batch(w, 0)
    th = meanshift_theta(R, w)[0] if init == "paper" else W.perturbed_theta(R, 16)
    n = th.size
    with E.Engine(R, len(q)) as eng:
        tth = PT.to_dev(th)
        m = torch.zeros(n, device=PT.DEV)
        v = torch.zeros(n, device=PT.DEV)
        loss = torch.zeros(2, device=PT.DEV, dtype=torch.float64)
        eng.fit_step(tth, m, v, 1, PT.to_dev(q), PT.to_dev(o), loss)
        torch.cuda.synchronize()
        th1, m1, v1, loss = (x.cpu().numpy() for x in (tth, m, v, loss))
    ref = orc.fit_step(orc.Grid(R=R), th, np.zeros(n), np.zeros(n), 1, q, o)
    assert abs(loss[0] - ref["loss"]) <= 1e-5 * ref["loss"]
    assert abs(loss[1] - ref["l1"]) <= 1e-5 * ref["l1"]
    # the GPU's gradient, recovered from the first moment m = (1 - beta1) g
    g_gpu = m1.astype(np.float64) / (1.0 - np.float32(0.9))
    O, _, _ = PT.oracle_values(R, th, q)
    _, ar, br = PT.oracle_grad(R, th, q, 2 * (O - o) / len(q))
    PT.check_grad(g_gpu, ref["grad"], ar, br)
    # AdamW on the GPU's own gradient
    th_ref, _, _ = orc.adam(th.reshape(-1), np.zeros(n), np.zeros(n), g_gpu.reshape(-1), 1)
    tol = 4 * PT.ulp32(th_ref) + 1e-6 * 6e-4
    assert np.all(np.abs(th1.reshape(-1) - th_ref) <= tol)
    # the library takes the hyper-parameters as float32: 1 - fl32(0.999)
    b2 = float(np.float32(0.999))
    assert np.allclose(v1.reshape(-1), (1 - b2) * g_gpu.reshape(-1) ** 2, rtol=1e-5, atol=1e-37)


@pytest.mark.parametrize("R,J,cap", [(16, 3000, 512), (8, 6000, 128)])
def test_merged_sparse_tiles_eval_grad_fit_step(E, R, J, cap):
    """Tiles shared by z-adjacent sparse cell blocks (R = 16: ~6 queries per
    block) or by z-adjacent sparse cells of blocks split into cell tiles
    (R = 8 with a 128-query cap) under group_cells = MERGE: fewer tiles than
    with group_cells = 1, and eval, grad and a fit step still match the
    oracle under the global definition."""
    q, o = W.make_batch(W.get("sphere_r8"), 2, J=J)
    th = W.perturbed_theta(R, 41)
    n = th.size
    ntiles = {}
    for grp in (1, MERGE):
        with E.Engine(R, J) as eng:
            eng.set_tuning(cap, grp, 8)
            tth = PT.to_dev(th)
            O, lse, _, _ = eng.eval(tth, PT.to_dev(q))
            ntiles[grp] = eng.stats()["n_tiles"]
            ref = PT.reference(R, th, q)
            dl = (2 * (ref["O"] - o) / J).astype(np.float32)
            G = eng.grad(tth, PT.to_dev(q), PT.to_dev(ref["O"]), PT.to_dev(ref["lse"]), PT.to_dev(dl))
            m = torch.zeros(n, device=PT.DEV)
            v = torch.zeros(n, device=PT.DEV)
            loss = torch.zeros(2, device=PT.DEV, dtype=torch.float64)
            eng.fit_step(tth, m, v, 1, PT.to_dev(q), PT.to_dev(o), loss)
            torch.cuda.synchronize()
            O, lse, G, m1, loss = (x.cpu().numpy() for x in (O, lse, G, m, loss))
        PT.check_eval(O, lse, ref)
        gr, ar, br = PT.oracle_grad(R, th, q, dl)
        PT.check_grad(G, gr, ar, br)
        fr = orc.fit_step(orc.Grid(R=R), th, np.zeros(n), np.zeros(n), 1, q, o)
        assert abs(loss[0] - fr["loss"]) <= 1e-5 * fr["loss"]
        _, ar, br = PT.oracle_grad(R, th, q, 2 * (ref["O"] - o) / J)
        PT.check_grad(m1.astype(np.float64) / (1.0 - np.float32(0.9)), fr["grad"], ar, br)
    assert ntiles[MERGE] < (0.75 if cap == 512 else 0.95) * ntiles[1], ntiles


def test_dense_tiles_half_batch_backward_fit_step_and_grad(E):
    """Tiles of ~300 queries with at most a few hundred kept keys (R = 12,
    2^16 points: 216 cell blocks): the single-shape kernel runs their
    backward in batches of at most 128 keys, two lanes per key.  The fit
    step's loss, gradient and AdamW update and the grad call match the
    oracle under the global definition."""
    R, J = 12, 1 << 16
    q, o = W.make_batch(W.get("sphere_r8"), 7, J=J)
    th = W.perturbed_theta(R, 43)
    n = th.size
    with E.Engine(R, J) as eng:
        tth = PT.to_dev(th)
        ref = PT.reference(R, th, q)
        dl = (2 * (ref["O"] - o) / J).astype(np.float32)
        G = eng.grad(tth, PT.to_dev(q), PT.to_dev(ref["O"]), PT.to_dev(ref["lse"]), PT.to_dev(dl))
        m = torch.zeros(n, device=PT.DEV)
        v = torch.zeros(n, device=PT.DEV)
        loss = torch.zeros(2, device=PT.DEV, dtype=torch.float64)
        eng.fit_step(tth, m, v, 1, PT.to_dev(q), PT.to_dev(o), loss)
        torch.cuda.synchronize()
        st = eng.stats()
        th1, m1, G, loss = (x.cpu().numpy() for x in (tth, m, G, loss))
    # the premise: many 2x2x2 blocks hold 192..512 queries, one tile each
    h = 2.0 / (R - 1)
    c = np.clip(np.floor((q.astype(np.float64) + 1.0) / h).astype(int), 0, R - 2)
    nb = (R - 1 + 1) // 2
    tot = np.bincount((c[:, 0] // 2 * nb + c[:, 1] // 2) * nb + c[:, 2] // 2, minlength=nb ** 3)
    assert ((tot >= 192) & (tot <= 512)).sum() >= 40 and st["W"] <= 3, st
    gr, ar, br = PT.oracle_grad(R, th, q, dl)
    PT.check_grad(G, gr, ar, br)
    fr = orc.fit_step(orc.Grid(R=R), th, np.zeros(n), np.zeros(n), 1, q, o)
    assert abs(loss[0] - fr["loss"]) <= 1e-5 * fr["loss"]
    assert abs(loss[1] - fr["l1"]) <= 1e-5 * fr["l1"]
    g_gpu = m1.astype(np.float64) / (1.0 - np.float32(0.9))
    PT.check_grad(g_gpu, fr["grad"], ar, br)
    th_ref, _, _ = orc.adam(th.reshape(-1), np.zeros(n), np.zeros(n), g_gpu.reshape(-1), 1)
    assert np.all(np.abs(th1.reshape(-1) - th_ref) <= 4 * PT.ulp32(th_ref) + 1e-6 * 6e-4)


@pytest.mark.parametrize("R", [2, 3])
def test_minimum_lattices_eval_grad_fit_step(E, R):
    """The smallest lattices: one cell (R = 2) and eight (R = 3), so every
    query's window is the whole lattice and every key is on a lattice face;
    eval, grad and one fit step against the oracle, with queries inside and
    a few outside the domain."""
    rng = np.random.default_rng(40 + R)
    q = rng.uniform(-1.0, 1.0, size=(3000, 3)).astype(np.float32)
    q[-40:] *= np.float32(1.3)
    o = (np.linalg.norm(q, axis=1) - 0.5).astype(np.float32)
    th = W.perturbed_theta(R, 41 + R, rho0=3.0)
    O, lse, nu, _ = run_eval(E, R, th, q)
    ref = PT.reference(R, th, q)
    PT.check_eval(O, lse, ref)
    Or, lr, _ = PT.oracle_values(R, th, q)
    dl = rng.standard_normal(len(q)) / len(q)
    n = th.size
    with E.Engine(R, len(q)) as eng:
        tth = PT.to_dev(th)
        G = eng.grad(tth, PT.to_dev(q), PT.to_dev(Or), PT.to_dev(lr), PT.to_dev(dl))
        m = torch.zeros(n, device=PT.DEV)
        v = torch.zeros(n, device=PT.DEV)
        loss = torch.zeros(2, device=PT.DEV, dtype=torch.float64)
        eng.fit_step(tth, m, v, 1, PT.to_dev(q), PT.to_dev(o), loss)
        torch.cuda.synchronize()
        G, m1, loss = G.cpu().numpy(), m.cpu().numpy(), loss.cpu().numpy()
    gr, ar, br = PT.oracle_grad(R, th, q, dl)
    PT.check_grad(G, gr, ar, br)
    fref = orc.fit_step(orc.Grid(R=R), th, np.zeros(n), np.zeros(n), 1, q, o)
    assert abs(loss[0] - fref["loss"]) <= 1e-5 * fref["loss"]
    g_gpu = m1.astype(np.float64) / (1.0 - np.float32(0.9))
    _, ar2, br2 = PT.oracle_grad(R, th, q, 2 * (Or - o) / len(q))
    PT.check_grad(g_gpu, fref["grad"], ar2, br2)


def test_second_fit_step_starts_from_clean_gradient(E):
    """Step 2 reports the loss of the parameters after step 1 and uses only
    their gradient: the internal gradient buffer is cleared by the update."""
    R = 6
    w = W.get("sphere_r8")
    q, o = W.make_batch(w, 9, J=20000)
    th = W.perturbed_theta(R, 17, rho0=5.0)
    n = th.size
    with E.Engine(R, len(q)) as eng:
        tth = PT.to_dev(th)
        m = torch.zeros(n, device=PT.DEV)
        v = torch.zeros(n, device=PT.DEV)
        loss = torch.zeros(2, device=PT.DEV, dtype=torch.float64)
        tq, to = PT.to_dev(q), PT.to_dev(o)
        eng.fit_step(tth, m, v, 1, tq, to, loss)
        th1, m1 = tth.clone(), m.clone()
        eng.fit_step(tth, m, v, 2, tq, to, loss)
        torch.cuda.synchronize()
        th1, m1, m2, l2 = (x.cpu().numpy() for x in (th1, m1, m, loss))
    O1, _, _ = PT.oracle_values(R, th1, q)
    assert abs(l2[0] - np.mean((O1 - o) ** 2)) <= 1e-5 * np.mean((O1 - o) ** 2)
    g2 = (m2.astype(np.float64) - np.float32(0.9) * m1.astype(np.float64)) / (1 - np.float32(0.9))
    gr, ar, br = PT.oracle_grad(R, th1, q, 2 * (O1 - o) / len(q))
    # the subtraction of the rescaled first moment adds a few ulps of m1
    PT.check_grad(g2, gr, ar + 20 * PT.ulp32(m1).reshape(ar.shape), br)


def test_loss_grad_equals_fit_step_gradient(E):
    """efunc_loss_grad accumulates the gradient the fused step applies (the
    same kernels): loss equal, gradient equal to m / (1 - beta1) of a first
    step, and a second call doubles it."""
    R = 8
    w = W.get("sphere_r8")
    q, o = W.make_batch(w, 5, J=20000)
    th = W.perturbed_theta(R, 81)
    n = th.size
    with E.Engine(R, len(q)) as eng:
        tq, to = PT.to_dev(q), PT.to_dev(o)
        g = torch.zeros(n, device=PT.DEV)
        l1 = torch.zeros(2, device=PT.DEV, dtype=torch.float64)
        eng.loss_grad(PT.to_dev(th), tq, to, g, l1)
        tth = PT.to_dev(th)
        m = torch.zeros(n, device=PT.DEV)
        v = torch.zeros(n, device=PT.DEV)
        l2 = torch.zeros(2, device=PT.DEV, dtype=torch.float64)
        eng.fit_step(tth, m, v, 1, tq, to, l2)
        g2 = g.clone()
        eng.loss_grad(PT.to_dev(th), tq, to, g2)
        torch.cuda.synchronize()
        g, g2, m, l1, l2 = (x.cpu().numpy() for x in (g, g2, m, l1, l2))
    assert np.allclose(l1, l2, rtol=1e-6, atol=0)
    gm = m.astype(np.float64) / (1.0 - np.float32(0.9))
    scale = np.abs(g).reshape(-1, 13).max(axis=0)
    assert np.all(np.abs(gm - g).reshape(-1, 13) <= 1e-4 * np.abs(g).reshape(-1, 13) + 1e-5 * scale)
    assert np.all(np.abs(g2 - 2 * g).reshape(-1, 13) <= 1e-4 * np.abs(g).reshape(-1, 13) + 1e-5 * scale)
