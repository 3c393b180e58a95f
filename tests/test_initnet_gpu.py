"""GPU parity of the learned-initialiser network (bf16 MFMA convolutions)
against the FP64 oracle oracle/initnet.py: every layer operation on its own
(forward with bias and ReLU, data gradient with the ReLU mask, weight and
bias gradients), the whole network forward and backward, and a short
training run whose loss must fall.

Tolerance: products of bf16 values are exact in fp32; the fp32 sum of K
terms is within gamma_K = K 2^-24 / (1 - K 2^-24) of sum |terms|, plus half
an ulp of the result."""
import numpy as np
import pytest
import torch

from oracle import initnet as N
from tests import parity as PT

pytestmark = pytest.mark.gpu
U = 2.0 ** -24


@pytest.fixture(scope="module")
def E():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2505_21319_amd import efunc
    efunc.lib()
    return efunc


def bf16_tensor(a):
    return torch.from_numpy(np.asarray(a, dtype=np.float32)).to(PT.DEV).to(torch.bfloat16).contiguous()


def gamma(K):
    return K * U / (1 - K * U)


def conv_abs(x, w):
    return N._conv(np.abs(N.bf16_round(x)), np.abs(N.bf16_round(w)))


def blocked(a, C):
    """[V][C] values -> the blocked channel-major copy ([ceil(V/32)][C][32]) as
    a bf16 device tensor; the slots past V hold NaN, which the kernels must
    ignore."""
    V = a.size // C
    nb = (V + 31) // 32
    t = np.full((nb * 32, C), np.nan, np.float32)
    t[:V] = np.asarray(a, np.float32).reshape(V, C)
    return bf16_tensor(t.reshape(nb, 32, C).transpose(0, 2, 1).reshape(-1))


def unblocked(t, V, C):
    """Blocked channel-major bf16 tensor -> [V][C] float values."""
    nb = (V + 31) // 32
    return t.float().cpu().numpy().reshape(nb, C, 32).transpose(0, 2, 1).reshape(nb * 32, C)[:V]


def test_blocked_layout_helpers_round_trip():
    a = np.arange(70 * 3, dtype=np.float32).reshape(70, 3)
    assert np.array_equal(unblocked(blocked(a, 3), 70, 3), a)


@pytest.mark.parametrize("Cin,Cout,R,B", [(1, 32, 6, 2), (32, 64, 5, 3), (64, 13, 4, 2), (13, 64, 4, 1),
                                           (8, 16, 7, 1), (64, 64, 8, 2), (32, 13, 16, 1), (32, 16, 13, 2),
                                           (64, 32, 32, 1), (32, 8, 2, 3), (32, 4, 1, 5)])
def test_conv_forward_matches_oracle(E, Cin, Cout, R, B):
    """Cin % 32 == 0 runs the LDS-staged kernel: R = 1, 2, 4, 5 and 13 put
    row, plane and shape ends inside one workgroup's 256 voxels (and R = 1
    leaves only the centre tap), R = 32 is the network's lattice."""
    rng = np.random.default_rng(Cin * 100 + Cout)
    x = N.bf16_round(rng.standard_normal((B, R, R, R, Cin)))
    W = rng.standard_normal((Cout, 27, Cin)) / np.sqrt(27 * Cin)
    b = rng.standard_normal(Cout)
    wf, _ = E.efunc_conv3d_pack_weights(PT.to_dev(W.reshape(-1)), Cin, Cout)
    V = B * R ** 3
    yf = torch.empty(V * Cout, device=PT.DEV)
    ybf = torch.empty(V * Cout, device=PT.DEV, dtype=torch.bfloat16)
    yT = torch.zeros(E.blocked_size(V, Cout), device=PT.DEV, dtype=torch.bfloat16)
    E.efunc_conv3d_bf16(bf16_tensor(x), Cin, wf, Cout, R, bias=PT.to_dev(b.astype(np.float32)), relu=True,
                        y_bf16=ybf, y_f32=yf, yT_bf16=yT)
    torch.cuda.synchronize()
    z, a = N.layer_forward(x, W, b.astype(np.float32).astype(np.float64), relu=True)
    got = yf.cpu().numpy().astype(np.float64).reshape(a.shape)
    tol = gamma(27 * Cin) * (conv_abs(x, W) + np.abs(b)) + U * np.abs(a) + 1e-30
    assert np.all(np.abs(got - a) <= tol), np.max(np.abs(got - a) / tol)
    # the bf16 output is the round-to-nearest-even of the fp32 output
    assert np.array_equal(ybf.float().cpu().numpy().reshape(a.shape), N.bf16_round(got))
    # the blocked channel-major copy holds the same values; slots past V stay untouched
    assert np.array_equal(unblocked(yT, V, Cout), ybf.float().cpu().numpy().reshape(V, Cout))
    nb = (V + 31) // 32
    assert not yT.float().cpu().numpy().reshape(nb, Cout, 32)[-1, :, V - 32 * (nb - 1):].any()


@pytest.mark.parametrize("R", [130])
def test_conv_forward_large_lattice_sampled(E, R):
    """Past 128 lattice points per axis the Cin % 32 == 0 forward runs the
    per-(dz, dy) staged kernel: its outputs on 4096 sampled voxels (all
    lattice faces and edges among them) against the definition evaluated
    at those voxels."""
    Cin, Cout = 32, 8
    rng = np.random.default_rng(130)
    x = N.bf16_round(rng.standard_normal((1, R, R, R, Cin)).astype(np.float32))
    W = rng.standard_normal((Cout, 27, Cin)) / np.sqrt(27 * Cin)
    b = rng.standard_normal(Cout).astype(np.float32)
    wf, _ = E.efunc_conv3d_pack_weights(PT.to_dev(W.reshape(-1)), Cin, Cout)
    V = R ** 3
    yf = torch.empty(V * Cout, device=PT.DEV)
    E.efunc_conv3d_bf16(bf16_tensor(x), Cin, wf, Cout, R, bias=PT.to_dev(b), relu=False, y_f32=yf)
    torch.cuda.synchronize()
    got = yf.cpu().numpy().astype(np.float64).reshape(V, Cout)
    idx = rng.integers(0, R, size=(4096, 3))
    idx[:64] = rng.choice([0, R - 1], size=(64, 3))  # corners and faces
    idx[64:256, rng.integers(0, 3)] = rng.choice([0, R - 1], size=192)
    Wr = N.bf16_round(W)
    xs = x[0]
    ref = np.zeros((len(idx), Cout))
    mag = np.zeros((len(idx), Cout))
    for tap in range(27):
        d = np.array([tap // 9 - 1, (tap // 3) % 3 - 1, tap % 3 - 1])
        nb = idx + d
        ok = np.all((nb >= 0) & (nb < R), axis=1)
        nbc = np.clip(nb, 0, R - 1)
        xv = xs[nbc[:, 0], nbc[:, 1], nbc[:, 2]] * ok[:, None]
        ref += xv @ Wr[:, tap, :].T
        mag += np.abs(xv) @ np.abs(Wr[:, tap, :]).T
    ref += b
    v = (idx[:, 0] * R + idx[:, 1]) * R + idx[:, 2]
    tol = gamma(27 * Cin) * (mag + np.abs(b)) + U * np.abs(ref) + 1e-30
    assert np.all(np.abs(got[v] - ref) <= tol), np.max(np.abs(got[v] - ref) / tol)


@pytest.mark.parametrize("Cin,Cout,R", [(32, 64, 5), (64, 13, 4), (1, 32, 4), (64, 64, 8)])
def test_conv_data_gradient_matches_oracle(E, Cin, Cout, R):
    """dL/dx through the flipped packing, masked by the input activation > 0."""
    rng = np.random.default_rng(7 + Cin)
    B = 2
    x = N.bf16_round(np.maximum(rng.standard_normal((B, R, R, R, Cin)), 0))  # a ReLU output: mask
    W = rng.standard_normal((Cout, 27, Cin)) / np.sqrt(27 * Cin)
    dz = N.bf16_round(rng.standard_normal((B, R, R, R, Cout)))
    _, wd = E.efunc_conv3d_pack_weights(PT.to_dev(W.reshape(-1)), Cin, Cout)
    V = B * R ** 3
    dx = torch.empty(V * Cin, device=PT.DEV)
    dxT = torch.empty(E.blocked_size(V, Cin), device=PT.DEV, dtype=torch.bfloat16)
    E.efunc_conv3d_bf16(bf16_tensor(dz), Cout, wd, Cin, R, mask=bf16_tensor(x), y_f32=dx, yT_bf16=dxT)
    torch.cuda.synchronize()
    _, _, dx_ref = N.layer_backward(x, W, dz)
    dx_ref = dx_ref * (x > 0)
    absref = np.abs(N.layer_backward(np.abs(x), np.abs(W), np.abs(dz))[2])
    got = dx.cpu().numpy().astype(np.float64).reshape(dx_ref.shape)
    tol = gamma(27 * Cout) * absref + U * np.abs(dx_ref) + 1e-30
    assert np.all(np.abs(got - dx_ref) <= tol), np.max(np.abs(got - dx_ref) / tol)
    assert np.array_equal(unblocked(dxT, V, Cin), N.bf16_round(got).reshape(V, Cin))


@pytest.mark.parametrize("Cin,Cout,R,B", [(1, 32, 6, 2), (32, 64, 5, 2), (64, 13, 4, 3), (13, 16, 3, 1),
                                           (64, 64, 8, 2), (1, 32, 16, 1), (64, 13, 8, 3), (13, 64, 16, 1),
                                           (1, 32, 56, 1), (64, 13, 56, 1)])
def test_conv_weight_gradient_matches_oracle(E, Cin, Cout, R, B):
    """R a multiple of 8 takes the x-row path (shifted aligned loads), other R
    the per-element path; several chunks of voxels per call at R = 16; at
    R = 56 the last chunk is partial (with the smallest tiles, some of its
    waves get no voxels)."""
    rng = np.random.default_rng(11 + Cout + R)
    x = N.bf16_round(rng.standard_normal((B, R, R, R, Cin)))
    dz = N.bf16_round(rng.standard_normal((B, R, R, R, Cout)))
    W = rng.standard_normal((Cout, 27, Cin))
    V = B * R ** 3
    dw = torch.zeros(Cout * 27 * Cin, device=PT.DEV)
    db = torch.zeros(Cout, device=PT.DEV)
    E.efunc_conv3d_wgrad_bf16(blocked(x, Cin), Cin, blocked(dz, Cout), Cout, R, V, dw, db)
    torch.cuda.synchronize()
    dW_ref, db_ref, _ = N.layer_backward(x, W, dz)
    dW_abs, db_abs, _ = N.layer_backward(np.abs(x), W, np.abs(dz))
    got = dw.cpu().numpy().astype(np.float64).reshape(dW_ref.shape)
    tol = gamma(V) * np.abs(dW_abs) + U * np.abs(dW_ref) + 1e-30
    assert np.all(np.abs(got - dW_ref) <= tol), np.max(np.abs(got - dW_ref) / tol)
    gb = db.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(gb - db_ref) <= gamma(V) * db_abs + 1e-30)


@pytest.mark.parametrize("R,B,ch", [(6, 2, (1, 16, 32, 16, 13)), (8, 2, (1, 16, 32, 16, 13)),
                                    (8, 1, (1, 12, 20, 13))])
def test_network_forward_backward_against_oracle_layers(E, R, B, ch):
    """The whole 4-layer network: the output and the parameter gradient
    against the oracle evaluated layer by layer on the same bf16 inputs (the
    GPU's rounding of intermediate activations to bf16 is reproduced by the
    oracle; fp32 accumulation may flip a rounding, so the comparison allows
    a few bf16 ulps of the output scale).  Channel counts that are not
    multiples of 8 run on padded channels-last buffers inside the network."""
    ch = list(ch)
    rng = np.random.default_rng(21)
    params = np.concatenate([np.concatenate([rng.standard_normal(co * 27 * ci) / np.sqrt(27 * ci),
                                             0.1 * rng.standard_normal(co)])
                             for ci, co in zip(ch[:-1], ch[1:])]).astype(np.float32)
    sdf = rng.uniform(-1, 1, (B, R, R, R)).astype(np.float32)
    dout = rng.standard_normal((B, R, R, R, ch[-1])).astype(np.float32)
    with E.InitNet(R, B, ch) as net:
        assert net.n_params == N.num_params(ch) == params.size
        P = PT.to_dev(params)
        out = net.forward(P, PT.to_dev(sdf))
        dp = torch.zeros(net.n_params, device=PT.DEV)
        net.backward(PT.to_dev(dout), dp)
        torch.cuda.synchronize()
        out, dp = out.cpu().numpy().astype(np.float64), dp.cpu().numpy().astype(np.float64)
    ref, _ = N.forward(params.astype(np.float64), ch, sdf[..., None].astype(np.float64))
    scale = np.abs(ref).max()
    assert np.abs(out.reshape(ref.shape) - ref).max() <= 4 * 2.0 ** -8 * scale
    g_ref = N.backward(params.astype(np.float64), ch, sdf[..., None].astype(np.float64), dout.astype(np.float64))
    gs = np.abs(g_ref).max()
    assert np.abs(dp - g_ref).max() <= 0.05 * gs, np.abs(dp - g_ref).max() / gs
    assert np.corrcoef(dp, g_ref)[0, 1] > 0.999


def test_adam_update_matches_oracle(E):
    import oracle as orc
    rng = np.random.default_rng(31)
    n = 1000
    p = rng.standard_normal(n).astype(np.float32)
    g = rng.standard_normal(n).astype(np.float32)
    P, M, Vv, G = PT.to_dev(p), torch.zeros(n, device=PT.DEV), torch.zeros(n, device=PT.DEV), PT.to_dev(g)
    E.efunc_adam_update(P, M, Vv, G, 1)
    torch.cuda.synchronize()
    ref, _, _ = orc.adam(p.astype(np.float64), np.zeros(n), np.zeros(n), g.astype(np.float64), 1)
    assert np.all(np.abs(P.cpu().numpy() - ref) <= 4 * PT.ulp32(ref) + 1e-6 * 6e-4)
    assert not G.any()


def test_training_reduces_a_regression_loss(E):
    """Fifty AdamW steps of the network on a fixed regression target lower
    the loss (the backward and the update wire together)."""
    R, B = 6, 2
    ch = [1, 16, 16, 3]
    rng = np.random.default_rng(41)
    params = np.concatenate([np.concatenate([rng.standard_normal(co * 27 * ci) / np.sqrt(27 * ci),
                                             np.zeros(co)]) for ci, co in zip(ch[:-1], ch[1:])])
    sdf = rng.uniform(-1, 1, (B, R, R, R)).astype(np.float32)
    tgt = np.stack([sdf, sdf ** 2, np.roll(sdf, 1, axis=1)], axis=-1).reshape(B, R ** 3, 3)
    with E.InitNet(R, B, ch) as net:
        P = PT.to_dev(params.astype(np.float32))
        M, Vv, G = (torch.zeros_like(P) for _ in range(3))
        S, T = PT.to_dev(sdf), PT.to_dev(tgt)
        adam = E.efunc_default_adam()
        adam.lr = 3e-3
        losses = []
        for step in range(1, 51):
            out = net.forward(P, S)
            d = out - T
            losses.append(float((d * d).mean()))
            net.backward((2.0 / d.numel()) * d, G)
            E.efunc_adam_update(P, M, Vv, G, step, adam)
        torch.cuda.synchronize()
    assert losses[-1] < 0.5 * losses[0], losses[::10]


def test_starting_parameters_match_the_fp64_reference(E):
    """efunc_initnet_theta (gradient, Newton-step base, residual, log-scale
    floor, mask) against oracle.initnet.base_theta on the coarse SDFs of
    three seeded CSG shapes at 32^3, and the floor's backward."""
    import workloads as W
    from paper_2505_21319_amd import initnet_train as T
    R, B = 32, 3
    sdf = torch.stack([T.coarse_sdf(lambda g, w=W.get(n): W.target(w, g), R, PT.DEV)
                       for n in ("csg16_r32", "sphere_r8", "csg16_r32")])
    sdf[2] = sdf[2] * 1.7 - 0.05
    rng = np.random.default_rng(5)
    res = rng.standard_normal((B, R ** 3, 13)).astype(np.float32) * 0.5
    tres = PT.to_dev(res)
    th, mask, gr = E.efunc_initnet_theta(sdf, R, res=tres, rho0=7.0, rho_min=7.0, mask=True, grad=True)
    torch.cuda.synchronize()
    ref, mref, gref = N.base_theta(sdf.cpu().numpy(), R, 7.0, res, 7.0)
    th, gr, mask = th.cpu().numpy().astype(np.float64), gr.cpu().numpy().astype(np.float64), mask.cpu().numpy()
    # Each quantity is a few float32 roundings of sums and products: the
    # tolerance is 4e-6 of the magnitudes of the terms that make it up (the
    # result itself may cancel: o' = o + Delta . d is 0 where the Newton step
    # lands, d + res where the residual opposes the slope)
    base = N.base_theta(sdf.cpu().numpy(), R)[0]
    h = 2.0 / (R - 1)
    g = np.abs(base[..., 1:4])
    dn = np.linalg.norm(base[..., 5:8], axis=-1, keepdims=True)
    mag = np.empty_like(base)
    mag[..., 0] = np.abs(base[..., 0])
    mag[..., 1:4] = g + 1e-3 * g.max()
    mag[..., 9:12] = mag[..., 1:4]
    mag[..., 5:8] = dn + 1e-3 * h
    mag[..., 8] = np.abs(base[..., 0]) + (np.abs(base[..., 5:8]) * g).sum(-1)
    mag[..., [4, 12]] = 7.0

    def close(a, b, scale):
        bad = np.abs(a - b) > 4e-6 * scale + 1e-30
        assert not bad.any(), (int(bad.sum()), np.argwhere(bad)[:3])
    close(gr, gref, mag[..., 1:4])
    close(th, ref, mag + np.abs(res))
    assert np.array_equal(mask.astype(bool), mref)
    assert 0 < mref.sum() < mref.size
    # without residual or floor: the plain Newton base, and the gradient alone
    th0 = E.efunc_initnet_theta(sdf, R)[0]
    close(th0.cpu().numpy().astype(np.float64), base, mag)
    # the floor's backward zeroes exactly the floored log-scale gradients
    dth = torch.ones(B, R ** 3, 13, device=PT.DEV)
    E.efunc_initnet_theta_backward(PT.to_dev(mask, torch.uint8), R, dth)
    d = dth.cpu().numpy()
    assert np.array_equal(d[..., 4] == 0, mref[..., 0]) and np.array_equal(d[..., 12] == 0, mref[..., 1])
    assert np.all(np.delete(d, [4, 12], axis=-1) == 1.0)
