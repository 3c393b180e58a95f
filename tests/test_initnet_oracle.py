"""Pins of the FP64 oracle of the learned-initialiser network
(oracle/initnet.py): bf16 rounding against torch's conversion, the
convolution against direct loops, the layer gradients against central
differences (with the bf16 rounding switched off) and the network's
composition."""
import numpy as np
import pytest
import torch

from oracle import initnet as N


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-20, 20, 20000),
                        [0.0, -0.0, 1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -(1.0 + 2 ** -9), 65504.0]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(N.bf16_round(x), ref)


def _direct_conv(x, w):
    B, D = x.shape[0], x.shape[1]
    co, _, ci = w.shape
    y = np.zeros((B, D, D, D, co))
    for b in range(B):
        for z in range(D):
            for yy in range(D):
                for xx in range(D):
                    for dz in range(3):
                        for dy in range(3):
                            for dx in range(3):
                                zz, y2, x2 = z + dz - 1, yy + dy - 1, xx + dx - 1
                                if 0 <= zz < D and 0 <= y2 < D and 0 <= x2 < D:
                                    y[b, z, yy, xx] += w[:, (dz * 3 + dy) * 3 + dx, :] @ x[b, zz, y2, x2]
    return y


def test_convolution_matches_direct_loops():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 4, 4, 4, 3))
    w = rng.standard_normal((5, 27, 3))
    assert np.allclose(N._conv(x, w), _direct_conv(x, w), rtol=1e-13, atol=1e-13)


def test_bias_relu_and_layer_rounding():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((1, 3, 3, 3, 2))
    w = rng.standard_normal((4, 27, 2))
    b = rng.standard_normal(4)
    z, a = N.layer_forward(x, w, b, relu=True)
    ref = _direct_conv(N.bf16_round(x), N.bf16_round(w)) + b
    assert np.allclose(z, ref, rtol=1e-13, atol=1e-13)
    assert np.array_equal(a, np.maximum(ref, 0) + 0 * a) or np.allclose(a, np.maximum(ref, 0), atol=1e-13)


@pytest.fixture
def exact(monkeypatch):
    monkeypatch.setattr(N, "ROUND", lambda a: np.asarray(a, dtype=np.float64))
    return N


def test_network_gradient_matches_central_differences(exact):
    """Every parameter of a 3-layer network (ReLU between layers) against
    central differences of L = sum(dout * forward) in exact arithmetic."""
    rng = np.random.default_rng(3)
    ch = [1, 3, 4, 2]
    p = rng.standard_normal(N.num_params(ch)) * 0.4
    x = rng.standard_normal((2, 4, 4, 4, 1))
    dout = rng.standard_normal((2, 4, 4, 4, 2))
    g = N.backward(p, ch, x, dout)
    h = 1e-6
    for i in rng.choice(p.size, 60, replace=False):
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (np.sum(dout * N.forward(pp, ch, x)[0]) - np.sum(dout * N.forward(pm, ch, x)[0])) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * (1 + abs(g[i])), (i, fd, g[i])


def test_forward_composes_layers():
    rng = np.random.default_rng(4)
    ch = [1, 2, 3]
    p = rng.standard_normal(N.num_params(ch))
    x = rng.standard_normal((1, 3, 3, 3, 1))
    (w1, b1), (w2, b2) = N.unpack(p, ch)
    _, a1 = N.layer_forward(x, w1, b1, relu=True)
    _, a2 = N.layer_forward(a1, w2, b2, relu=False)
    out, inputs = N.forward(p, ch, x)
    assert np.array_equal(out, a2) and np.array_equal(inputs[1], a1)


def test_num_params():
    assert N.num_params([1, 32, 64, 64, 13]) == 27 * (32 + 32 * 64 + 64 * 64 + 64 * 13) + 32 + 64 + 64 + 13
