"""The learned initialiser's starting parameters (CPU): the FP64 reference
(oracle.initnet.base_theta) pinned by fields whose answers are known -- the
central-difference gradient of a linear field is exact, one Newton step
from a vertex lands on a plane exactly, longer steps are capped at one
spacing, the log-scale floor and its mask -- and the network's initial
parameters."""
import numpy as np

from oracle import initnet as N
from paper_2505_21319_amd import initnet_train as T


def lattice_points(R):
    t = T.lattice(R)
    return np.stack(np.meshgrid(t, t, t, indexing="ij"), -1).reshape(-1, 3)


def test_gradient_of_a_linear_field_is_exact():
    R = 9
    g = lattice_points(R)
    sdf = (0.3 * g[:, 0] - 0.5 * g[:, 1] + 0.2 * g[:, 2] + 0.1).astype(np.float32)
    _, _, gr = N.base_theta(sdf, R)
    assert np.allclose(gr[0], [0.3, -0.5, 0.2], atol=1e-6)


def test_gradient_uses_one_sided_differences_on_the_faces():
    R = 6
    g = lattice_points(R)
    sdf = (g[:, 0] ** 2).astype(np.float32)   # d/dx = 2x, central differences exact inside
    _, _, gr = N.base_theta(sdf, R)
    h = 2.0 / (R - 1)
    x = g[:, 0]
    inner = (np.abs(x) < 1 - 1e-9)
    assert np.allclose(gr[0, inner, 0], 2 * x[inner], atol=1e-6)
    lo, hi = np.isclose(x, -1.0), np.isclose(x, 1.0)
    assert np.allclose(gr[0, lo, 0], ((-1 + h) ** 2 - 1) / h, atol=1e-6)
    assert np.allclose(gr[0, hi, 0], (1 - (1 - h) ** 2) / h, atol=1e-6)
    assert np.allclose(gr[0, :, 1:], 0.0)


def test_newton_base_moves_keys_onto_a_plane_and_caps_the_step():
    """For a plane the one Newton step lands exactly on the zero set (within
    one lattice spacing); o' is then 0 and d' the plane's normal.  Farther
    vertices move by exactly one spacing."""
    R = 11
    h = 2.0 / (R - 1)
    g = lattice_points(R)
    n = np.array([0.6, 0.0, 0.8])
    sdf = (g @ n - 0.05).astype(np.float32)
    th, mask, _ = N.base_theta(sdf, R)
    th = th[0]
    assert th.shape == (R ** 3, 13) and not mask.any()
    delta = th[:, 5:8]
    moved = g + delta
    near = np.abs(sdf) <= h * 0.999
    assert near.any() and (~near).any()
    assert np.allclose(moved[near] @ n - 0.05, 0.0, atol=1e-6)
    assert np.allclose(th[near, 8], 0.0, atol=1e-6)
    assert np.allclose(np.linalg.norm(delta[~near], axis=1), h, rtol=1e-9)
    assert np.array_equal(th[:, 0], sdf.astype(np.float64)) and np.allclose(th[:, 1:4], n, atol=1e-6)
    assert np.all(th[:, 4] == 7.0) and np.all(th[:, 12] == 7.0)


def test_residual_and_log_scale_floor():
    R = 3
    sdf = np.zeros(R ** 3, np.float32)
    res = np.zeros((1, R ** 3, 13), np.float32)
    res[0, :5, 4] = [-1.0, 0.0, 1.0, -8.0, 0.5]
    res[0, :5, 12] = [2.0, -0.1, 0.0, 0.1, -7.0]
    res[0, :, 0] = 0.25
    th, mask, _ = N.base_theta(sdf, R, res=res, rho_min=7.0)
    assert np.array_equal(th[0, :5, 4], [7.0, 7.0, 8.0, 7.0, 7.5])
    assert np.allclose(th[0, :5, 12], [9.0, 7.0, 7.0, 7.1, 7.0], rtol=0, atol=1e-6)
    assert mask[0, :5].tolist() == [[True, False], [False, True], [False, False], [True, False], [False, True]]
    assert np.all(th[0, :, 0] == 0.25) and np.all(th[0, 5:, [4, 12]] == 7.0)


def test_initial_parameters_match_the_network_size_and_start_small():
    p = T.initial_params(3)
    assert p.size == N.num_params(T.CHANNELS) and p.dtype == np.float32
    layers = N.unpack(p.astype(np.float64), T.CHANNELS)
    assert all(not b.any() for _, b in layers)          # zero biases: a zero residual at the start ...
    assert np.abs(layers[-1][0]).std() < 0.2 * np.abs(layers[-2][0]).std()   # ... and a small last layer
