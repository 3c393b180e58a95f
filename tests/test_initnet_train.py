"""Host-side pieces of the learned-initialiser experiment (CPU): the
Newton-step base parameters, the central-difference SDF gradient and the
log-scale floor."""
import numpy as np
import torch

from paper_2505_21319_amd import initnet_train as T


def lattice_points(R):
    t = torch.from_numpy(T.lattice(R))
    return torch.stack(torch.meshgrid(t, t, t, indexing="ij"), -1).reshape(-1, 3)


def test_sdf_gradient_of_a_linear_field_is_exact():
    R = 9
    g = lattice_points(R)
    sdf = (0.3 * g[:, 0] - 0.5 * g[:, 1] + 0.2 * g[:, 2] + 0.1).float()
    gr = T.sdf_gradient(sdf, R)
    assert torch.allclose(gr, torch.tensor([0.3, -0.5, 0.2]).expand_as(gr), atol=1e-5)


def test_newton_base_moves_keys_onto_a_plane_and_caps_the_step():
    """For a plane the one Newton step lands exactly on the zero set (within
    one lattice spacing); o' is then 0 and d' the plane's normal.  Farther
    vertices move by exactly one spacing."""
    R = 11
    h = 2.0 / (R - 1)
    g = lattice_points(R)
    n = torch.tensor([0.6, 0.0, 0.8])
    sdf = (g @ n.double() - 0.05).float()
    th = T.newton_theta(sdf, R)
    assert th.shape == (R ** 3, 13)
    delta = th[:, 5:8]
    moved = g.float() + delta
    near = sdf.abs() <= h * 0.999
    assert near.any() and (~near).any()
    assert torch.allclose((moved[near] @ n) - 0.05, torch.zeros(int(near.sum())), atol=1e-5)
    assert torch.allclose(th[near, 8], torch.zeros(int(near.sum())), atol=1e-5)
    assert torch.allclose(delta[~near].norm(dim=1), torch.full((int((~near).sum()),), h), rtol=1e-5)
    assert torch.allclose(th[:, 0], sdf) and torch.allclose(th[:, 1:4], n.expand(R ** 3, 3), atol=1e-5)
    assert torch.all(th[:, 4] == 7.0) and torch.all(th[:, 12] == 7.0)


def test_rho_floor_clamps_both_scale_channels_and_reports_them():
    th = torch.zeros(5, 13)
    th[:, 4] = torch.tensor([6.0, 7.0, 8.0, -1.0, 7.5])
    th[:, 12] = torch.tensor([9.0, 6.9, 7.0, 7.1, 0.0])
    mask = T.rho_floor(th)
    assert torch.equal(th[:, 4], torch.tensor([7.0, 7.0, 8.0, 7.0, 7.5]))
    assert torch.equal(th[:, 12], torch.tensor([9.0, 7.0, 7.0, 7.1, 7.0]))
    assert mask.tolist() == [[True, False], [False, True], [False, False], [True, False], [False, True]]
    # the other channels are untouched
    assert not th[:, [0, 1, 2, 3, 5, 6, 7, 8, 9, 10, 11]].any()


def test_initial_parameters_match_the_network_size_and_start_small():
    from oracle import initnet as N
    p = T.initial_params(3)
    assert p.size == N.num_params(T.CHANNELS) and p.dtype == np.float32
    layers = N.unpack(p.astype(np.float64), T.CHANNELS)
    assert all(not b.any() for _, b in layers)          # zero biases: a zero residual at the start ...
    assert np.abs(layers[-1][0]).std() < 0.2 * np.abs(layers[-2][0]).std()   # ... and a small last layer
