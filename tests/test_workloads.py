"""Seeded workload generators: determinism, mix and target correctness."""
import numpy as np
import torch

import workloads as W


def test_batches_are_seeded_and_distinct():
    w = W.get("sphere_r8")
    q0, o0 = W.make_batch(w, 0)
    q0b, o0b = W.make_batch(w, 0)
    q1, _ = W.make_batch(w, 1)
    assert np.array_equal(q0, q0b) and np.array_equal(o0, o0b)
    assert not np.array_equal(q0, q1)
    assert q0.dtype == np.float32 and q0.shape == (w.J, 3)


def test_half_uniform_half_near_surface():
    w = W.get("sphere_r8")
    q, o = W.make_batch(w, 3)
    n = w.J // 2
    assert np.all(np.abs(q[:n]) <= 1.0)
    # near-surface half: |sdf| ~ |N(0, 0.01^2)| projected on the normal
    assert np.abs(o[n:]).mean() < 0.02
    assert np.abs(o[:n]).mean() > 0.2


def test_sphere_target_is_exact():
    w = W.get("sphere_r8")
    q = np.array([[0.0, 0.0, 0.0], [0.5, 0.0, 0.0], [1.0, 1.0, 1.0]], np.float32)
    o = W.target(w, torch.as_tensor(q)).numpy()
    assert np.allclose(o, [-0.5, 0.0, np.sqrt(3) - 0.5])


def test_csg_surface_points_lie_on_zero_set():
    w = W.get("csg16_r32")
    s = W.surface_points(w, 2000, seed=1)
    f = W.target(w, torch.as_tensor(s)).numpy()
    assert np.abs(f).max() <= 1e-6


def test_box_sdf_properties():
    from workloads.shapes import Primitive
    p = Primitive("box", np.zeros(3), half=np.array([0.1, 0.2, 0.3]))
    q = torch.tensor([[0.0, 0.0, 0.0], [0.5, 0.0, 0.0], [0.1, 0.2, 0.3], [0.4, 0.6, 0.3]],
                     dtype=torch.float64)
    d = p.sdf(q).numpy()
    assert np.allclose(d, [-0.1, 0.4, 0.0, np.hypot(0.3, 0.4)])


def test_perturbed_theta_layout():
    th = W.perturbed_theta(4, 0)
    assert th.shape == (4, 4, 4, 13) and th.dtype == np.float32
    assert np.all(np.abs(th[..., 4] - 7.0) <= 0.5) and np.all(np.abs(th[..., 12] - 7.0) <= 0.5)
    pl = W.plain_theta(4)
    assert np.all(pl[..., [4, 12]] == 7.0) and np.count_nonzero(pl[..., [0, 1, 2, 3, 5, 6, 7, 8, 9, 10, 11]]) == 0
