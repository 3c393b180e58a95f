"""Checkpoint files (CPU): theta, m, v round-trip bit for bit with the step,
sampler position and configuration."""
import numpy as np
import pytest
import torch

from paper_2505_21319_amd import checkpoint as CK


def test_round_trip_is_bitwise(tmp_path):
    g = torch.Generator().manual_seed(3)
    th = torch.randn(5, 5, 5, 13, generator=g)
    th.view(-1)[7] = float.fromhex("0x1.fffffep-127")  # a subnormal survives
    m = torch.randn(th.shape, generator=g) * 1e-3
    v = torch.rand(th.shape, generator=g) * 1e-6
    p = str(tmp_path / "fit.safetensors")
    CK.save(p, th, m, v, 17, sampler={"workload": "sphere_r8", "next_iteration": 17}, config={"R": 5})
    r = CK.load(p)
    for a, b in ((r["theta"], th), (r["m"], m), (r["v"], v)):
        assert a.dtype == torch.float32 and a.shape == b.shape
        assert np.array_equal(a.numpy().view(np.uint32), b.numpy().view(np.uint32))
    assert r["step"] == 17 and r["sampler"]["next_iteration"] == 17 and r["config"]["R"] == 5


def test_rejects_bad_inputs(tmp_path):
    th = torch.zeros(2, 2, 2, 13)
    with pytest.raises(TypeError):
        CK.save(str(tmp_path / "a"), th.double(), th, th, 1)
    with pytest.raises(ValueError):
        CK.save(str(tmp_path / "b"), th, th[:1], th, 1)
    with pytest.raises(ValueError):
        CK.save(str(tmp_path / "c"), th, th, th, -1)
    from safetensors.torch import save_file
    save_file({"x": th}, str(tmp_path / "d"))
    with pytest.raises(ValueError):
        CK.load(str(tmp_path / "d"))
