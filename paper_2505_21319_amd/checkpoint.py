"""Checkpoint and resume of a fit.

The representation is its own checkpoint: the paper stores a shape as the
regular grid of per-vertex parameters (Sec. 4.6).  Resuming a fit also needs
the AdamW moments and step counter (Sec. 3.4 / Sec. 4.2 optimiser) and the
position of the minibatch sampler; the library's samplers draw every
minibatch as a seeded function of (workload, iteration), so that position is
the next iteration number.  A checkpoint is one safetensors file: theta, m,
v as float32 tensors (bit for bit) and the step, sampler and configuration
as JSON metadata.  With efunc_config.deterministic set, a fit resumed from a
checkpoint after step k reproduces the uninterrupted fit bit for bit.
"""
from __future__ import annotations

import json
from typing import Optional

import torch
from safetensors.torch import load_file, save_file


def save(path: str, theta: torch.Tensor, m: torch.Tensor, v: torch.Tensor, step: int,
         sampler: Optional[dict] = None, config: Optional[dict] = None) -> None:
    """Write theta, the moments and the number of completed steps."""
    if step < 0:
        raise ValueError("step must be >= 0")
    for name, t in (("theta", theta), ("m", m), ("v", v)):
        if t.dtype != torch.float32:
            raise TypeError(f"{name} must be float32")
    if not (theta.shape == m.shape == v.shape):
        raise ValueError("theta, m and v must have one shape")
    meta = {"step": str(int(step)), "sampler": json.dumps(sampler or {}),
            "config": json.dumps(config or {}), "format": "efunc-checkpoint-1"}
    save_file({"theta": theta.detach().contiguous().cpu(), "m": m.detach().contiguous().cpu(),
               "v": v.detach().contiguous().cpu()}, path, metadata=meta)


def load(path: str, device="cpu") -> dict:
    """Read a checkpoint: {theta, m, v (on device), step, sampler, config}."""
    from safetensors import safe_open
    with safe_open(path, framework="pt") as f:
        meta = f.metadata() or {}
    if meta.get("format") != "efunc-checkpoint-1":
        raise ValueError(f"{path} is not an efunc checkpoint")
    t = load_file(path)
    return {"theta": t["theta"].to(device), "m": t["m"].to(device), "v": t["v"].to(device),
            "step": int(meta["step"]), "sampler": json.loads(meta["sampler"]),
            "config": json.loads(meta["config"])}
