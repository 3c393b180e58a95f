"""Analytic signed-distance targets for the synthetic fitting workloads.

These stand in for the paper's meshes, which are not available here: a
centred sphere, and smooth unions of seeded random spheres and boxes,
optionally with a sinusoidal displacement.  Evaluation is float64 and runs on
whatever torch device the caller passes (CPU for tests, the GPU for
multi-million-point batches); nothing here is part of the fitted method.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import torch


def sphere_sdf(q: torch.Tensor, radius: float = 0.5) -> torch.Tensor:
    return torch.linalg.vector_norm(q, dim=-1) - radius


def smin(a: torch.Tensor, b: torch.Tensor, k: float) -> torch.Tensor:
    """Polynomial smooth minimum: min(a, b) - max(k - |a - b|, 0)^2 / (4k)."""
    hcl = torch.clamp(k - torch.abs(a - b), min=0.0)
    return torch.minimum(a, b) - hcl * hcl / (4.0 * k)


def _quat_to_matrix(qt: np.ndarray) -> np.ndarray:
    w, x, y, z = qt / np.linalg.norm(qt)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


@dataclass
class Primitive:
    kind: str                 # "sphere" or "box"
    centre: np.ndarray        # (3,)
    radius: float = 0.0       # sphere
    half: np.ndarray = field(default_factory=lambda: np.zeros(3))  # box half-extents
    rot: np.ndarray = field(default_factory=lambda: np.eye(3))     # box local->world

    def sdf(self, q: torch.Tensor) -> torch.Tensor:
        c = torch.as_tensor(self.centre, dtype=q.dtype, device=q.device)
        if self.kind == "sphere":
            return torch.linalg.vector_norm(q - c, dim=-1) - self.radius
        rot = torch.as_tensor(self.rot, dtype=q.dtype, device=q.device)
        b = torch.as_tensor(self.half, dtype=q.dtype, device=q.device)
        p = (q - c) @ rot            # world -> local: p_local = R^T (q - c)
        d = torch.abs(p) - b
        outside = torch.linalg.vector_norm(torch.clamp(d, min=0.0), dim=-1)
        inside = torch.clamp(torch.max(d, dim=-1).values, max=0.0)
        return outside + inside

    def area(self) -> float:
        if self.kind == "sphere":
            return 4.0 * np.pi * self.radius ** 2
        a, b, c = self.half
        return 8.0 * (a * b + a * c + b * c)

    def sample_surface(self, n: int, rng: np.random.Generator) -> np.ndarray:
        """Uniform-area samples on the primitive's own surface."""
        if self.kind == "sphere":
            u = rng.standard_normal((n, 3))
            u /= np.linalg.norm(u, axis=1, keepdims=True)
            return self.centre + self.radius * u
        a, b, c = self.half
        # faces: +-x (area 4bc), +-y (4ac), +-z (4ab)
        w = np.array([b * c, b * c, a * c, a * c, a * b, a * b])
        face = rng.choice(6, size=n, p=w / w.sum())
        uv = rng.uniform(-1.0, 1.0, size=(n, 2))
        p = np.empty((n, 3))
        axis = face // 2
        sign = np.where(face % 2 == 0, 1.0, -1.0)
        for ax in range(3):
            m = axis == ax
            o1, o2 = [x for x in range(3) if x != ax]
            p[m, ax] = sign[m] * self.half[ax]
            p[m, o1] = uv[m, 0] * self.half[o1]
            p[m, o2] = uv[m, 1] * self.half[o2]
        return self.centre + p @ self.rot.T


@dataclass
class CSGShape:
    """Left fold of smooth unions over the primitives, in their seeded order
    (the smooth minimum is not associative, so the order is part of the
    shape), plus an optional amp * sin(f x) sin(f y) sin(f z) displacement."""
    prims: list
    k: float = 0.05
    disp_amp: float = 0.0
    disp_freq: float = 20.0

    def sdf(self, q: torch.Tensor, chunk: int = 1 << 20) -> torch.Tensor:
        out = torch.empty(q.shape[0], dtype=q.dtype, device=q.device)
        for s in range(0, q.shape[0], chunk):
            qq = q[s:s + chunk]
            f = self.prims[0].sdf(qq)
            for p in self.prims[1:]:
                f = smin(f, p.sdf(qq), self.k)
            if self.disp_amp != 0.0:
                w = self.disp_freq
                f = f + self.disp_amp * torch.sin(w * qq[:, 0]) * torch.sin(w * qq[:, 1]) * \
                    torch.sin(w * qq[:, 2])
            out[s:s + chunk] = f
        return out


def random_csg(n_prims: int, seed: int, k: float = 0.05, disp_amp: float = 0.0,
               disp_freq: float = 20.0) -> CSGShape:
    """Seeded random smooth union: centres U[-0.6, 0.6]^3, 50/50 spheres
    (radius U[0.1, 0.35]) and boxes (half-extents U[0.1, 0.35] per axis,
    rotation from a normalised Gaussian quaternion)."""
    rng = np.random.default_rng(seed)
    prims = []
    for _ in range(n_prims):
        centre = rng.uniform(-0.6, 0.6, size=3)
        if rng.uniform() < 0.5:
            prims.append(Primitive("sphere", centre, radius=float(rng.uniform(0.1, 0.35))))
        else:
            half = rng.uniform(0.1, 0.35, size=3)
            rot = _quat_to_matrix(rng.standard_normal(4))
            prims.append(Primitive("box", centre, half=half, rot=rot))
    return CSGShape(prims, k=k, disp_amp=disp_amp, disp_freq=disp_freq)
