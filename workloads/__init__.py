"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke
check.  This package holds the workload recipes only (targets, samplers,
parameter initialisations drawn from a seed); none of the fitted method's
arithmetic lives here, so both the HIP path and the oracle consume exactly
the same arrays.

Each iteration of a fit draws half of its points uniformly in the bounding
cube and half near the surface (surface samples plus an isotropic Gaussian
offset), the per-iteration mix of the paper's Sec. 4.2.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

from .shapes import CSGShape, random_csg, sphere_sdf

NCH = 13


@dataclass(frozen=True)
class Workload:
    name: str
    R: int                 # vertices per axis
    J: int                 # points per iteration (half uniform, half near-surface)
    shape: str             # "sphere" or "csg"
    n_prims: int = 0
    shape_seed: int = 0
    disp_amp: float = 0.0
    disp_freq: float = 20.0
    sigma: float = 0.01    # near-surface Gaussian offset
    seed: int = 0          # batch seed base


WORKLOADS = {
    # tiny: sphere r=0.5, 8^3 grid, 65,536 points per iteration
    "sphere_r8": Workload("sphere_r8", R=8, J=1 << 16, shape="sphere", seed=0),
    # plain fused fit: smooth union of 16 primitives, 32^3 grid, 2^21 points per iteration
    "csg16_r32": Workload("csg16_r32", R=32, J=1 << 21, shape="csg", n_prims=16,
                          shape_seed=2, seed=100),
    # differentiation at scale: 256 primitives + displacement, 128^3 grid, 2^23 points
    "csg256_r128": Workload("csg256_r128", R=128, J=1 << 23, shape="csg", n_prims=256,
                            shape_seed=3, disp_amp=0.01, disp_freq=20.0, seed=200),
}



def batch_set(name: str = "batch64", n_shapes: int = 64, seed: int = 300,
              R_range=(16, 64), J_range=(1 << 18, 1 << 22), prims_range=(4, 64)) -> list:
    """A seeded set of independent shapes for batched fitting: per shape a
    smooth CSG union with a random primitive count, a lattice resolution R
    and a per-iteration point count J both log-uniform in the given ranges."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(n_shapes):
        R = int(round(np.exp(rng.uniform(np.log(R_range[0]), np.log(R_range[1])))))
        J = int(round(np.exp(rng.uniform(np.log(J_range[0]), np.log(J_range[1])))))
        n_prims = int(rng.integers(prims_range[0], prims_range[1] + 1))
        out.append(Workload(f"{name}_s{s:02d}", R=R, J=J, shape="csg", n_prims=n_prims,
                            shape_seed=1000 * seed + s, seed=1000 * seed + s))
    return out


_SHAPES: dict = {}
_POOLS: dict = {}


def get(name: str) -> Workload:
    return WORKLOADS[name]


def _shape(w: Workload) -> Optional[CSGShape]:
    if w.shape != "csg":
        return None
    key = (w.n_prims, w.shape_seed, w.disp_amp, w.disp_freq)
    if key not in _SHAPES:
        _SHAPES[key] = random_csg(w.n_prims, w.shape_seed, disp_amp=w.disp_amp,
                                  disp_freq=w.disp_freq)
    return _SHAPES[key]


def target(w: Workload, q: torch.Tensor) -> torch.Tensor:
    """Exact float64 signed distance of the workload's shape at q."""
    q = q.to(torch.float64)
    if w.shape == "sphere":
        return sphere_sdf(q, 0.5)
    return _shape(w).sdf(q)


def seed_for(w: Workload, iteration: int, salt: str = "") -> int:
    """Deterministic per-(workload, iteration) seed."""
    h = hashlib.sha256(f"{w.name}:{w.seed}:{iteration}:{salt}".encode()).digest()
    return int.from_bytes(h[:8], "little")


def _project(shape: CSGShape, p: np.ndarray, device, steps: int = 5, tol: float = 1e-6):
    """Newton projection onto the zero set, q <- q - F grad F / |grad F|^2,
    with a central-difference gradient; returns the points that converged."""
    q = torch.as_tensor(p, dtype=torch.float64, device=device)
    eps = 1e-6
    for _ in range(steps):
        f = shape.sdf(q)
        g = torch.empty_like(q)
        for ax in range(3):
            dq = torch.zeros(3, dtype=torch.float64, device=device)
            dq[ax] = eps
            g[:, ax] = (shape.sdf(q + dq) - shape.sdf(q - dq)) / (2 * eps)
        gn = (g * g).sum(-1).clamp(min=1e-30)
        q = q - (f / gn)[:, None] * g
    f = shape.sdf(q)
    ok = torch.abs(f) <= tol
    return q[ok].cpu().numpy()


def surface_points(w: Workload, n: int, seed: int, device="cpu") -> np.ndarray:
    """n seeded samples on the workload's zero level set (float64)."""
    rng = np.random.default_rng(seed)
    if w.shape == "sphere":
        u = rng.standard_normal((n, 3))
        return 0.5 * u / np.linalg.norm(u, axis=1, keepdims=True)
    shape = _shape(w)
    areas = np.array([p.area() for p in shape.prims])
    out = []
    have = 0
    acc = 0.5  # running estimate of the fraction of samples that survive
    while have < n:
        m = int(1.25 * (n - have) / acc) + 64
        counts = rng.multinomial(m, areas / areas.sum())
        pts = np.concatenate([p.sample_surface(c, rng) for p, c in zip(shape.prims, counts)
                              if c > 0])
        # discard samples buried inside another primitive
        qt = torch.as_tensor(pts, dtype=torch.float64, device=device)
        owner = np.repeat(np.arange(len(shape.prims)), counts)
        buried = torch.zeros(len(pts), dtype=torch.bool, device=device)
        for i, p in enumerate(shape.prims):
            d = p.sdf(qt)
            mine = torch.as_tensor(owner == i, device=device)
            buried |= (d < -1e-6) & ~mine
        pts = pts[~buried.cpu().numpy()]
        pts = _project(shape, pts, device)
        acc = min(1.0, max(0.02, len(pts) / m))
        # samples come grouped by primitive: shuffle before the final cut to n
        out.append(pts[rng.permutation(len(pts))])
        have += len(pts)
    pts = np.concatenate(out)[:n]
    return pts[rng.permutation(n)]


def _pool(w: Workload, device) -> np.ndarray:
    """A fixed pool of surface samples from which near-surface points are drawn."""
    key = w.name
    if key not in _POOLS:
        n = 1 << 18 if w.shape == "csg" else 1 << 16
        _POOLS[key] = surface_points(w, n, seed_for(w, -1, "pool"), device)
    return _POOLS[key]


def make_points(w: Workload, iteration: int, J: Optional[int] = None, device="cpu"):
    """Seeded query points of one iteration: J//2 uniform in [-1,1]^3 followed by
    J - J//2 near-surface points.  Returns float32 numpy (J, 3)."""
    J = w.J if J is None else J
    rng = np.random.default_rng(seed_for(w, iteration))
    nu = J // 2
    ns = J - nu
    uni = rng.uniform(-1.0, 1.0, size=(nu, 3))
    if w.shape == "sphere":
        u = rng.standard_normal((ns, 3))
        surf = 0.5 * u / np.linalg.norm(u, axis=1, keepdims=True)
    else:
        pool = _pool(w, device)
        surf = pool[rng.integers(0, len(pool), size=ns)]
    near = surf + w.sigma * rng.standard_normal((ns, 3))
    return np.concatenate([uni, near]).astype(np.float32)


def make_batch(w: Workload, iteration: int, J: Optional[int] = None, device="cpu"):
    """(q, o): float32 points and their float64-exact signed distances rounded
    to float32 (numpy arrays)."""
    q = make_points(w, iteration, J, device)
    o = target(w, torch.as_tensor(q, device=device)).to(torch.float32).cpu().numpy()
    return q, o


def plain_theta(R: int, rho0: float = 7.0) -> np.ndarray:
    """Parameter tensor before mean-shift: all values and offsets zero, both
    log-scales rho0 (beta = exp(7), Sec. 4.3 'Scales/radius')."""
    th = np.zeros((R, R, R, NCH), np.float32)
    th[..., 4] = rho0
    th[..., 12] = rho0
    return th


def perturbed_theta(R: int, seed: int, rho0: float = 7.0, rho_spread: float = 0.5,
                    offset_cells: float = 0.6, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """Seeded random parameters that exercise every gradient path: values
    U[-1,1], slopes N(0,1), log-scales rho0 + U[-spread, spread], offsets
    N(0, (offset_cells * h)^2) per axis."""
    rng = np.random.default_rng(seed)
    h = (hi - lo) / (R - 1)
    th = np.empty((R, R, R, NCH), np.float64)
    th[..., 0] = rng.uniform(-1, 1, size=(R, R, R))
    th[..., 1:4] = rng.standard_normal((R, R, R, 3))
    th[..., 4] = rho0 + rng.uniform(-rho_spread, rho_spread, size=(R, R, R))
    th[..., 5:8] = offset_cells * h * rng.standard_normal((R, R, R, 3))
    th[..., 8] = rng.uniform(-1, 1, size=(R, R, R))
    th[..., 9:12] = rng.standard_normal((R, R, R, 3))
    th[..., 12] = rho0 + rng.uniform(-rho_spread, rho_spread, size=(R, R, R))
    return th.astype(np.float32)
