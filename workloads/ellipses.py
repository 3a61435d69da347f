"""Seeded random problems on unions of ellipses (the learned-initial-guess workload).

Each problem: phi = min over 1-4 ellipses of their exact signed distance functions (exact
outside, approximate inside near overlaps); f = sum of 8 Gaussians; g = 0; Dirichlet on one
side of a random line, Neumann on the rest.  Samples whose domain comes within 3 coarsest
mesh widths of the box are rejected.

The SDF is computed in torch (CPU or GPU) in batches: the closest point of an ellipse in
its local frame solves (x - p_x) a_x... by a Newton iteration on the angle parameter started
from two points, keeping the better.  This module holds none of the solver's arithmetic.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class EllipseProblem:
    seed: int
    centers: np.ndarray   # (k, 2)
    axes: np.ndarray      # (k, 2)
    rot: np.ndarray       # (k,)
    p: np.ndarray         # point on the Dirichlet/Neumann line
    nu: np.ndarray        # unit normal of the line: Dirichlet where (B - p) . nu > 0
    amp: np.ndarray       # (8,) Gaussian amplitudes
    sig: np.ndarray       # (8,) widths
    gc: np.ndarray        # (8, 2) Gaussian centres

    @property
    def rule(self) -> dict:
        return dict(a=[float(self.nu[0]), float(self.nu[1]), 0.0],
                    c=float(-self.p @ self.nu), strict=1)


def draw(seed: int) -> EllipseProblem:
    rng = np.random.default_rng(seed)
    k = int(rng.integers(1, 5))
    centers = rng.uniform(-0.6, 0.6, (k, 2))
    axes = rng.uniform(0.15, 0.5, (k, 2))
    rot = rng.uniform(0.0, np.pi, k)
    p = rng.uniform(-0.3, 0.3, 2)
    ang = rng.uniform(0.0, 2 * np.pi)
    nu = np.array([np.cos(ang), np.sin(ang)])
    amp = rng.normal(0.0, 1.0, 8)
    sig = rng.uniform(0.05, 0.2, 8)
    gc = rng.uniform(-0.6, 0.6, (8, 2))
    return EllipseProblem(seed, centers, axes, rot, p, nu, amp, sig, gc)


def _ellipse_sdf_torch(X, Y, cx, cy, a, b, th, iters=12):
    import torch

    c, s = np.cos(th), np.sin(th)
    qx = (X - cx) * c + (Y - cy) * s
    qy = -(X - cx) * s + (Y - cy) * c
    px, py = qx.abs(), qy.abs()
    best = None
    for t0 in (torch.atan2(a * py, b * px), torch.full_like(px, np.pi / 4)):
        t = t0.clamp(0.0, np.pi / 2)
        for _ in range(iters):
            ct, st = torch.cos(t), torch.sin(t)
            ex, ey = a * ct - px, b * st - py
            dx, dy = -a * st, b * ct
            F = ex * dx + ey * dy
            dF = dx * dx + dy * dy + ex * (-a * ct) + ey * (-b * st)
            step = torch.where(dF > 0, F / torch.where(dF > 0, dF, torch.ones_like(dF)),
                               torch.zeros_like(dF))
            t = (t - step.clamp(-0.5, 0.5)).clamp(0.0, np.pi / 2)
        d = torch.sqrt((a * torch.cos(t) - px) ** 2 + (b * torch.sin(t) - py) ** 2)
        best = d if best is None else torch.minimum(best, d)
    inside = (qx / a) ** 2 + (qy / b) ** 2 < 1.0
    return torch.where(inside, -best, best)


def nodal_phi(prob: EllipseProblem, n: int, device="cpu", dtype=None):
    """phi at the (n+1)^2 nodes of [-1, 1]^2 (x fastest) as a torch tensor."""
    import torch

    dtype = dtype or torch.float64
    h = 2.0 / n
    ax = -1.0 + h * torch.arange(n + 1, dtype=dtype, device=device)
    Y, X = torch.meshgrid(ax, ax, indexing="ij")
    phi = None
    for (cx, cy), (a, b), th in zip(prob.centers, prob.axes, prob.rot):
        d = _ellipse_sdf_torch(X, Y, float(cx), float(cy), float(a), float(b), float(th))
        phi = d if phi is None else torch.minimum(phi, d)
    return phi.reshape(-1)


def nodal_f(prob: EllipseProblem, n: int, device="cpu", dtype=None):
    import torch

    dtype = dtype or torch.float64
    h = 2.0 / n
    ax = -1.0 + h * torch.arange(n + 1, dtype=dtype, device=device)
    Y, X = torch.meshgrid(ax, ax, indexing="ij")
    f = torch.zeros_like(X)
    for A, s, (cx, cy) in zip(prob.amp, prob.sig, prob.gc):
        f += float(A) * torch.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2.0 * float(s) ** 2))
    return f.reshape(-1)


def accept(phi, n: int, margin: float = 0.1875) -> bool:
    """Reject domains that come within `margin` of the box faces."""
    import torch

    h = 2.0 / n
    ax = -1.0 + h * torch.arange(n + 1, dtype=phi.dtype, device=phi.device)
    Y, X = torch.meshgrid(ax, ax, indexing="ij")
    near = (X.abs() > 1.0 - margin) | (Y.abs() > 1.0 - margin)
    return not bool(((phi.reshape(n + 1, n + 1) < 0) & near).any())
