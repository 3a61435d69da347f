"""Seeded 3D projection-style sequence: an ellipsoidal tank moving through the box.

Step t of the sequence: the ellipsoid with semi-axes (0.8, 0.6, 0.5) centred at
c(t) = (0, -0.2 + 0.002 t, 0) on [-1, 1]^3; Dirichlet (p = 0) on the free surface z_B > 0.2,
homogeneous Neumann on the walls (g = 0 everywhere); f = a sum of 20 Gaussians fixed in the
tank's frame (amplitudes N(0, 1), widths U[0.05, 0.2], centres U[-0.4, 0.4]^3, seed 5), so
that the right-hand side moves with the tank.  The centre moves along y: moving along x
would carry the 0.8 semi-axis out of the box within the 200 steps.

The signed distance is exact: the closest point x of an axis-aligned ellipsoid to p solves
x_i = p_i a_i^2 / (a_i^2 + t) with sum_i (x_i / a_i)^2 = 1; the root t is found by
bisection on the interval where that sum decreases monotonically.  Points on the plane of
the smallest axis inside the tank, where no root lies in that interval, take the degenerate
branch t = -a_min^2.  Computed in torch (CPU or GPU).  This module holds none of the
solver's arithmetic.
"""
from __future__ import annotations

import numpy as np

AXES = (0.8, 0.6, 0.5)


def centre(t: int) -> tuple:
    return (0.0, -0.2 + 0.002 * t, 0.0)


RULE = dict(a=[0.0, 0.0, 1.0], c=-0.2, strict=1)  # Dirichlet where z_B > 0.2


def _grid(n, device, dtype):
    import torch

    x = torch.linspace(-1.0, 1.0, n + 1, device=device, dtype=dtype)
    return x


def ellipsoid_sdf(n: int, c=(0.0, 0.0, 0.0), axes=AXES, device="cpu", iters: int = 64,
                  slab: int = 32):
    """phi at the (n+1)^3 nodes of [-1, 1]^3 (x fastest), negative inside."""
    import torch

    dt = torch.float64
    x = _grid(n, device, dt)
    a = torch.tensor(axes, dtype=dt, device=device)
    a2 = a * a
    imin = int(torch.argmin(a).item())
    out = torch.empty((n + 1) ** 3, dtype=dt, device=device)
    npl = (n + 1) ** 2
    for z0 in range(0, n + 1, slab):
        z1 = min(n + 1, z0 + slab)
        Z, Y, X = torch.meshgrid(x[z0:z1], x, x, indexing="ij")
        p = torch.stack([(X - c[0]).abs(), (Y - c[1]).abs(), (Z - c[2]).abs()], dim=-1).reshape(-1, 3)
        inside = ((p / a) ** 2).sum(dim=1) < 1.0

        def g(t):
            return ((a * p / (a2 + t[:, None])) ** 2).sum(dim=1) - 1.0

        lo = torch.full((p.shape[0],), -float(a2[imin]), dtype=dt, device=device)
        hi = torch.clamp(p.norm(dim=1) * a.max(), min=1e-12)
        # the sum decreases on (-a_min^2, inf); with p_min = 0 it stays bounded at -a_min^2
        eps = 1e-12 * float(a2[imin])
        bracketed = g(lo + eps) > 0
        lo = lo + eps
        for _ in range(iters):
            mid = 0.5 * (lo + hi)
            pos = g(mid) > 0
            lo = torch.where(pos, mid, lo)
            hi = torch.where(pos, hi, mid)
        t = 0.5 * (lo + hi)
        xc = p * a2 / (a2 + t[:, None])
        # degenerate branch: t = -a_min^2, the free coordinate from the surface equation
        den = a2 - a2[imin]
        den[imin] = 1.0
        xd = p * a2 / den
        xd[:, imin] = 0.0
        rest = 1.0 - ((xd / a) ** 2).sum(dim=1)
        xd[:, imin] = a[imin] * torch.sqrt(torch.clamp(rest, min=0.0))
        use_d = ~bracketed & inside
        xs = torch.where(use_d[:, None], xd, xc)
        d = (xs - p).norm(dim=1)
        out[z0 * npl:z1 * npl] = torch.where(inside, -d, d)
    return out


class Gaussians:
    def __init__(self, seed: int = 5, k: int = 20):
        rng = np.random.default_rng(seed)
        self.A = rng.normal(0.0, 1.0, k)
        self.s = rng.uniform(0.05, 0.2, k)
        self.c = rng.uniform(-0.4, 0.4, (k, 3))

    def nodal(self, n: int, shift=(0.0, 0.0, 0.0), device="cpu"):
        import torch

        dt = torch.float64
        x = _grid(n, device, dt)
        Z, Y, X = torch.meshgrid(x, x, x, indexing="ij")
        f = torch.zeros_like(X)
        for A, s, c in zip(self.A, self.s, self.c):
            r2 = (X - shift[0] - c[0]) ** 2 + (Y - shift[1] - c[1]) ** 2 + (Z - shift[2] - c[2]) ** 2
            f += A * torch.exp(-r2 / (2.0 * s * s))
        return f.reshape(-1)


class TankSequence:
    """Inputs of step t: phi, f (g = 0), the BC rule."""

    def __init__(self, n: int = 384, seed: int = 5):
        self.n = n
        self.gauss = Gaussians(seed)
        self.rule = RULE

    def phi(self, t: int, device="cpu"):
        return ellipsoid_sdf(self.n, centre(t), AXES, device=device)

    def f(self, t: int, device="cpu"):
        return self.gauss.nodal(self.n, centre(t), device=device)
