"""Seeded synthetic problems: manufactured solutions, boundary-condition rules and the
workloads the solver is measured on.

Nothing here belongs to the multigrid method.  ``rhs_from_ghosts`` fills the right-hand
side of Eq. (discr): f at interior nodes and g(B) at ghost nodes, where B is the closest
boundary point that *the caller's own* setup computed (the oracle and the GPU library each
pass their own B, so neither side's input depends on the other).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import geometry as geo


# ---- manufactured solutions -----------------------------------------------------------
class Manufactured:
    def u(self, P):
        raise NotImplementedError

    def grad(self, P):
        raise NotImplementedError

    def f(self, P):  # f = -Laplace(u)
        raise NotImplementedError


class ExpSin(Manufactured):
    """u = exp(x) sin(y): harmonic, so f = 0."""

    def u(self, P):
        return np.exp(P[:, 0]) * np.sin(P[:, 1])

    def grad(self, P):
        e = np.exp(P[:, 0])
        return np.stack([e * np.sin(P[:, 1]), e * np.cos(P[:, 1])], axis=1)

    def f(self, P):
        return np.zeros(len(P))


class SinCosXY(Manufactured):
    """u = sin(3x) cos(2y) + x y, f = 13 sin(3x) cos(2y)."""

    def u(self, P):
        x, y = P[:, 0], P[:, 1]
        return np.sin(3 * x) * np.cos(2 * y) + x * y

    def grad(self, P):
        x, y = P[:, 0], P[:, 1]
        return np.stack([3 * np.cos(3 * x) * np.cos(2 * y) + y,
                         -2 * np.sin(3 * x) * np.sin(2 * y) + x], axis=1)

    def f(self, P):
        x, y = P[:, 0], P[:, 1]
        return 13.0 * np.sin(3 * x) * np.cos(2 * y)


class ExpCos3D(Manufactured):
    """u = exp(x + y) cos(z), f = -exp(x + y) cos(z)."""

    def u(self, P):
        return np.exp(P[:, 0] + P[:, 1]) * np.cos(P[:, 2])

    def grad(self, P):
        e = np.exp(P[:, 0] + P[:, 1])
        return np.stack([e * np.cos(P[:, 2]), e * np.cos(P[:, 2]), -e * np.sin(P[:, 2])], axis=1)

    def f(self, P):
        return -np.exp(P[:, 0] + P[:, 1]) * np.cos(P[:, 2])


class Polynomial(Manufactured):
    """Quadratic polynomial u = c0 + b.x + x^T Q x (the patch test of the discretisation)."""

    def __init__(self, dim, rng):
        self.c0 = rng.uniform(-1, 1)
        self.b = rng.uniform(-1, 1, dim)
        A = rng.uniform(-1, 1, (dim, dim))
        self.Q = 0.5 * (A + A.T)

    def u(self, P):
        return self.c0 + P @ self.b + np.einsum("ni,ij,nj->n", P, self.Q, P)

    def grad(self, P):
        return self.b[None, :] + 2.0 * P @ self.Q

    def f(self, P):
        return np.full(len(P), -2.0 * np.trace(self.Q))


class Zero(Manufactured):
    def u(self, P):
        return np.zeros(len(P))

    def grad(self, P):
        return np.zeros_like(P)

    def f(self, P):
        return np.zeros(len(P))


# ---- boundary-condition rules ---------------------------------------------------------
def halfspace_rule(a, c=0.0, strict=True) -> dict:
    """Dirichlet where a.B + c > 0 (strict) or >= 0; Neumann elsewhere."""
    a = list(a) + [0.0] * (3 - len(a))
    return dict(a=a, c=float(c), strict=int(strict))


def paper_rule(dim=2) -> dict:
    """The paper's tests: Dirichlet on x <= 0, Neumann on x > 0 (Sec. 3)."""
    return halfspace_rule([-1.0] + [0.0] * (dim - 1), 0.0, strict=False)


# ---- right-hand side of Eq. (discr) ---------------------------------------------------
def rhs_from_ghosts(dim, n, cls, g_node, g_B, g_type, sol: Manufactured, domain: geo.Domain,
                    normal_override=None, lo=-1.0, hi=1.0):
    """f at interior nodes (cls == 1); g_D(B) = u(B) or g_N(B) = grad u(B) . n(B) at the
    ghost nodes, with n the analytic outward normal of the domain at B (or a supplied
    normal, e.g. the discrete n_B for the patch test)."""
    P = geo.grid_points(dim, n, lo, hi)
    rhs = np.zeros(len(P))
    inside = cls == 1
    rhs[inside] = sol.f(P[inside])
    if len(g_node):
        B = np.asarray(g_B)[:, :dim]
        nrm = domain.normal(B) if normal_override is None else np.asarray(normal_override)[:, :dim]
        gD = sol.u(B)
        gN = (sol.grad(B) * nrm).sum(axis=1)
        rhs[np.asarray(g_node)] = np.where(np.asarray(g_type) == 1, gD, gN)
    return rhs


# ---- the measured workloads -----------------------------------------------------------
@dataclass
class Workload:
    name: str
    dim: int
    n: int
    n_coarse: int
    domain: geo.Domain
    rule: dict
    solution: Manufactured
    description: str = ""
    extra: dict = field(default_factory=dict)


def disk64() -> Workload:
    """2D, box [-1,1]^2, 64 intervals, disk phi = r - 0.6; Dirichlet where y > 0, Neumann
    where y <= 0; u = exp(x) sin(y); coarsest grid 4."""
    return Workload("disk-64", 2, 64, 4, geo.Disk((0.0, 0.0), 0.6),
                    halfspace_rule([0.0, 1.0], 0.0, True), ExpSin(),
                    "2D disk r=0.6, N=64, Nc=4, Dirichlet y>0, u=exp(x)sin(y)")


def flower(n=2048, n_coarse=32) -> Workload:
    """2D flower r < 0.5 + 0.15 sin(5 theta) on [-1,1]^2; Dirichlet where x > 0, Neumann
    elsewhere; u = sin(3x) cos(2y) + x y."""
    return Workload(f"flower-{n}", 2, n, n_coarse, geo.Flower(0.5, 0.15, 5),
                    halfspace_rule([1.0, 0.0], 0.0, True), SinCosXY(),
                    f"2D flower r<0.5+0.15sin(5t), N={n}, Nc={n_coarse}, Dirichlet x>0, "
                    "u=sin(3x)cos(2y)+xy")


def torus(n=256, n_coarse=16) -> Workload:
    """3D torus (R, r) = (0.5, 0.25); Neumann where z < 0, Dirichlet where z >= 0;
    u = exp(x + y) cos(z)."""
    return Workload(f"torus-{n}", 3, n, n_coarse, geo.Torus(0.5, 0.25),
                    halfspace_rule([0.0, 0.0, 1.0], 0.0, False), ExpCos3D(),
                    f"3D torus R=0.5 r=0.25, N={n}, Nc={n_coarse}, Dirichlet z>=0, "
                    "u=exp(x+y)cos(z)")
