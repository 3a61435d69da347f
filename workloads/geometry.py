"""Seeded synthetic inputs: level-set domains as signed distance functions.

This module holds no part of the multigrid method.  It produces the nodal phi that the
solver (and the oracle) take as input, and the analytic outward normal of each domain,
which the boundary data g_N needs.  The paper assumes phi is a signed distance function
(Sec. 2.2); every domain here therefore returns an SDF, either in closed form or by a
closest-point search on a parametric description of the boundary curve.
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree


def grid_points(dim: int, n: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """Node coordinates lo + h j, j in {0..n}^dim, x fastest; shape ((n+1)^dim, dim)."""
    h = (hi - lo) / n
    ax = lo + h * np.arange(n + 1, dtype=np.float64)
    mesh = np.meshgrid(*([ax] * dim), indexing="ij")  # mesh[a][j0, j1, ...]
    # x fastest: flat index = j0 + (n+1) j1 + (n+1)^2 j2 -> order axes reversed
    cols = [m.transpose(tuple(range(dim))[::-1]).ravel() for m in mesh]
    return np.stack(cols, axis=1)


class Domain:
    dim = 2

    def phi(self, P: np.ndarray) -> np.ndarray:  # signed distance, negative inside
        raise NotImplementedError

    def normal(self, P: np.ndarray) -> np.ndarray:  # outward unit normal of the SDF
        raise NotImplementedError

    def nodal_phi(self, n: int, lo=-1.0, hi=1.0) -> np.ndarray:
        return self.phi(grid_points(self.dim, n, lo, hi))


class Interval(Domain):
    dim = 1

    def __init__(self, a: float, b: float):
        self.a, self.b = a, b

    def phi(self, P):
        x = P[:, 0]
        return np.maximum(self.a - x, x - self.b)

    def normal(self, P):
        x = P[:, 0]
        return np.where(x > 0.5 * (self.a + self.b), 1.0, -1.0)[:, None]


class Disk(Domain):
    def __init__(self, center=(0.0, 0.0), radius=0.6):
        self.c = np.asarray(center, dtype=np.float64)
        self.r = float(radius)

    def phi(self, P):
        return np.sqrt(((P - self.c) ** 2).sum(axis=1)) - self.r

    def normal(self, P):
        d = P - self.c
        return d / np.sqrt((d ** 2).sum(axis=1))[:, None]


class ParametricCurve(Domain):
    """Closed counter-clockwise curve c(t), t in [0, 2 pi); SDF by nearest sample followed
    by Newton refinement of the closest-point parameter."""

    samples = 40000

    def c(self, t):
        raise NotImplementedError

    def dc(self, t):
        raise NotImplementedError

    def ddc(self, t):
        raise NotImplementedError

    def inside(self, P):
        raise NotImplementedError

    def _tree(self):
        if getattr(self, "_kd", None) is None:
            self._t = np.linspace(0.0, 2 * np.pi, self.samples, endpoint=False)
            self._kd = cKDTree(self.c(self._t))
        return self._kd

    def closest_param(self, P):
        kd = self._tree()
        out = np.empty(len(P))
        for s in range(0, len(P), 1 << 20):
            Q = P[s:s + (1 << 20)]
            _, i = kd.query(Q)
            t = self._t[i].copy()
            dt = 2 * np.pi / self.samples
            best = ((self.c(t) - Q) ** 2).sum(axis=1)
            tb = t.copy()
            for _ in range(4):
                cc, d1, d2 = self.c(t), self.dc(t), self.ddc(t)
                diff = cc - Q
                F = (diff * d1).sum(axis=1)
                dF = (d1 * d1).sum(axis=1) + (diff * d2).sum(axis=1)
                step = np.where(dF > 0, F / np.where(dF > 0, dF, 1.0), 0.0)
                t = t - np.clip(step, -4 * dt, 4 * dt)
                dd = ((self.c(t) - Q) ** 2).sum(axis=1)
                better = dd < best
                best = np.where(better, dd, best)
                tb = np.where(better, t, tb)
            out[s:s + len(Q)] = tb
        return out

    def phi(self, P):
        t = self.closest_param(P)
        d = np.sqrt(((self.c(t) - P) ** 2).sum(axis=1))
        return np.where(self.inside(P), -d, d)

    def normal(self, P):
        t = self.closest_param(P)
        d1 = self.dc(t)
        n = np.stack([d1[:, 1], -d1[:, 0]], axis=1)
        return n / np.sqrt((n ** 2).sum(axis=1))[:, None]


class Flower(ParametricCurve):
    """r = r0 + amp sin(k theta).  amp = 0.15 is the large-scale flower; amp = 1/5 is the
    flower of the paper's last test (its quintic fraction equals sin(5 theta)/5)."""

    def __init__(self, r0=0.5, amp=0.15, k=5):
        self.r0, self.amp, self.k = r0, amp, k

    def phi(self, P):
        # for odd k the curve is symmetric about the y axis; evaluating at (|x|, y) makes
        # the nodal SDF mirror-symmetric bit for bit on a grid symmetric about x = 0
        if self.k % 2 == 1:
            P = np.stack([np.abs(P[:, 0]), P[:, 1]], axis=1)
        return super().phi(P)

    def nodal_phi(self, n: int, lo=-1.0, hi=1.0) -> np.ndarray:
        if self.k % 2 == 0 or lo != -hi or n % 2:
            return super().nodal_phi(n, lo, hi)
        # evaluate the columns x >= 0 only and mirror them (the grid is symmetric)
        h = (hi - lo) / n
        ax = lo + h * np.arange(n + 1, dtype=np.float64)
        half = ax[n // 2:]
        X, Y = np.meshgrid(half, ax)  # Y rows, X columns
        vals = super().phi(np.stack([X.ravel(), Y.ravel()], axis=1)).reshape(n + 1, -1)
        full = np.concatenate([vals[:, :0:-1], vals], axis=1)
        return full.ravel()

    def _r(self, t):
        return (self.r0 + self.amp * np.sin(self.k * t), self.amp * self.k * np.cos(self.k * t),
                -self.amp * self.k ** 2 * np.sin(self.k * t))

    def c(self, t):
        r, _, _ = self._r(t)
        return np.stack([r * np.cos(t), r * np.sin(t)], axis=1)

    def dc(self, t):
        r, r1, _ = self._r(t)
        return np.stack([r1 * np.cos(t) - r * np.sin(t), r1 * np.sin(t) + r * np.cos(t)], axis=1)

    def ddc(self, t):
        r, r1, r2 = self._r(t)
        return np.stack([r2 * np.cos(t) - 2 * r1 * np.sin(t) - r * np.cos(t),
                         r2 * np.sin(t) + 2 * r1 * np.cos(t) - r * np.sin(t)], axis=1)

    def inside(self, P):
        th = np.arctan2(P[:, 1], P[:, 0])
        return np.hypot(P[:, 0], P[:, 1]) < self.r0 + self.amp * np.sin(self.k * th)


class Ellipse(ParametricCurve):
    def __init__(self, center=(0.0, 0.0), a=0.5, b=0.3, rot=0.0):
        self.cen = np.asarray(center, dtype=np.float64)
        self.a, self.b, self.rot = float(a), float(b), float(rot)
        cr, sr = np.cos(rot), np.sin(rot)
        self.R = np.array([[cr, -sr], [sr, cr]])

    def c(self, t):
        loc = np.stack([self.a * np.cos(t), self.b * np.sin(t)], axis=1)
        return loc @ self.R.T + self.cen

    def dc(self, t):
        return np.stack([-self.a * np.sin(t), self.b * np.cos(t)], axis=1) @ self.R.T

    def ddc(self, t):
        return np.stack([-self.a * np.cos(t), -self.b * np.sin(t)], axis=1) @ self.R.T

    def inside(self, P):
        loc = (P - self.cen) @ self.R
        return (loc[:, 0] / self.a) ** 2 + (loc[:, 1] / self.b) ** 2 < 1.0


class UnionOfEllipses(Domain):
    """min of the per-ellipse SDFs: exact outside, approximate inside near overlaps."""

    def __init__(self, ellipses):
        self.parts = list(ellipses)

    def phi(self, P):
        return np.min(np.stack([e.phi(P) for e in self.parts]), axis=0)

    def normal(self, P):
        vals = np.stack([e.phi(P) for e in self.parts])
        k = np.argmin(vals, axis=0)
        out = np.zeros_like(P)
        for i, e in enumerate(self.parts):
            m = k == i
            if m.any():
                out[m] = e.normal(P[m])
        return out


class PolylineCurve(Domain):
    """Closed curve given by dense ordered samples; SDF by projection on the nearest
    segments.  Used where no convenient parametrisation exists (the saddle domain)."""

    def __init__(self, pts: np.ndarray, phi0):
        self.pts = np.asarray(pts, dtype=np.float64)
        self.phi0 = phi0
        self.kd = cKDTree(self.pts)

    def _closest(self, P):
        m = len(self.pts)
        _, idx = self.kd.query(P, k=4)
        best = np.full(len(P), np.inf)
        cp = np.zeros_like(P)
        tang = np.zeros_like(P)
        for c in range(idx.shape[1]):
            i = idx[:, c]
            for j0, j1 in ((i - 1) % m, i), (i, (i + 1) % m):
                A, B = self.pts[j0], self.pts[j1]
                AB = B - A
                L2 = (AB ** 2).sum(axis=1)
                s = np.clip(((P - A) * AB).sum(axis=1) / np.where(L2 > 0, L2, 1.0), 0, 1)
                Q = A + s[:, None] * AB
                d = ((P - Q) ** 2).sum(axis=1)
                bt = d < best
                best = np.where(bt, d, best)
                cp[bt] = Q[bt]
                tang[bt] = AB[bt]
        return np.sqrt(best), cp, tang

    def phi(self, P):
        d, _, _ = self._closest(P)
        return np.where(self.phi0(P) < 0, -d, d)

    def normal(self, P):
        _, _, t = self._closest(P)
        n = np.stack([t[:, 1], -t[:, 0]], axis=1)
        n /= np.sqrt((n ** 2).sum(axis=1))[:, None]
        # orient outwards: phi0 grows along the outward normal
        probe = self.phi0(P + 1e-6 * n) - self.phi0(P - 1e-6 * n)
        return np.where((probe >= 0)[:, None], n, -n)


def saddle_domain(samples: int = 200000) -> PolylineCurve:
    """The saddle-shaped domain of the paper's Sec. 3.3 test: with p = (sqrt3/2) x + y/2,
    q = x/2 - (sqrt3/2) y and tau = 3p - 1, phi0 = 9 q^2 + tau^2 sin(tau) - 1."""
    from scipy.optimize import brentq

    s3 = np.sqrt(3.0)

    def phi0(P):
        x, y = P[:, 0], P[:, 1]
        q = 0.5 * x - 0.5 * s3 * y
        tau = 1.5 * s3 * x + 1.5 * y - 1.0
        return 9.0 * q ** 2 + tau ** 2 * np.sin(tau) - 1.0

    fz = lambda t: 1.0 - t * t * np.sin(t)
    tmin = brentq(fz, -3.6, -np.pi)
    tmax = brentq(fz, 0.5, 1.5)
    psi = np.linspace(0, 2 * np.pi, samples, endpoint=False)
    tau = 0.5 * (tmax + tmin) + 0.5 * (tmax - tmin) * np.cos(psi)
    q = np.sign(np.sin(psi)) * np.sqrt(np.maximum(0.0, fz(tau))) / 3.0
    p = (tau + 1.0) / 3.0
    x = 0.5 * s3 * p + 0.5 * q
    y = 0.5 * p - 0.5 * s3 * q
    return PolylineCurve(np.stack([x, y], axis=1), phi0)


def rotated_ellipse_paper() -> Ellipse:
    """Sec. 3.3 ellipse: semi-axes 0.563 and 0.263 about (sqrt2/20, sqrt3/30) in the
    coordinates rotated by pi/6 (the second map printed as X is read as Y)."""
    # phi0 = ((X - cx)/0.563)^2 + ((Y - cy)/0.263)^2 - 1 with (X, Y) = R(pi/6)(x, y);
    # the zero set is the ellipse with centre R(-pi/6)(cx, cy) rotated by -pi/6.
    c = np.array([np.sqrt(2) / 20, np.sqrt(3) / 30])
    th = np.pi / 6
    Rm = np.array([[np.cos(th), np.sin(th)], [-np.sin(th), np.cos(th)]])  # R(-pi/6)
    return Ellipse(center=Rm @ c, a=0.563, b=0.263, rot=-th)


def paper_circle() -> Disk:
    return Disk(center=(np.sqrt(2) / 20, np.sqrt(3) / 30), radius=0.563)


class Torus(Domain):
    dim = 3

    def __init__(self, R=0.5, r=0.25):
        self.R, self.r = R, r

    def phi(self, P):
        rho = np.hypot(P[:, 0], P[:, 1])
        return np.hypot(rho - self.R, P[:, 2]) - self.r

    def normal(self, P):
        rho = np.hypot(P[:, 0], P[:, 1])
        rs = np.where(rho > 0, rho, 1.0)
        v = np.stack([(rho - self.R) * P[:, 0] / rs, (rho - self.R) * P[:, 1] / rs, P[:, 2]],
                     axis=1)
        return v / np.sqrt((v ** 2).sum(axis=1))[:, None]


