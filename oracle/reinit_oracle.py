"""FP64 CPU oracle of the level-set reinitialisation, Eq. (sdf) (Sec. 2.2).

TEST INFRASTRUCTURE ONLY: the test-suite and the benchmark's CPU baseline may import this
module; the product library never does.  It shares no code with the GPU kernel.

Eq. (sdf) evolves phi in pseudo-time, d phi / d t = sgn(phi0) (1 - |grad phi|), from
phi = phi0 until phi is a signed distance function a few mesh widths from the boundary (the
paper solves it "for a few time steps").  The paper fixes no scheme; it cites the upwind
(Godunov) discretisation of the Hamiltonian and the subcell fix of Russo and Smereka for
nodes next to the boundary.  Reading taken here, step by step:

1. Time step dt = h / 2 (within the CFL bound h / sqrt(d) of the upwind scheme), forward
   Euler, `iters` steps; phi0 is kept for the sign and the subcell fix.
2. One-sided differences along each axis a: Dm = (phi_i - phi_{i-1}) / h,
   Dp = (phi_{i+1} - phi_i) / h; a missing neighbour (a face of the box) counts as phi_i.
3. Godunov Hamiltonian: where phi0 > 0, |grad phi|^2 = sum_a max(max(Dm, 0)^2, min(Dp, 0)^2);
   where phi0 < 0, sum_a max(min(Dm, 0)^2, max(Dp, 0)^2).
4. Nodes next to the boundary (phi0 changes sign, or vanishes, towards an axis neighbour)
   take the subcell update phi <- phi - (dt / h) (sgn(phi0) |phi| - D), with D the distance
   estimated from phi0 alone: D = phi0 / |grad phi0|, |grad phi0| = sqrt(sum_a (g_a / h)^2),
   g_a = max(|phi0_{i+1} - phi0_{i-1}| / 2, |phi0_{i+1} - phi0_i|, |phi0_i - phi0_{i-1}|,
   1e-12 h) (the one-sided terms keep the estimate bounded where phi0 has a kink).
5. Every other node: phi <- phi - dt sgn(phi0) (|grad phi| - 1); sgn(0) = 0 keeps nodes on
   the boundary fixed.

Arrays are (n+1)^d nodes, x fastest (index j0 + (n+1) j1 + (n+1)^2 j2), as everywhere.
"""
from __future__ import annotations

import numpy as np


def _shape(phi, dim, n):
    return np.asarray(phi, dtype=np.float64).reshape((n + 1,) * dim)  # axes (z,) y, x


def _neighbours(a, axis):
    """(value at i - 1, value at i + 1) along one array axis; the face counts as the node."""
    lo = np.concatenate([np.take(a, [0], axis=axis), np.take(a, range(a.shape[axis] - 1),
                                                           axis=axis)], axis=axis)
    hi = np.concatenate([np.take(a, range(1, a.shape[axis]), axis=axis),
                         np.take(a, [a.shape[axis] - 1], axis=axis)], axis=axis)
    return lo, hi


def near_boundary(phi0, dim, n):
    """Nodes whose phi0 changes sign, or vanishes, towards an axis neighbour (including
    themselves on the boundary)."""
    p = _shape(phi0, dim, n)
    out = p == 0.0
    for ax in range(dim):
        lo, hi = _neighbours(p, ax)
        out |= (p * lo <= 0.0) | (p * hi <= 0.0)
    return out.reshape(-1)


def subcell_distance(phi0, dim, n, h):
    """D = phi0 / |grad phi0| with the bounded differences of step 4."""
    p = _shape(phi0, dim, n)
    g2 = np.zeros_like(p)
    for ax in range(dim):
        lo, hi = _neighbours(p, ax)
        ga = np.maximum.reduce([np.abs(hi - lo) / 2.0, np.abs(hi - p), np.abs(p - lo),
                                np.full_like(p, 1e-12 * h)])
        g2 += (ga / h) ** 2
    return (p / np.sqrt(g2)).reshape(-1)


def godunov_grad(phi, phi0, dim, n, h):
    """|grad phi| by the upwind (Godunov) rule of step 3, for the sign of phi0."""
    p = _shape(phi, dim, n)
    s = _shape(phi0, dim, n)
    tot_pos = np.zeros_like(p)
    tot_neg = np.zeros_like(p)
    for ax in range(dim):
        lo, hi = _neighbours(p, ax)
        dm = (p - lo) / h
        dp = (hi - p) / h
        tot_pos += np.maximum(np.maximum(dm, 0.0) ** 2, np.minimum(dp, 0.0) ** 2)
        tot_neg += np.maximum(np.minimum(dm, 0.0) ** 2, np.maximum(dp, 0.0) ** 2)
    return np.sqrt(np.where(s > 0.0, tot_pos, tot_neg)).reshape(-1)


def reinit(phi0, dim, n, iters, lo=-1.0, hi=1.0):
    """phi after `iters` forward-Euler steps of Eq. (sdf) from phi0."""
    h = (hi - lo) / n
    dt = 0.5 * h
    phi0 = np.asarray(phi0, dtype=np.float64).reshape(-1)
    sgn = np.sign(phi0)
    near = near_boundary(phi0, dim, n)
    D = subcell_distance(phi0, dim, n, h)
    phi = phi0.copy()
    for _ in range(iters):
        grad = godunov_grad(phi, phi0, dim, n, h)
        far_new = phi - dt * sgn * (grad - 1.0)
        near_new = phi - (dt / h) * (sgn * np.abs(phi) - D)
        phi = np.where(near, near_new, far_new)
    return phi
