"""Pins of the reinitialisation oracle (Eq. (sdf), Sec. 2.2) against what the mathematics
fixes: a signed distance function of a plane is reached exactly (to rounding) from any
positive multiple of it; the circle's distance is reached to second order in h; the zero
set never moves (every node keeps the sign of phi0); the subcell distance estimate is exact
for linear phi0."""
import numpy as np

from oracle import reinit_oracle as ro
from workloads import geometry as geo


def test_plane_becomes_its_distance_function():
    """Away from the faces of the box (where a missing neighbour truncates the upwind
    difference) the plane's distance function is the scheme's fixed point, reached to
    rounding."""
    n = 64
    P = geo.grid_points(2, n)
    h = 2.0 / n
    d = (P[:, 0] - 0.1) * 0.8 + (P[:, 1] + 0.05) * 0.6   # unit normal (0.8, 0.6)
    phi = ro.reinit(3.0 * d, 2, n, 200)
    m = (np.abs(d) < 10 * h) & (np.abs(P[:, 0]) < 0.6) & (np.abs(P[:, 1]) < 0.6)
    assert np.abs(phi - d)[m].max() < 1e-13


def test_subcell_distance_exact_for_linear_phi0():
    n = 32
    P = geo.grid_points(3, n)
    d = (P[:, 0] - 0.1)
    D = ro.subcell_distance(5.0 * d, 3, n, 2.0 / n)
    assert np.abs(D - d).max() < 1e-14


def test_circle_distance_second_order():
    errs = []
    for n in (64, 128, 256):
        P = geo.grid_points(2, n)
        h = 2.0 / n
        phi0 = (P ** 2).sum(axis=1) - 0.5 ** 2
        phi = ro.reinit(phi0, 2, n, 40)
        ex = np.sqrt((P ** 2).sum(axis=1)) - 0.5
        errs.append(np.abs(phi - ex)[np.abs(ex) < 3 * h].max())
        assert np.all(np.sign(phi) == np.sign(phi0))
    ratios = [errs[i] / errs[i + 1] for i in range(2)]
    assert all(3.5 < r < 4.5 for r in ratios), (errs, ratios)


def test_sphere_3d_sign_and_second_order():
    errs = []
    for n in (24, 48):
        P = geo.grid_points(3, n)
        h = 2.0 / n
        phi0 = np.exp((P ** 2).sum(axis=1)) - np.exp(0.45 ** 2)  # the zero set of r - 0.45
        phi = ro.reinit(phi0, 3, n, 30)
        ex = np.sqrt((P ** 2).sum(axis=1)) - 0.45
        assert np.all(np.sign(phi) == np.sign(phi0))
        errs.append(np.abs(phi - ex)[np.abs(ex) < 4 * h].max())
    assert 3.0 < errs[0] / errs[1] < 5.0, errs
