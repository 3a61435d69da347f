"""The boundary relaxations the paper compares (Sec. 3.3): Kaczmarz sweeps over the band and
block relaxation of the band, in the oracle (GS-LEX, as in the paper).  Pinned by what the
mathematics fixes (a Kaczmarz step solves its equation and, on the homogeneous problem, never
lengthens u; a block step solves the equations of its block) and by the paper's measured
behaviour on the circle with the two-grid cycle at N = 64 (Fig. convFactLambda): the new
iteration reaches the interior smoothing limit (the local Fourier analysis value of Table
rholoc) after about five extra sweeps, Kaczmarz falls much more slowly with lambda, and block
relaxation is near that limit without extra sweeps."""
import numpy as np
import pytest

from oracle import Oracle, default_grid
from workloads import geometry as geo, problems as pr

N = 64
LFA = {2: 0.193, 3: 0.119}


@pytest.fixture(scope="module")
def circle():
    return geo.paper_circle().nodal_phi(N)


def _oracle(phi, smoother, lam, nu1=1, nu2=1):
    return Oracle(phi, default_grid(2, N, N // 2, nu1=nu1, nu2=nu2, gamma=1, lam=lam, ordering=0,
                                    split=1, smoother=smoother), pr.paper_rule())


def _rho(phi, smoother, lam, nu1=1, nu2=1):
    o = _oracle(phi, smoother, lam, nu1, nu2)
    c, _ = o.cls(0)
    u0 = np.where(c > 0, np.random.default_rng(1).uniform(-1, 1, c.size), 0.0)
    return o.rho(u0, max_cycles=200)[0]


def test_kaczmarz_step_solves_its_equation_and_never_lengthens_u(circle):
    o = _oracle(circle, 1, 5)
    c, band = o.cls(0)
    rng = np.random.default_rng(2)
    rhs = np.where(c > 0, rng.normal(size=c.size), 0.0)
    u = np.where(c > 0, rng.normal(size=c.size), 0.0)
    z = np.zeros_like(u)
    for P in np.flatnonzero(band)[::7]:
        o.boundary_step(0, P, u, rhs, 1)
        r, _ = o.defect(0, u, rhs)
        scale = max(1.0, abs(rhs[P]))
        assert abs(r[P]) <= 1e-9 * scale * (N / 2.0) ** 2, (P, r[P])
    # homogeneous problem: every step is an orthogonal projection onto a hyperplane through 0
    v = np.where(c > 0, rng.normal(size=c.size), 0.0)
    prev = np.linalg.norm(v)
    for P in np.flatnonzero(band):
        o.boundary_step(0, P, v, z, 1)
        nv = np.linalg.norm(v)
        assert nv <= prev * (1 + 1e-14)
        prev = nv


def test_block_step_solves_its_equations(circle):
    o = _oracle(circle, 2, 0)
    c, band = o.cls(0)
    G = o.ghosts(0)
    gi = {int(k): i for i, k in enumerate(G["node"])}
    rng = np.random.default_rng(3)
    rhs = np.where(c > 0, rng.normal(size=c.size), 0.0)
    u = np.where(c > 0, rng.normal(size=c.size), 0.0)
    for P in np.flatnonzero(band)[::5]:
        assert o.boundary_step(0, P, u, rhs, 2) == 0
        r, _ = o.defect(0, u, rhs)
        if c[P] == 2:
            blk = [k for k in G["wn"][gi[int(P)]] if k >= 0]
        else:
            jy, jx = divmod(int(P), N + 1)
            blk = [x + (N + 1) * y for y in (jy - 1, jy, jy + 1) for x in (jx - 1, jx, jx + 1)
                   if c[x + (N + 1) * y] > 0]
        assert np.abs(r[blk]).max() <= 1e-8 * (N / 2.0) ** 2, (P, np.abs(r[blk]).max())


@pytest.mark.parametrize("nu1,nu2", [(1, 1), (2, 1)])
def test_convergence_factor_against_lambda(circle, nu1, nu2):
    nu = nu1 + nu2
    new = [_rho(circle, 0, lam, nu1, nu2) for lam in (0, 2, 5, 8)]
    kac = [_rho(circle, 1, lam, nu1, nu2) for lam in (2, 5, 8)]
    blk = _rho(circle, 2, 0, nu1, nu2)
    print(f"nu {nu}: new {np.round(new, 3)}, Kaczmarz {np.round(kac, 3)}, block {blk:.3f}")
    # the new iteration: far from the limit without extra sweeps, at it by lambda = 5 and no
    # worse with more sweeps
    assert new[0] > 0.5 and new[1] > new[2]
    assert abs(new[2] - LFA[nu]) <= 0.05 and new[3] <= LFA[nu] + 0.05
    # Kaczmarz falls with lambda, more slowly
    assert kac[0] > kac[1] > kac[2] and kac[1] > new[2] + 0.2
    # block relaxation: at the limit with no extra sweep
    assert abs(blk - LFA[nu]) <= 0.05


def test_smoothing_factor_on_oscillating_error(circle):
    """Sec. 3.3: the relaxation alone on the error sin(40 pi x) sin(50 pi y): every scheme
    damps it strongly in its first sweeps (factors well below 1)."""
    P = geo.grid_points(2, N)
    for sm, lam in ((0, 5), (1, 5), (2, 0)):
        o = _oracle(circle, sm, lam)
        c, _ = o.cls(0)
        u0 = np.where(c > 0, np.sin(40 * np.pi * P[:, 0]) * np.sin(50 * np.pi * P[:, 1]), 0.0)
        mu = o.smoothing(u0, 4)
        assert np.all(mu[:3] < 0.5), (sm, mu)
