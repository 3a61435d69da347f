"""Parity at the full sizes of the benchmark workloads, in the launch configuration the
benchmark times.  The reference is the discrete solution of Eq. (discr): a sparse direct
solve of the oracle's assembled rows (2D), or the oracle's own multigrid iterated to its
FP64 rounding floor (3D, where a direct solve is out of reach).  Every GPU solution must
match it to 1e-10 in the relative max norm, and the oracle's own evaluation of the rows must
put the GPU solution's defect at the 1e-10 target."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.slow]

import oracle as orc  # noqa: E402
from oracle import Oracle, default_grid  # noqa: E402
from workloads import geometry as geo, problems as pr  # noqa: E402

DEV = "cuda:0"
TOL = 1e-10


def _gm():
    from paper_1111_0983_amd import ghostmg as gm
    return gm


def _oracle_rel(o, u, rhs):
    """max(||r||_inf over Omega_h, over Gamma_h) / ||(f_h, g_h)||_inf, by the oracle."""
    _, (ni, ng) = o.defect(0, u, rhs)
    c, _ = o.cls(0)
    return max(ni, ng) / np.abs(rhs[c > 0]).max()


def _rel_diff(u, ref):
    return float(np.abs(u - ref).max() / np.abs(ref).max())


def _floor_solve(o, rhs, first_cycles=60):
    """The oracle's multigrid to the tolerance, then on until the relative defect stops
    falling (its rounding floor): the discrete solution to the last few bits."""
    st, u, h = o.solve(rhs, tol=TOL, max_cycles=first_cycles)
    assert st == 0, st
    best = h[-1]
    for _ in range(6):
        st, u2, h2 = o.solve(rhs, u0=u, tol=1e-15, max_cycles=2)
        u = u2
        if h2.min() > 0.5 * best:
            break
        best = min(best, h2.min())
    return u


def _gpu_solve(phi, rule, dim, n, nc, prec, make_rhs, tol=TOL):
    gm = _gm()
    s = gm.Solver(torch.from_numpy(phi).to(DEV), [rule],
                  gm.mg_grid_default(dim, n, nc, precision=prec, inner_cycles=2))
    c = s.classes()
    f, g = make_rhs(c, s.ghosts())
    u = torch.zeros(f.size, dtype=torch.float64, device=DEV)
    info = s.solve(torch.from_numpy(f).to(DEV), torch.from_numpy(g).to(DEV), u, tol=tol)
    assert info["status"] == 0 and info["rel"] <= tol, info
    s.close()
    return u.cpu().numpy(), c, info


@pytest.fixture(scope="module")
def flower2048():
    """phi, the oracle's level-0 system and its direct solution (the finest system does not
    depend on the coarsest grid)."""
    w = pr.flower(2048, 128)
    phi = w.domain.nodal_phi(2048)
    o = Oracle(phi, default_grid(2, 2048, 128), w.rule)
    c, _ = o.cls(0)
    G = o.ghosts(0)
    rhs = pr.rhs_from_ghosts(2, 2048, c, G["node"], G["B"], G["type"], w.solution, w.domain)
    ref = o.direct_solve(rhs)
    return w, phi, o, rhs, ref


@pytest.mark.parametrize("prec,nc", [("fp64", 128), ("fp32dc", 128), ("fp64", 32), ("fp32dc", 32)])
def test_flower_2048_matches_direct_solution(flower2048, prec, nc):
    """Coarsest grids of 128 (5 levels, the benchmark's) and of 32 (7 levels)."""
    gm = _gm()
    w, phi, o, rhs, ref = flower2048

    def make_rhs(c, G):
        P = geo.grid_points(2, 2048)
        f = np.where(c == 1, w.solution.f(P), 0.0)
        g = pr.rhs_from_ghosts(2, 2048, c, G["node"], G["B"], G["type"], w.solution, w.domain)
        return f, g

    u, c, info = _gpu_solve(phi, w.rule, 2, 2048, nc,
                            gm.MG_FP64 if prec == "fp64" else gm.MG_FP32_DC, make_rhs)
    d = _rel_diff(u, ref)
    print(f"flower 2048 {prec} Nc={nc}: {info['cycles']} cycles, rel {info['rel']:.2e}, "
          f"|u - u*| / |u*| = {d:.2e}")
    assert _oracle_rel(o, u, rhs) <= 1.01 * TOL
    assert d <= TOL
    assert np.all(u[c == 0] == 0.0)


@pytest.fixture(scope="module")
def torus256():
    w = pr.torus(256, 16)
    phi = w.domain.nodal_phi(256)
    o = Oracle(phi, default_grid(3, 256, 16), w.rule)
    c, _ = o.cls(0)
    G = o.ghosts(0)
    rhs = pr.rhs_from_ghosts(3, 256, c, G["node"], G["B"], G["type"], w.solution, w.domain)
    before = orc.threads()
    orc.threads(16)
    try:
        ref = _floor_solve(o, rhs)
    finally:
        orc.threads(before)
    return w, phi, o, rhs, ref


@pytest.mark.parametrize("prec", ["fp64", "fp32dc"])
def test_torus_256_matches_discrete_solution(torus256, prec):
    gm = _gm()
    w, phi, o, rhs, ref = torus256

    def make_rhs(c, G):
        P = geo.grid_points(3, 256)
        f = np.where(c == 1, w.solution.f(P), 0.0)
        g = pr.rhs_from_ghosts(3, 256, c, G["node"], G["B"], G["type"], w.solution, w.domain)
        return f, g

    u, c, info = _gpu_solve(phi, w.rule, 3, 256, 16,
                            gm.MG_FP64 if prec == "fp64" else gm.MG_FP32_DC, make_rhs)
    d = _rel_diff(u, ref)
    print(f"torus 256 {prec}: {info['cycles']} cycles, rel {info['rel']:.2e}, "
          f"|u - u*| / |u*| = {d:.2e}")
    assert _oracle_rel(o, u, rhs) <= 1.01 * TOL
    assert d <= TOL
    assert np.all(u[c == 0] == 0.0)


def test_tank_384_step_matches_discrete_solution():
    """Step 0 of the 3D projection sequence at its full size (384^3, FP32 cycles inside FP64
    defect correction, the benchmark's configuration) against the oracle's multigrid at its
    rounding floor."""
    gm = _gm()
    from workloads import tank

    seq = tank.TankSequence(384)
    phi_t = seq.phi(0, DEV)
    f_full = seq.f(0, DEV)
    s = gm.Solver(phi_t, [seq.rule],
                  gm.mg_grid_default(3, 384, 24, precision=gm.MG_FP32_DC, inner_cycles=2))
    c = torch.from_numpy(s.classes()).to(DEV)
    f = torch.where(c == 1, f_full, torch.zeros((), dtype=torch.float64, device=DEV)).contiguous()
    g = torch.zeros_like(f)
    u = torch.zeros_like(f)
    info = s.solve(f, g, u, tol=TOL)
    assert info["status"] == 0 and info["rel"] <= TOL
    s.close()
    ug = u.cpu().numpy()
    phi = phi_t.cpu().numpy()
    fa = f.cpu().numpy()
    del phi_t, f_full, f, g, u, c
    o = Oracle(phi, default_grid(3, 384, 24), tank.RULE)
    oc, _ = o.cls(0)
    rhs = np.where(oc == 1, fa, 0.0)  # g = 0 on every ghost
    before = orc.threads()
    orc.threads(16)
    try:
        ref = _floor_solve(o, rhs, first_cycles=40)
    finally:
        orc.threads(before)
    d = _rel_diff(ug, ref)
    print(f"tank 384 step 0: {info['cycles']} FP32 cycles, rel {info['rel']:.2e}, "
          f"|u - u*| / |u*| = {d:.2e}")
    assert _oracle_rel(o, ug, rhs) <= 1.01 * TOL
    assert d <= TOL


def test_ellipse_batch_512():
    """The learned-guess workload: 64 seeded ellipse-union problems at 512^2 (after the
    workload's rejections, all decided from phi) solved as one batch in FP32 defect
    correction; every problem must reach the tolerance, and the oracle's evaluation of four
    of them confirms it."""
    gm = _gm()
    from paper_1111_0983_amd import learned

    seeds = list(range(1_000_000, 1_000_000 + 320))
    s, f, g, probs = learned.build_batch(seeds, precision=gm.MG_FP32_DC)
    if len(probs) > 64:
        s.close()
        s, f, g, probs = learned.build_batch([p.seed for p in probs[:64]],
                                             precision=gm.MG_FP32_DC)
    assert len(probs) == 64
    u = torch.zeros_like(f)
    info = s.solve(f, g, u, tol=TOL, check=False)
    assert info["status"] == gm.MG_OK, info
    from workloads import ellipses as el

    nn = 513 * 513
    fa, ua = f.cpu().numpy(), u.cpu().numpy()
    rels = s.residual(f, g, u).max(axis=1)
    for i in (0, len(probs) // 3, 2 * len(probs) // 3, len(probs) - 1):
        p = probs[i]
        phi = el.nodal_phi(p, 512, device=DEV).cpu().numpy()
        o = Oracle(phi, default_grid(2, 512, 32), p.rule)
        c, _ = o.cls(0)
        rhs = np.where(c == 1, fa[i * nn:(i + 1) * nn], 0.0)  # g = 0 on every ghost
        rel_o = _oracle_rel(o, ua[i * nn:(i + 1) * nn], rhs)
        rel_g = rels[i] / np.abs(rhs).max()
        assert abs(rel_o - rel_g) <= 1e-3 * rel_g + 1e-15, (i, rel_o, rel_g)
        assert rel_o <= 1.01 * TOL
