"""mg_setup_partition: a boundary partition given as a function of the closest boundary
point (Sec. 2.1), checked against the oracle's function-driven setup."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import Oracle, default_grid  # noqa: E402
from workloads import geometry as geo, problems as pr  # noqa: E402

DEV = "cuda:0"


def _gm():
    from paper_1111_0983_amd import ghostmg as gm
    return gm


def _two_arcs(B):
    return abs(B[1]) > 0.3


def _quadrants(B):
    return B[0] * B[1] > 0.0


def _case(name):
    if name == "disk64":
        w = pr.disk64()
        return w, 64, 4, _two_arcs
    w = pr.flower(256, 32)
    return w, 256, 32, _quadrants


def test_partition_function_equals_rule():
    gm = _gm()
    w = pr.flower(256, 32)
    phi = torch.from_numpy(w.domain.nodal_phi(256)).to(DEV)
    r = w.rule
    a = list(r["a"]) + [0.0] * 3

    def part(p, B):
        v = r.get("c", 0.0) + sum(a[k] * B[k] for k in range(3))
        return v > 0.0 if r.get("strict", 1) else v >= 0.0

    s1 = gm.Solver(phi, [r], gm.mg_grid_default(2, 256, 32))
    s2 = gm.Solver(phi, None, gm.mg_grid_default(2, 256, 32), partition=part)
    for lev in range(s1.nlev):
        g1, g2 = s1.ghosts(0, lev), s2.ghosts(0, lev)
        for k in g1:
            assert np.array_equal(g1[k], g2[k]), (lev, k)
    c = s1.classes()
    G = s1.ghosts()
    P = geo.grid_points(2, 256)
    f = torch.from_numpy(np.where(c == 1, w.solution.f(P), 0.0)).to(DEV)
    g = torch.from_numpy(pr.rhs_from_ghosts(2, 256, c, G["node"], G["B"], G["type"],
                                            w.solution, w.domain)).to(DEV)
    u1, u2 = torch.zeros_like(f), torch.zeros_like(f)
    s1.solve(f, g, u1, tol=1e-10)
    s2.solve(f, g, u2, tol=1e-10)
    assert torch.equal(u1, u2)


@pytest.mark.parametrize("name", ["disk64", "flower256"])
def test_partition_matches_oracle(name):
    gm = _gm()
    w, n, nc, part = _case(name)
    phi = w.domain.nodal_phi(n)
    s = gm.Solver(torch.from_numpy(phi).to(DEV), None, gm.mg_grid_default(2, n, nc),
                  partition=lambda p, B: part(B))
    o = Oracle(phi, default_grid(2, n, nc), partition=part)
    G, OG = s.ghosts(), o.ghosts(0)
    assert np.array_equal(G["type"], OG["type"])
    assert 0 < G["type"].sum() < len(G["type"])
    c, _ = o.cls(0)
    rhs = pr.rhs_from_ghosts(2, n, c, OG["node"], OG["B"], OG["type"], w.solution, w.domain)
    rng = np.random.default_rng(3)
    u0 = np.where(c > 0, rng.uniform(-1, 1, c.size), 0.0)
    uo = u0.copy()
    ug = torch.from_numpy(u0.copy()).to(DEV)
    rt = torch.from_numpy(rhs).to(DEV)
    for k in range(4):
        o.cycle(uo, rhs)
        s.cycles(rt, rt, ug, 1)
        err = np.abs(ug.cpu().numpy() - uo).max() / np.abs(uo).max()
        assert err <= 1e-12, (k, err)
    u = torch.zeros_like(rt)
    info = s.solve(rt, rt, u, tol=1e-11)
    assert info["status"] == 0
    ref = o.direct_solve(rhs)
    assert np.abs(u.cpu().numpy() - ref).max() <= 1e-10 * np.abs(ref).max()
