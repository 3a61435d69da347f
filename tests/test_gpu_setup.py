"""The setup's classification runs on the GPU from phi in device memory; phi given in host
memory is uploaded first.  Both give the same hierarchy (classes and ghost records of every
level, bit for bit) and the same solve, in 2D and 3D, for one problem and for a batch."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from workloads import problems as pr, tank  # noqa: E402

DEV = "cuda:0"


def _cases():
    w = pr.flower(256, 16)
    yield "flower256", 2, 256, 16, np.ascontiguousarray(w.domain.nodal_phi(256)), [w.rule]
    w = pr.torus(64, 8)
    yield "torus64", 3, 64, 8, np.ascontiguousarray(w.domain.nodal_phi(64)), [w.rule]
    s = tank.TankSequence(64)
    phi = np.concatenate([s.phi(0, "cpu").numpy(), s.phi(5, "cpu").numpy()])
    yield "tank64x2", 3, 64, 16, np.ascontiguousarray(phi, dtype=np.float64), [s.rule, s.rule]


@pytest.mark.parametrize("case", list(_cases()), ids=lambda c: c[0])
def test_host_and_device_phi_give_the_same_hierarchy_and_solve(case):
    from paper_1111_0983_amd import ghostmg as gm
    name, dim, n, nc, phi, rules = case
    batch = len(rules)
    handles = [gm.Solver(phi, rules, gm.mg_grid_default(dim, n, nc, batch=batch)),
               gm.Solver(torch.from_numpy(phi).to(DEV), rules,
                         gm.mg_grid_default(dim, n, nc, batch=batch))]
    assert handles[0].nlev == handles[1].nlev
    for lev in range(handles[0].nlev):
        for p in range(batch):
            c0, c1 = handles[0].classes(p, lev), handles[1].classes(p, lev)
            assert np.array_equal(c0, c1), (lev, p)
            assert (c0 == 1).any() and (c0 == 2).any()
            g0, g1 = handles[0].ghosts(p, lev), handles[1].ghosts(p, lev)
            for k in g0:
                assert np.array_equal(g0[k], g1[k]), (lev, p, k)
    us = []
    for h in handles:
        c = torch.from_numpy(np.concatenate([h.classes(p) for p in range(batch)])).to(DEV)
        # the same right-hand side for both handles
        f = torch.from_numpy(np.random.default_rng(3).normal(size=c.numel())).to(DEV)
        f = torch.where(c == 1, f, torch.zeros_like(f)).contiguous()
        u = torch.zeros_like(f)
        info = h.solve(f, torch.zeros_like(f), u, tol=1e-10)
        assert info["rel"] <= 1e-10
        us.append(u.cpu().numpy())
        h.close()
    assert np.array_equal(us[0], us[1])


def test_non_finite_phi_is_rejected():
    from paper_1111_0983_amd import ghostmg as gm
    w = pr.flower(64, 8)
    phi = np.ascontiguousarray(w.domain.nodal_phi(64))
    phi[100] = np.nan
    with pytest.raises(gm.GhostMGError) as e:
        gm.Solver(torch.from_numpy(phi).to(DEV), [w.rule], gm.mg_grid_default(2, 64, 8))
    assert e.value.code == gm.MG_EINVAL
