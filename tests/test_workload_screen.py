"""The learned-guess workload's rejection rule for topology the coarse grids cannot
represent (interior components that merge on a coarser level), decided from phi alone,
checked against what the oracle's multigrid does on the same problems: it converges where
the rule accepts and fails where it rejects."""
import numpy as np
import pytest

from oracle import Oracle, default_grid, OK
from workloads import ellipses as el

N, NC = 512, 32


def _levels(o):
    out = []
    for lev in range(o.nlev):
        c, _ = o.cls(lev)
        m = o.info(lev)["n"] + 1
        out.append(c.reshape(m, m))
    return out


@pytest.mark.parametrize("seed,merges", [(1_000_003, False), (1_000_049, False),
                                         (1_000_027, True), (1_000_078, True)])
def test_merge_rule_matches_oracle_convergence(seed, merges):
    from paper_1111_0983_amd.learned import components_merge

    p = el.draw(seed)
    phi = el.nodal_phi(p, N).numpy()
    assert el.accept(el.nodal_phi(p, N), N, 3.0 * 2.0 / NC)
    o = Oracle(phi, default_grid(2, N, NC), p.rule)
    assert components_merge(_levels(o)) == merges
    c, _ = o.cls(0)
    rhs = np.where(c == 1, el.nodal_f(p, N).numpy(), 0.0)
    st, _, h = o.solve(rhs, tol=1e-10, max_cycles=40)
    if merges:
        assert st != OK
    else:
        assert st == OK and len(h) <= 35


def test_merge_rule_on_hand_made_levels():
    from paper_1111_0983_amd.learned import components_merge

    a = np.zeros((9, 9), np.int8)
    a[2:4, 2:7] = 1
    a[5:7, 2:7] = 1           # two bars
    b = np.zeros((5, 5), np.int8)
    b[1:4, 1:4] = 1           # one block: the bars merged
    c = np.zeros((5, 5), np.int8)
    c[1, 1:4] = 1
    c[3, 1:4] = 1             # two bars kept
    assert components_merge([a, b])
    assert not components_merge([a, c])
    assert not components_merge([b, b])
