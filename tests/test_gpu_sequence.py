"""The 3D projection-style sequence at its full size (384^3, moving ellipsoidal tank, FP32
cycles inside FP64 defect correction): every step reaches the tolerance from the warm start
(the previous step's solution) and from a cold start, and the oracle's own evaluation of the
discrete system (Eq. (discr)) confirms the defect of the last solution.  The cycle counts of
warm and cold starts are printed, not asserted: the previous solution differs from the new
one mostly at the moved boundary, which the cycle reduces no faster than a zero guess."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.slow]

from oracle import Oracle, default_grid  # noqa: E402


def test_tank_sequence_warm_start():
    from paper_1111_0983_amd import sequence
    from workloads import tank

    warm = sequence.run(steps=2, n=384, keep_last=True, log=None)
    cold = sequence.run(steps=1, n=384, start=1, warm=False, log=None)
    assert all(r <= 1e-10 for r in warm["rel"]) and cold["rel"][0] <= 1e-10
    print("cycles: steps 0, 1 warm", warm["cycles"], "step 1 cold", cold["cycles"])
    phi = warm["phi"].cpu().numpy()
    o = Oracle(phi, default_grid(3, 384, 24), tank.RULE)
    c, _ = o.cls(0)
    rhs = np.where(c == 1, warm["f"].cpu().numpy(), 0.0)  # g = 0 on every ghost
    _, (ni, ng) = o.defect(0, warm["u"].cpu().numpy(), rhs)
    assert max(ni, ng) / np.abs(rhs).max() <= 1.01e-10
