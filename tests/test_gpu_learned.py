"""The learned initial guess end to end on a small budget: solver-generated training data,
training with the BF16 MFMA kernels, and solves from the learned guess that still reach the
tolerance and agree with the zero-guess FP64 solution.  The per-problem cycle counts with and
without the guess (what the network gains) are measured and printed; they are not asserted,
since the gain of a guess interpolated from a coarse level is not positive for this solver."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_learned_guess_pipeline():
    from paper_1111_0983_amd import cnn, learned
    data = learned.generate(192, seed0=0, log=None)
    assert data["x"].shape[0] == 192
    net = cnn.GuessNet(seed=0)
    val = learned.generate(64, seed0=50000, log=None)
    before = learned.validate(net, val)
    learned.train(net, data, 400, batch=32, lr=3e-3, log=None)
    after = learned.validate(net, val)
    assert after < 0.8 * before, (before, after)
    seeds = [1_000_000 + i for i in range(40)]
    res = learned.evaluate(net, seeds, reps=1)
    assert res["problems"] >= 4
    assert res["fp32dc_learned"]["rel"] <= 1e-10 and res["fp64_zero"]["rel"] <= 1e-10
    assert res["fp32dc_learned"]["diff_vs_fp64"] <= 1e-9
    pp = res["per_problem"]
    print("cycles per problem, zero guess FP64:", pp["zero64_cycles"])
    print("cycles per problem, learned guess FP32-DC:", pp["learned_dc_cycles"])
    assert len(pp["zero64_cycles"]) == res["problems"]
