"""Pins of the network's FP64 reference: its hand-written gradients equal central finite
differences of its loss; a dilated convolution equals the direct sum over taps."""
import numpy as np

from oracle import cnn_oracle as co


def _params(rng, layers):
    return [(rng.normal(0, (2.0 / (9 * ci)) ** 0.5, (c, 3, 3, ci)), rng.normal(0, 0.1, c))
            for ci, c, _ in layers]


def test_conv_equals_direct_tap_sum():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 7, 9, 3))
    w = rng.normal(size=(4, 3, 3, 3))
    b = rng.normal(size=4)
    for dil in (1, 2, 3):
        z = co.conv(x, w, b, dil)
        for (bb, y, xx, o) in [(0, 0, 0, 0), (1, 6, 8, 3), (0, 3, 4, 2), (1, 2, 7, 1)]:
            s = b[o]
            for ky in range(3):
                for kx in range(3):
                    yy, xq = y + dil * (ky - 1), xx + dil * (kx - 1)
                    if 0 <= yy < 7 and 0 <= xq < 9:
                        s += w[o, ky, kx] @ x[bb, yy, xq]
            assert abs(z[bb, y, xx, o] - s) < 1e-12


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(1)
    layers = ((3, 5, 1), (5, 4, 2), (4, 1, 1))
    dils = [d for _, _, d in layers]
    params = _params(rng, layers)
    x = rng.normal(size=(2, 6, 5, 3))
    tgt = rng.normal(size=(2, 6, 5))
    mask = (rng.uniform(size=(2, 6, 5)) > 0.3).astype(float)
    loss, grads, _ = co.loss_and_grads(params, x, tgt, mask, dils)
    eps = 1e-6
    for li in range(len(params)):
        w, b = params[li]
        for idx in [(0, 0, 0, 0), (0, 1, 2, 0), (w.shape[0] - 1, 2, 1, w.shape[3] - 1)]:
            wp = w.copy(); wp[idx] += eps
            wm = w.copy(); wm[idx] -= eps
            pp = list(params); pp[li] = (wp, b)
            pm = list(params); pm[li] = (wm, b)
            fd = (co.loss_and_grads(pp, x, tgt, mask, dils)[0] -
                  co.loss_and_grads(pm, x, tgt, mask, dils)[0]) / (2 * eps)
            assert abs(fd - grads[li][0][idx]) < 1e-6 * max(1.0, abs(fd)), (li, idx)
        bp = b.copy(); bp[0] += eps
        bm = b.copy(); bm[0] -= eps
        pp = list(params); pp[li] = (w, bp)
        pm = list(params); pm[li] = (w, bm)
        fd = (co.loss_and_grads(pp, x, tgt, mask, dils)[0] -
              co.loss_and_grads(pm, x, tgt, mask, dils)[0]) / (2 * eps)
        assert abs(fd - grads[li][1][0]) < 1e-6 * max(1.0, abs(fd))


def test_bf16_rounding_is_round_to_nearest_even():
    one = 1.0
    ulp = 2.0 ** -7  # BF16 has 8 significand bits
    vals = np.array([one, one + ulp / 4, one + ulp / 2, one + 3 * ulp / 2, one + 0.75 * ulp,
                     -3.0 - 2 * ulp, 0.0])
    got = co.bf16(vals)
    # ties go to the even significand: 1 + ulp/2 -> 1, 1 + 3 ulp / 2 -> 1 + 2 ulp
    want = np.array([one, one, one, one + 2 * ulp, one + ulp, -3.0 - 2 * ulp, 0.0])
    assert np.array_equal(got, want), (got, want)
    assert np.array_equal(co.bf16(got), got)


def test_adam_step_closed_form():
    """First step: m = (1 - b1) g, v = (1 - b2) g^2, so the bias-corrected step is
    lr g / (|g| + eps): -lr sign(g) up to eps."""
    g = np.array([0.5, -2.0, 1e-3])
    w, m, v = co.adam(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    assert np.allclose(w, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    w2, m2, v2 = co.adam(w, g, m, v, 2, lr=0.01)
    mh = (0.9 * m + 0.1 * g) / (1 - 0.81)
    vh = (0.999 * v + 0.001 * g * g) / (1 - 0.999 ** 2)
    assert np.allclose(w2, w - 0.01 * mh / (np.sqrt(vh) + 1e-8), rtol=1e-12, atol=0)
