"""GPU parity of the learned-guess kernels (BF16 MFMA, FP32 accumulation) with the FP64
numpy reference on the same BF16-rounded inputs."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import cnn_oracle as co  # noqa: E402

DEV = "cuda:0"


def _bf(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(torch.bfloat16)


def _to_nhwc_padded(x, cp):
    B, H, W, C = x.shape
    out = np.zeros((B, H, W, cp), np.float32)
    out[..., :C] = x
    return out


def _rounded(a):
    return _bf(a).float().numpy().astype(np.float64)


@pytest.mark.parametrize("cin,cout,dil,f32", [(4, 32, 1, False), (32, 32, 4, False),
                                              (32, 1, 1, True), (32, 32, 8, False)])
def test_conv_forward_matches_reference(cin, cout, dil, f32):
    from paper_1111_0983_amd import cnn
    rng = np.random.default_rng(cin + cout + dil)
    B, H, W = 2, 33, 29
    x = _rounded(rng.normal(size=(B, H, W, cin)))
    w = rng.normal(0, (2.0 / (9 * cin)) ** 0.5, (cout, 3, 3, cin))
    b = rng.normal(0, 0.1, cout)
    wr = _rounded(w)
    xd = _bf(_to_nhwc_padded(x, cnn.cpad(cin))).to(DEV).reshape(-1)
    wt, _ = cnn.pack(torch.from_numpy(w.astype(np.float32)).to(DEV).reshape(-1), cin, cout)
    y = cnn.conv(xd, B, H, W, cin, wt, torch.from_numpy(b.astype(np.float32)).to(DEV), cout, dil,
                 relu=not f32, out_f32=f32)
    ref = co.conv(x, wr, b.astype(np.float32).astype(np.float64), dil)
    if not f32:
        ref = np.maximum(ref, 0)
        got = y.float().cpu().numpy().reshape(B, H, W, cnn.cpad(cout))[..., :cout]
        assert np.abs(got - ref).max() <= 1e-2 * np.abs(ref).max()
        assert np.all(y.float().cpu().numpy().reshape(B, H, W, -1)[..., cout:] == 0)
    else:
        got = y.cpu().numpy().reshape(B, H, W)
        assert np.abs(got - ref[..., 0]).max() <= 1e-4 * np.abs(ref).max()


def test_network_loss_and_gradients_match_reference():
    from paper_1111_0983_amd import cnn
    rng = np.random.default_rng(3)
    B, H, W = 2, 21, 23
    net = cnn.GuessNet(seed=4, device=DEV)
    # the output layer starts at zero (which zeroes every upstream gradient): give it random
    # weights so that every layer's gradient is exercised
    cin, cout, _ = net.layers[-1]
    net.w[-1].copy_(torch.from_numpy(rng.normal(0.0, (2.0 / (9 * cin)) ** 0.5,
                                                size=cout * 9 * cin).astype(np.float32)))
    net.repack()
    x = _rounded(rng.normal(size=(B, H, W, 4)))
    tgt = rng.normal(size=(B, H, W))
    mask = (rng.uniform(size=(B, H, W)) > 0.2).astype(np.float64)
    xd = _bf(_to_nhwc_padded(x, 8)).to(DEV).reshape(-1)
    pred = net.forward(xd, B, H, W)
    out, dy = cnn.loss(pred, torch.from_numpy(tgt.astype(np.float32)).to(DEV).reshape(-1),
                       torch.from_numpy(mask.astype(np.float32)).to(DEV).reshape(-1))
    grads = net.backward(dy, B, H, W)
    params = []
    for (cin, cout, _), w, b in zip(net.layers, net.w, net.b):
        params.append((_rounded(w.cpu().numpy().reshape(cout, 3, 3, cin)),
                       b.cpu().numpy().astype(np.float64)))
    dils = [d for _, _, d in net.layers]
    loss, rgrads, rpred = co.loss_and_grads(params, x, tgt, mask, dils)
    gp = pred.cpu().numpy().reshape(B, H, W)
    assert np.abs(gp - rpred).max() <= 3e-2 * np.abs(rpred).max()
    assert abs(out[0].item() - loss) <= 3e-2 * loss
    for i, ((dw, db), (rdw, rdb)) in enumerate(zip(grads, rgrads)):
        cin, cout, _ = net.layers[i]
        gw = dw.cpu().numpy().reshape(cout, 3, 3, cin)
        rel = np.linalg.norm(gw - rdw) / np.linalg.norm(rdw)
        relb = np.linalg.norm(db.cpu().numpy() - rdb) / max(np.linalg.norm(rdb), 1e-30)
        assert rel < 5e-2 and relb < 5e-2, (i, rel, relb)


def test_training_reduces_loss():
    from paper_1111_0983_amd import cnn
    rng = np.random.default_rng(5)
    B, H, W = 4, 17, 17
    net = cnn.GuessNet(seed=1, device=DEV)
    x = _bf(_to_nhwc_padded(rng.normal(size=(B, H, W, 4)), 8)).to(DEV).reshape(-1)
    # a smooth target the network can fit: a blurred copy of channel 1
    tgt = torch.from_numpy(rng.normal(size=(B, H, W)).astype(np.float32)).to(DEV).reshape(-1)
    mask = torch.ones_like(tgt)
    losses = []
    for _ in range(60):
        pred = net.forward(x, B, H, W)
        out, dy = cnn.loss(pred, tgt, mask)
        losses.append(out[0].item())
        net.adam(net.backward(dy, B, H, W), lr=3e-3)
    assert losses[-1] < 0.5 * losses[0], losses[::10]
