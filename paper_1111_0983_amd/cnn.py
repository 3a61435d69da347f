"""Learned initial guess: ctypes binding of include/ghostmg_cnn.h and the network driver.

The network is five dilated 3x3 convolutions, 4 -> 32 -> 32 -> 32 -> 32 -> 1 channels,
ReLU between layers, dilations 1, 2, 4, 8, 1 (receptive field 33 nodes), evaluated on one
coarse level of the solver hierarchy.  Every arithmetic step (convolutions, gradients,
loss, Adam, features, interpolation to the finest grid) runs in the HIP library; this
module allocates the tensors and sequences the calls.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import ghostmg as gm

_lib = gm.lib
_vp = ctypes.c_void_p
_lib.cnn_cpad.argtypes = [ctypes.c_int]
_lib.cnn_kpad.argtypes = [ctypes.c_int]
_lib.cnn_pack.argtypes = [_vp, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp]
_lib.cnn_conv.argtypes = [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _vp,
                          ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _vp,
                          ctypes.c_int, _vp]
_lib.cnn_wgrad_work.argtypes = [ctypes.c_int] * 5
_lib.cnn_wgrad_work.restype = ctypes.c_int64
_lib.cnn_wgrad.argtypes = [_vp, _vp] + [ctypes.c_int] * 8 + [_vp, _vp, _vp, _vp]
_lib.cnn_wgrad_noalloc.argtypes = [_vp, _vp] + [ctypes.c_int] * 8 + [_vp, _vp, _vp]
_lib.cnn_loss.argtypes = [_vp, _vp, _vp, ctypes.c_int64, _vp, _vp, _vp]
_lib.cnn_adam.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_int64, ctypes.c_float, ctypes.c_float,
                          ctypes.c_float, ctypes.c_float, ctypes.c_int, _vp]
_lib.mg_cnn_features.argtypes = [_vp, ctypes.c_int, _vp, _vp, _vp, _vp]
_lib.mg_cnn_target.argtypes = [_vp, ctypes.c_int, _vp, _vp, _vp, _vp]
_lib.mg_cnn_apply.argtypes = [_vp, ctypes.c_int, _vp, _vp, _vp]

LAYERS = ((4, 32, 1), (32, 32, 2), (32, 32, 4), (32, 32, 8), (32, 1, 1))
# a deeper variant whose receptive field (131 nodes) covers the whole 65 x 65 level: every
# prediction sees the whole domain, its boundary data and its right-hand side
LAYERS_LARGE = ((4, 32, 1), (32, 32, 2), (32, 32, 4), (32, 32, 8), (32, 32, 16), (32, 32, 32),
                (32, 32, 1), (32, 1, 1))


def _p(t):
    return _vp(t.data_ptr()) if t is not None else None


def _check(rc, what):
    if rc != 0:
        raise gm.GhostMGError(rc, what)


def cpad(c: int) -> int:
    return _lib.cnn_cpad(c)


def kpad(cp: int) -> int:
    return _lib.cnn_kpad(cp)


def pack(w, cin, cout, stream=None):
    dev = w.device
    cinp, coutp = cpad(cin), cpad(cout)
    rf = max(16, -(-cout // 16) * 16)
    rb = max(16, -(-cin // 16) * 16)
    wf = torch.zeros(rf * kpad(cinp), dtype=torch.bfloat16, device=dev)
    wb = torch.zeros(rb * kpad(coutp), dtype=torch.bfloat16, device=dev)
    _check(_lib.cnn_pack(_p(w), cin, cout, _p(wf), _p(wb), _vp(stream)), "cnn_pack")
    return wf, wb


def conv(x, B, H, W, cin, wt, bias, cout, dil, relu, relu_of=None, out_f32=False, stream=None):
    coutp = cpad(cout)
    dev = x.device
    if out_f32:
        y = torch.empty(B * H * W, dtype=torch.float32, device=dev)
    else:
        y = torch.empty(B * H * W * coutp, dtype=torch.bfloat16, device=dev)
    _check(_lib.cnn_conv(_p(x), B, H, W, cpad(cin), _p(wt), _p(bias), cout, coutp, dil,
                         int(relu), _p(relu_of), _p(y), int(out_f32), _vp(stream)), "cnn_conv")
    return y


def wgrad(x, dy, B, H, W, cin, cout, dil, stream=None):
    dev = x.device
    work = torch.empty(int(_lib.cnn_wgrad_work(B, H, W, cin, cout)), dtype=torch.float32,
                       device=dev)
    dw = torch.empty(cout * 9 * cin, dtype=torch.float32, device=dev)
    db = torch.empty(cout, dtype=torch.float32, device=dev)
    _check(_lib.cnn_wgrad(_p(x), _p(dy), B, H, W, cin, cpad(cin), cout, cpad(cout), dil,
                          _p(work), _p(dw), _p(db), _vp(stream)), "cnn_wgrad")
    return dw, db


def wgrad_noalloc(x, dy, B, H, W, cin, cout, dil, dw, db, stream=None):
    """cnn_wgrad_noalloc: the weight gradient into the caller's dw, db with no allocation
    (neither by the library nor here)."""
    _check(_lib.cnn_wgrad_noalloc(_p(x), _p(dy), B, H, W, cin, cpad(cin), cout, cpad(cout), dil,
                                  _p(dw), _p(db), _vp(stream)), "cnn_wgrad_noalloc")


def loss(pred, target, mask, with_grad=True, stream=None):
    n = pred.numel()
    out = torch.zeros(2 + 2 * 128, dtype=torch.float32, device=pred.device)
    dy = torch.empty(n * 8, dtype=torch.bfloat16, device=pred.device) if with_grad else None
    _check(_lib.cnn_loss(_p(pred), _p(target), _p(mask), n, _p(out), _p(dy), _vp(stream)),
           "cnn_loss")
    return out, dy


class GuessNet:
    """FP32 master weights [cout][3][3][cin] with Adam state; BF16 packed operands."""

    # the network predicts gain * u / s: u / s is O(1e-2) for these problems
    GAIN = 32.0

    def __init__(self, seed: int = 0, device="cuda:0", layers=LAYERS):
        self.layers = layers
        self.device = torch.device(device)
        self.gain = self.GAIN
        g = torch.Generator().manual_seed(seed)
        self.w, self.b = [], []
        for i, (cin, cout, _) in enumerate(layers):
            # He initialisation; the output layer starts at zero, so the first updates do
            # not have to undo a random O(1) output (which drives hidden units dead)
            std = (2.0 / (9 * cin)) ** 0.5 if i < len(layers) - 1 else 0.0
            self.w.append((torch.randn(cout * 9 * cin, generator=g) * std).to(self.device))
            self.b.append(torch.zeros(cout, device=self.device))
        self.m = [torch.zeros_like(t) for t in self.w + self.b]
        self.v = [torch.zeros_like(t) for t in self.w + self.b]
        self.t = 0
        self.repack()

    def repack(self):
        self.wf, self.wb = [], []
        for w, (cin, cout, _) in zip(self.w, self.layers):
            f, b = pack(w, cin, cout)
            self.wf.append(f)
            self.wb.append(b)

    def forward(self, x, B, H, W):
        acts = [x]
        a = x
        for i, (cin, cout, dil) in enumerate(self.layers):
            last = i == len(self.layers) - 1
            a = conv(a, B, H, W, cin, self.wf[i], self.b[i], cout, dil, relu=not last,
                     out_f32=last)
            acts.append(a)
        self.acts = acts
        return a

    def backward(self, dy, B, H, W):
        """dy: BF16 [B H W][8] gradient of the loss w.r.t. the output (channel 0)."""
        grads = [None] * len(self.layers)
        for i in range(len(self.layers) - 1, -1, -1):
            cin, cout, dil = self.layers[i]
            dw, db = wgrad(self.acts[i], dy, B, H, W, cin, cout, dil)
            grads[i] = (dw, db)
            if i > 0:
                # input gradient: the same convolution kernel on the flipped, transposed
                # weights, times the ReLU derivative of this layer's input
                dy = conv(dy, B, H, W, cout, self.wb[i], None, cin, dil, relu=False,
                          relu_of=self.acts[i])
        return grads

    def adam(self, grads, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.t += 1
        params = self.w + self.b
        gl = [g[0] for g in grads] + [g[1] for g in grads]
        for p, g, m, v in zip(params, gl, self.m, self.v):
            _check(_lib.cnn_adam(_p(p), _p(g), _p(m), _p(v), p.numel(), lr, b1, b2, eps, self.t,
                                 None), "cnn_adam")
        self.repack()

    def state(self) -> dict:
        d = {"gain": np.float64(self.gain)}
        for i, (w, b) in enumerate(zip(self.w, self.b)):
            d[f"w{i}"] = w.detach().cpu().numpy()
            d[f"b{i}"] = b.detach().cpu().numpy()
        return d

    def load(self, d: dict):
        self.gain = float(d["gain"]) if "gain" in d else self.GAIN
        for i in range(len(self.layers)):
            self.w[i].copy_(torch.from_numpy(np.asarray(d[f"w{i}"])))
            self.b[i].copy_(torch.from_numpy(np.asarray(d[f"b{i}"])))
        self.repack()


def features(solver: gm.Solver, level: int, f, g):
    n_l = solver.level(level)["n"]
    B, H = solver.batch, n_l + 1
    x = torch.zeros(B * H * H * 8, dtype=torch.bfloat16, device=f.device)
    scale = torch.zeros(B, dtype=torch.float32, device=f.device)
    _check(_lib.mg_cnn_features(solver._h, level, _p(f), _p(g), _p(x), _p(scale)),
           "mg_cnn_features")
    return x, scale, (B, H, H)


def target(solver: gm.Solver, level: int, u, scale):
    n_l = solver.level(level)["n"]
    npx = solver.batch * (n_l + 1) ** 2
    tgt = torch.empty(npx, dtype=torch.float32, device=u.device)
    mask = torch.empty(npx, dtype=torch.float32, device=u.device)
    _check(_lib.mg_cnn_target(solver._h, level, _p(u), _p(scale), _p(tgt), _p(mask)),
           "mg_cnn_target")
    return tgt, mask


def apply(solver: gm.Solver, level: int, pred, scale, u0):
    _check(_lib.mg_cnn_apply(solver._h, level, _p(pred), _p(scale), _p(u0)), "mg_cnn_apply")


def guess(net: GuessNet, solver: gm.Solver, level: int, f, g, u0):
    """Write the network's initial iterate for (f, g) into u0 (finest grid)."""
    x, scale, (B, H, W) = features(solver, level, f, g)
    pred = net.forward(x, B, H, W)
    apply(solver, level, pred, scale / net.gain, u0)
