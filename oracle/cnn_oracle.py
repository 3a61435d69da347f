"""FP64 numpy reference of the learned-guess network (TEST INFRASTRUCTURE ONLY).

Dilated 3x3 convolutions with zero padding on NHWC tensors, ReLU, masked mean squared
error, and their gradients written out by the chain rule; one Adam step.  The gradients are
pinned by finite differences in the CPU tests; the GPU kernels are compared with these
functions.  Weights are [cout][3][3][cin]; tap (ky, kx) reads the input at
(y + dil (ky - 1), x + dil (kx - 1)).

With `bf16=True` the values that a BF16 network stores in BF16 are rounded to BF16 (round
to nearest, ties to even) at those points: the weights of every convolution, each hidden
layer's output after its ReLU, the loss gradient and each data gradient after its ReLU
mask; all arithmetic stays FP64.  The network's own output and every gradient of the
weights stay unrounded.
"""
from __future__ import annotations

import numpy as np


def conv(x, w, b, dil):
    B, H, W, _ = x.shape
    cout = w.shape[0]
    xp = np.pad(x, ((0, 0), (dil, dil), (dil, dil), (0, 0)))
    z = np.zeros((B, H, W, cout))
    for ky in range(3):
        for kx in range(3):
            sl = xp[:, ky * dil:ky * dil + H, kx * dil:kx * dil + W, :]
            z += sl @ w[:, ky, kx, :].T
    if b is not None:
        z += b
    return z


def conv_dgrad(dz, w, dil):
    B, H, W, _ = dz.shape
    cin = w.shape[3]
    dxp = np.zeros((B, H + 2 * dil, W + 2 * dil, cin))
    for ky in range(3):
        for kx in range(3):
            dxp[:, ky * dil:ky * dil + H, kx * dil:kx * dil + W, :] += dz @ w[:, ky, kx, :]
    return dxp[:, dil:dil + H, dil:dil + W, :]


def conv_wgrad(x, dz, dil):
    B, H, W, cin = x.shape
    cout = dz.shape[3]
    xp = np.pad(x, ((0, 0), (dil, dil), (dil, dil), (0, 0)))
    dw = np.zeros((cout, 3, 3, cin))
    for ky in range(3):
        for kx in range(3):
            sl = xp[:, ky * dil:ky * dil + H, kx * dil:kx * dil + W, :]
            dw[:, ky, kx, :] = np.einsum("bhwo,bhwi->oi", dz, sl)
    db = dz.sum(axis=(0, 1, 2))
    return dw, db


def bf16(a):
    """Round to the nearest BF16 value (ties to even) and return FP64."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def adam(w, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One bias-corrected Adam step (t >= 1); returns the new (w, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def forward(params, x, dils, bf16_points=False):
    """params: list of (w, b); ReLU after every layer but the last.  Returns the list of
    layer inputs and the output [B, H, W] (channel 0 of the last layer)."""
    q = bf16 if bf16_points else (lambda a: a)
    acts = [x]
    a = x
    for i, ((w, b), d) in enumerate(zip(params, dils)):
        z = conv(a, q(w), b, d)
        a = q(np.maximum(z, 0.0)) if i < len(params) - 1 else z
        acts.append(a)
    return acts, a[..., 0]


def loss_and_grads(params, x, target, mask, dils, bf16_points=False):
    q = bf16 if bf16_points else (lambda a: a)
    acts, pred = forward(params, x, dils, bf16_points)
    cnt = mask.sum()
    diff = pred - target
    loss = (mask * diff ** 2).sum() / cnt
    dz = np.zeros_like(acts[-1])
    dz[..., 0] = q(2.0 * mask * diff / cnt)
    grads = [None] * len(params)
    for i in range(len(params) - 1, -1, -1):
        w, _ = params[i]
        dw, db = conv_wgrad(acts[i], dz, dils[i])
        grads[i] = (dw, db)
        if i > 0:
            da = conv_dgrad(dz, q(w), dils[i])
            dz = q(da * (acts[i] > 0.0))
    return loss, grads, pred
