"""Reference of the learned-start net (TEST INFRASTRUCTURE ONLY).

The learned initial guess and preconditioner are an addition to the method
(the paper names machine learning only as context): a net of three periodic
3 x 3 x 3 convolutions, 16 channels, ReLU after the first two, BF16 weights and
activations, FP32 accumulation. This module computes one training step of that
net the plain way, in float64 over values rounded to BF16 where the kernels
store BF16, with no tiling, so that the hand-written kernels (forward, data
gradient, weight gradient, loss, Adam) can be checked against it.

Layout: per layer, weights [16 out][27 taps][16 in] with tap n meaning the
offset d = (n // 9 - 1, (n // 3) % 3 - 1, n % 3 - 1), then 16 biases;
out(x) = bias + sum_n W[:, n, :] in(x + d_n) (periodic). Fields are channels
last, [solve][ix][iy][iz][channel].
"""
from __future__ import annotations

import numpy as np

C = 16
TAPS = [(n // 9 - 1, (n // 3) % 3 - 1, n % 3 - 1) for n in range(27)]
LAYER = C * 27 * C + C


def bf16(a: np.ndarray) -> np.ndarray:
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(params: np.ndarray, layer: int):
    p = np.asarray(params[layer * LAYER:(layer + 1) * LAYER], dtype=np.float64)
    return p[:C * 27 * C].reshape(C, 27, C), p[C * 27 * C:]


def shifted(a: np.ndarray, d) -> np.ndarray:
    """a(x + d) for fields [s][x][y][z][c] on the periodic grid."""
    return np.roll(a, shift=(-d[0], -d[1], -d[2]), axis=(1, 2, 3))


def conv(a: np.ndarray, W: np.ndarray, bias) -> np.ndarray:
    out = np.zeros(a.shape[:4] + (W.shape[0],))
    for n, d in enumerate(TAPS):
        out += shifted(a, d) @ W[:, n, :].T
    if bias is not None:
        out += bias
    return out


def conv_data_grad(g: np.ndarray, W: np.ndarray) -> np.ndarray:
    """d/d in of sum <g, conv(in)>: sum_n W[:, n, :]^T g(x - d_n)."""
    out = np.zeros(g.shape[:4] + (W.shape[2],))
    for n, d in enumerate(TAPS):
        out += shifted(g, (-d[0], -d[1], -d[2])) @ W[:, n, :]
    return out


def conv_weight_grad(a: np.ndarray, g: np.ndarray):
    """dW[o, n, i] = sum_{s, x} g[s, x, o] a[s, x + d_n, i]; db = sum g."""
    gf = g.reshape(-1, g.shape[-1])
    dW = np.stack([gf.T @ shifted(a, d).reshape(-1, a.shape[-1]) for d in TAPS], axis=1)
    return dW, gf.sum(axis=0)


def fit_step(params: np.ndarray, inp: np.ndarray, target: np.ndarray, rounding: bool = True):
    """Forward, loss and gradient of one batch.

    inp [s][x][y][z][5], target [s][x][y][z][2]. Loss per solve: relative L2 of
    output channels 0, 1 against the target. Returns (out [s,x,y,z,2], loss [s],
    grad (the three layers' weights and biases, summed over solves, in the
    parameter layout)). rounding=False keeps every value in float64 (for
    finite-difference checks of the gradient)."""
    rnd = bf16 if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    a0 = np.zeros(inp.shape[:4] + (C,))
    a0[..., :inp.shape[-1]] = inp
    a0 = rnd(a0)
    W = [rnd(unpack(params, l)[0]) for l in range(3)]
    b = [unpack(params, l)[1] for l in range(3)]
    a1 = rnd(np.maximum(conv(a0, W[0], b[0]), 0.0))
    a2 = rnd(np.maximum(conv(a1, W[1], b[1]), 0.0))
    out = conv(a2, W[2], b[2])
    diff = out[..., :2] - target
    den = np.sum(target ** 2, axis=(1, 2, 3, 4))
    loss = np.sum(diff ** 2, axis=(1, 2, 3, 4)) / den
    g3 = np.zeros_like(out)
    g3[..., :2] = 2.0 * diff / den[:, None, None, None, None]
    grads = [None, None, None]
    grads[2] = conv_weight_grad(a2, g3)
    g2 = conv_data_grad(rnd(g3), W[2]) * (a2 > 0)
    grads[1] = conv_weight_grad(a1, g2)
    g1 = conv_data_grad(rnd(g2), W[1]) * (a1 > 0)
    grads[0] = conv_weight_grad(a0, g1)
    flat = np.concatenate([np.concatenate([gw.ravel(), gb]) for gw, gb in grads])
    return out[..., :2], loss, flat


def adam_update(w: np.ndarray, g: np.ndarray, lr: float, step: int, scale: float,
                b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8) -> np.ndarray:
    """Weights after one bias-corrected Adam step (Kingma and Ba, arXiv:1412.6980) from
    zero moments at step `step` = 1, with the gradient scaled by `scale`."""
    gs = g * scale
    m = (1 - b1) * gs
    v = (1 - b2) * gs * gs
    c1 = 1 - b1 ** step
    c2 = 1 - b2 ** step
    return w - lr * (m / c1) / (np.sqrt(v / c2) + eps)
