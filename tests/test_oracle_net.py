"""Pins of the learned net's reference (oracle/net.py), CPU only.

The reference's convolution is checked against the definition written out
point by point, its gradient against central finite differences of its own
loss (float64, no BF16 rounding), its BF16 rounding against the format's bit
layout, and its Adam step against the first-step closed form lr * sign(g)."""
import numpy as np

from oracle import net


def _params(rng, scale=0.3):
    p = rng.standard_normal(3 * net.LAYER) * scale
    return p


def test_conv_equals_pointwise_definition():
    rng = np.random.default_rng(1)
    Nc = 3
    a = rng.standard_normal((1, Nc, Nc, Nc, net.C))
    W = rng.standard_normal((net.C, 27, net.C))
    bias = rng.standard_normal(net.C)
    got = net.conv(a, W, bias)
    for x, y, z in [(0, 0, 0), (2, 1, 0), (1, 2, 2)]:
        want = bias.copy()
        for n in range(27):
            dx, dy, dz = n // 9 - 1, (n // 3) % 3 - 1, n % 3 - 1
            want += W[:, n, :] @ a[0, (x + dx) % Nc, (y + dy) % Nc, (z + dz) % Nc]
        assert np.allclose(got[0, x, y, z], want, rtol=1e-13, atol=1e-13)


def test_bf16_rounding_bits():
    v = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -9, -3.140625, 1e-3])
    r = net.bf16(v)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7 (even mantissa wins: 1); 1 + 3 * 2^-8 rounds up to
    # 1 + 2^-6 (the even neighbour); -3.140625 = -(1 + 36/64) * 2 is exact in 8 bits
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0 + 2.0 ** -6 and r[3] == 1.0 and r[4] == -3.140625
    assert abs(r[5] - 1e-3) <= 2.0 ** -9 * 1e-3


def test_gradient_equals_finite_differences():
    rng = np.random.default_rng(2)
    Nc = 4
    p = _params(rng)
    inp = rng.standard_normal((2, Nc, Nc, Nc, 5))
    tgt = rng.standard_normal((2, Nc, Nc, Nc, 2))
    _, _, g = net.fit_step(p, inp, tgt, rounding=False)
    h = 1e-6
    for k in list(rng.choice(3 * net.LAYER, 24, replace=False)) + [net.LAYER - 1, 3 * net.LAYER - 1]:
        e = np.zeros_like(p)
        e[k] = h
        lp = net.fit_step(p + e, inp, tgt, rounding=False)[1].sum()
        lm = net.fit_step(p - e, inp, tgt, rounding=False)[1].sum()
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])), (k, fd, g[k])


def test_adam_first_step_is_signed_learning_rate():
    g = np.array([3.0, -0.5, 1e-2, -7e3])
    w = np.zeros(4)
    w1 = net.adam_update(w, g, lr=1e-3, step=1, scale=1.0)
    assert np.allclose(w1, -1e-3 * np.sign(g), rtol=1e-6, atol=0)
