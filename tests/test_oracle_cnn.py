"""Pins of the oracle's learned-shrinkage network (no GPU): the convolution
against its defining sum, gradients against central finite differences, the
bfloat16 rounding against hand-worked bit patterns, Adam against its formula
on a scalar."""
import numpy as np
import pytest

from oracle import cnn


def _conv_direct(x, w, b):
    Cout, Cin = w.shape[:2]
    _, H, W = x.shape
    y = np.zeros((Cout, H, W))
    for o in range(Cout):
        for yy in range(H):
            for xx in range(W):
                s = b[o]
                for i in range(Cin):
                    for dy in range(3):
                        for dx in range(3):
                            r, c = yy + dy - 1, xx + dx - 1
                            if 0 <= r < H and 0 <= c < W:
                                s += w[o, i, dy, dx] * x[i, r, c]
                y[o, yy, xx] = s
    return y


def test_conv_matches_definition():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((3, 5, 7))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    assert np.max(np.abs(cnn.conv3x3(x, w, b) - _conv_direct(x, w, b))) < 1e-12


def _loss(p, c, sigma, l2, tgt):
    g, _ = cnn.forward(p, c, sigma, l2)
    return 0.5 * np.sum((g * c - tgt) ** 2)


def test_gradients_finite_difference():
    rng = np.random.default_rng(1)
    p = cnn.init_params(C=4, seed=2)
    for k in ("b1", "b2", "b3"):
        p[k] = rng.standard_normal(p[k].shape) * 0.1
    c = rng.standard_normal((6, 5))
    tgt = rng.standard_normal((6, 5))
    sigma, l2 = 0.3, 0.7
    g, cache = cnn.forward(p, c, sigma, l2)
    grads = cnn.backward(cache, (g * c - tgt) * c)
    eps = 1e-6
    for k in p:
        flat = p[k].ravel()
        idx = rng.choice(flat.size, size=min(6, flat.size), replace=False)
        for i in idx:
            old = flat[i]
            flat[i] = old + eps
            lp = _loss(p, c, sigma, l2, tgt)
            flat[i] = old - eps
            lm = _loss(p, c, sigma, l2, tgt)
            flat[i] = old
            fd = (lp - lm) / (2 * eps)
            an = grads[k].ravel()[i]
            assert abs(fd - an) <= 1e-6 * max(1e-3, abs(fd)), (k, i, fd, an)


def test_bf16_round():
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: even mantissa (1) wins
    assert cnn.bf16_round(1.0 + 2 ** -8) == 1.0
    # 1 + 3 * 2^-8 is a tie between 1 + 2^-7 and 1 + 2^-6: rounds up to the even one
    assert cnn.bf16_round(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6
    assert cnn.bf16_round(1.0 + 2 ** -7) == 1.0 + 2 ** -7
    assert cnn.bf16_round(-3.0) == -3.0
    v = np.random.default_rng(3).standard_normal(1000)
    r = cnn.bf16_round(v)
    assert np.max(np.abs(r - v) / np.abs(v)) <= 2 ** -8


def test_adam_scalar():
    p = {"w": np.array([1.0])}
    st = {}
    cnn.adam_step(p, {"w": np.array([0.5])}, st, lr=0.1)
    # first step: m_hat = g, v_hat = g^2, update = lr * g / (|g| + eps)
    assert abs(p["w"][0] - (1.0 - 0.1 * 0.5 / (0.5 + 1e-8))) < 1e-15


def test_param_count():
    p = cnn.init_params(C=32)
    assert sum(v.size for v in p.values()) == 10145


def test_gain_range_and_shape():
    p = cnn.init_params(C=8, seed=5)
    c = np.random.default_rng(6).standard_normal((9, 11))
    g, _ = cnn.forward(p, c, 0.1, 0.5, bf16=True)
    assert g.shape == c.shape and np.all(g > 0) and np.all(g < 1)


def test_adam_three_steps_hand_values():
    # Kingma and Ba's update with beta1 = 9/10, beta2 = 999/1000, lr = 1/10 and
    # gradients 1/2, -1/4, 1/8.  The moments, worked out by hand in exact
    # fractions, are
    #   m1 = 1/20,   v1 = 1/4000
    #   m2 = 9/10 * 1/20 - 1/10 * 1/4   = 1/50
    #   v2 = 999/1000 * 1/4000 + 1/1000 * 1/16 = 1249/4000000
    #   m3 = 9/10 * 1/50 + 1/10 * 1/8   = 61/2000
    #   v3 = 999/1000 * 1249/4000000 + 1/1000 * 1/64 = 1310251/4000000000
    # and the bias-corrected step t is lr * (m_t / (1 - beta1^t)) /
    # (sqrt(v_t / (1 - beta2^t)) + eps).  From t = 2 on the two betas enter
    # differently, so swapping them, using g instead of g^2 in v, or dropping
    # the bias correction each changes these values.
    p = {"w": np.array([1.0])}
    st = {}
    grads = [0.5, -0.25, 0.125]
    m_hand = [1 / 20, 1 / 50, 61 / 2000]
    v_hand = [1 / 4000, 1249 / 4000000, 1310251 / 4000000000]
    w = 1.0
    for t, g in enumerate(grads, start=1):
        cnn.adam_step(p, {"w": np.array([g])}, st, lr=0.1)
        assert abs(st["m_w"][0] - m_hand[t - 1]) < 1e-14 * m_hand[t - 1]
        assert abs(st["v_w"][0] - v_hand[t - 1]) < 1e-14 * v_hand[t - 1]
        mh = m_hand[t - 1] / (1 - 0.9 ** t)
        vh = v_hand[t - 1] / (1 - 0.999 ** t)
        w -= 0.1 * mh / (np.sqrt(vh) + 1e-8)
        assert abs(p["w"][0] - w) < 1e-14, (t, p["w"][0], w)
    # the values after steps 2 and 3 (bias corrections 2/19, 1249/7996 at t = 2)
    assert abs((1.0 - 0.1 * 0.5 / (0.5 + 1e-8)) - 0.1 * (2 / 19) / (np.sqrt(1249 / 7996) + 1e-8)
               - 0.8733662987078462) < 1e-14
    assert abs(p["w"][0] - 0.839323384916654) < 1e-13
