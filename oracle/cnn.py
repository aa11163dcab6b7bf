"""Learned shrinkage network in FP64 (an extension beyond the paper: a small
per-scale CNN that predicts a gain in [0, 1] for every detail coefficient;
hard thresholding, Section 5.3, is its fallback and its yardstick).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Architecture, applied to one detail subband plane c of size H x W:
  input  x0[0] = |c| / (sigma ||psi_i||_2),  x0[1] = sigma * 255 / 50
  h1 = relu(conv3x3(x0; W1, b1))     2 -> C channels
  h2 = relu(conv3x3(h1; W2, b2))     C -> C channels
  g  = sigmoid(conv3x3(h2; W3, b3))  C -> 1 channel
  shrunk coefficient = g * c
conv3x3 is a cross-correlation with zero padding ("same" size):
  y[o, p] = b[o] + sum_{i, dy, dx} W[o, i, dy, dx] x[i, p + (dy - 1, dx - 1)].
One weight set per scale j, shared by all cones and shears of that scale.

bf16 emulation rounds, to bfloat16 with round-to-nearest-even, exactly the
operands the device kernels feed to the matrix cores: the weights and the
input of every convolution (x0, h1, h2) in the forward pass, and in the
backward pass the output gradients of every convolution and the weights they
meet.  Biases, accumulations and elementwise activations stay in full
precision.
"""
import numpy as np


def bf16_round(a):
    """Round float64/float32 values to the nearest bfloat16 (ties to even),
    returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _cols(x):
    """im2col for a 3x3 'same' cross-correlation: [Cin*9, H*W]."""
    C, H, W = x.shape
    xp = np.zeros((C, H + 2, W + 2))
    xp[:, 1:-1, 1:-1] = x
    cols = np.empty((C, 9, H, W))
    for dy in range(3):
        for dx in range(3):
            cols[:, dy * 3 + dx] = xp[:, dy:dy + H, dx:dx + W]
    return cols.reshape(C * 9, H * W)


def _col2im(dcols, C, H, W):
    dcols = dcols.reshape(C, 9, H, W)
    dxp = np.zeros((C, H + 2, W + 2))
    for dy in range(3):
        for dx in range(3):
            dxp[:, dy:dy + H, dx:dx + W] += dcols[:, dy * 3 + dx]
    return dxp[:, 1:-1, 1:-1]


def conv3x3(x, w, b):
    Cout = w.shape[0]
    _, H, W = x.shape
    return (w.reshape(Cout, -1) @ _cols(x)).reshape(Cout, H, W) + b[:, None, None]


def conv3x3_backward(x, w, dy):
    """Gradients of y = conv3x3(x, w, b) given dL/dy: (dx, dw, db)."""
    Cout, Cin = w.shape[:2]
    _, H, W = x.shape
    dyf = dy.reshape(Cout, H * W)
    dw = (dyf @ _cols(x).T).reshape(w.shape)
    db = dyf.sum(axis=1)
    dx = _col2im(w.reshape(Cout, -1).T @ dyf, Cin, H, W)
    return dx, dw, db


def init_params(C=32, seed=0):
    """He-style initial weights for one scale (float64)."""
    rng = np.random.default_rng(seed)
    p = {
        "W1": rng.standard_normal((C, 2, 3, 3)) * np.sqrt(2.0 / 18),
        "b1": np.zeros(C),
        "W2": rng.standard_normal((C, C, 3, 3)) * np.sqrt(2.0 / (9 * C)),
        "b2": np.zeros(C),
        "W3": rng.standard_normal((1, C, 3, 3)) * np.sqrt(1.0 / (9 * C)),
        "b3": np.zeros(1),
    }
    return p


def input_planes(c, sigma, l2norm):
    x0 = np.empty((2, *c.shape))
    x0[0] = np.abs(c) / (sigma * l2norm)
    x0[1] = sigma * 255.0 / 50.0
    return x0


def forward(p, c, sigma, l2norm, bf16=False):
    """Gain g for one subband plane and the cache for backward."""
    r = bf16_round if bf16 else (lambda a: a)
    x0 = r(input_planes(c, sigma, l2norm))
    W1, W2, W3 = r(p["W1"]), r(p["W2"]), r(p["W3"])
    a1 = conv3x3(x0, W1, p["b1"])
    h1 = r(np.maximum(a1, 0.0))
    a2 = conv3x3(h1, W2, p["b2"])
    h2 = r(np.maximum(a2, 0.0))
    z = conv3x3(h2, W3, p["b3"])[0]
    g = 1.0 / (1.0 + np.exp(-z))
    cache = dict(x0=x0, a1=a1, h1=h1, a2=a2, h2=h2, g=g, W1=W1, W2=W2, W3=W3, bf16=bf16)
    return g, cache


def backward(cache, dg):
    """Parameter gradients from dL/dg (one plane)."""
    r = bf16_round if cache["bf16"] else (lambda a: a)
    g = cache["g"]
    dz = (dg * g * (1.0 - g))[None]
    dh2, dW3, db3 = conv3x3_backward(cache["h2"], cache["W3"], r(dz))
    da2 = dh2 * (cache["a2"] > 0)
    dh1, dW2, db2 = conv3x3_backward(cache["h1"], cache["W2"], r(da2))
    da1 = dh1 * (cache["a1"] > 0)
    _, dW1, db1 = conv3x3_backward(cache["x0"], cache["W1"], r(da1))
    return {"W1": dW1, "b1": db1, "W2": dW2, "b2": db2, "W3": dW3, "b3": db3}


def adam_step(p, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba) of a parameter dict, in place."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in p:
        m = state.setdefault("m_" + k, np.zeros_like(p[k]))
        v = state.setdefault("v_" + k, np.zeros_like(p[k]))
        m[:] = b1 * m + (1 - b1) * grads[k]
        v[:] = b2 * v + (1 - b2) * grads[k] ** 2
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
    return p
