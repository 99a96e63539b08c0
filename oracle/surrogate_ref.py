"""FP64 NumPy reference of the learned surrogate -- TEST INFRASTRUCTURE.

A 3-level 3-D convolutional encoder-decoder (U-Net) on a G^3 grid with
32/64/128 channels, written out plainly so that a reader can check each
operation: 3x3x3 convolutions with zero padding (stride 1), ReLU, 2x2x2
average pooling, nearest-neighbour 2x upsampling, skip connections by channel
concatenation, a 1x1x1 output head, a masked mean-squared-error loss, and
the hand-derived backward pass of every operation.  The backward pass is
pinned by central finite differences in the tests.

Tensors are channels-last: [B, G, G, G, C] (z, y, x, channel), float64.
Weights of a 3x3x3 convolution are [Cout, 3, 3, 3, Cin] (dz, dy, dx, ci).

`forward` and `backward` take an optional storage rounding q (default: none,
i.e. FP64 throughout).  When given, q is applied wherever a tensor is
stored between operations -- every activation after a convolution, pooled
tensor, gradient leaving the head, a convolution's input gradient, and the
upsampling / pooling backward sums -- so the reference can mirror kernels
that keep such tensors in a narrower format while computing in wider
precision.
"""
from __future__ import annotations

import numpy as np

# (name, input channels, output channels); the network's input has 8
# channels (4 used: source raster, k0, perfusion, occupancy mask)
LAYERS = [("e1a", 8, 32), ("e1b", 32, 32), ("e2a", 32, 64), ("e2b", 64, 64),
          ("e3a", 64, 128), ("e3b", 128, 128), ("d2a", 192, 64), ("d2b", 64, 64),
          ("d1a", 96, 32), ("d1b", 32, 32)]
IN_CHANNELS = 8


# -- single operations ------------------------------------------------------
def conv3(x, W, b):
    """y[v, co] = sum_{d, ci} W[co, d, ci] x[v + d - 1, ci] + b[co]."""
    B, G1, G2, G3, _ = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (1, 1), (0, 0)))
    y = np.zeros((B, G1, G2, G3, W.shape[0]))
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                xs = xp[:, dz:dz + G1, dy:dy + G2, dx:dx + G3, :]
                y += xs @ W[:, dz, dy, dx, :].T
    return y + b


def conv3_backward(x, W, dy):
    """Gradients of conv3 with respect to x, W and b."""
    B, G1, G2, G3, _ = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (1, 1), (0, 0)))
    dxp = np.zeros_like(xp)
    dW = np.zeros_like(W)
    for dz in range(3):
        for dy_ in range(3):
            for dx in range(3):
                xs = xp[:, dz:dz + G1, dy_:dy_ + G2, dx:dx + G3, :]
                dW[:, dz, dy_, dx, :] = np.einsum("bzyxo,bzyxi->oi", dy, xs)
                dxp[:, dz:dz + G1, dy_:dy_ + G2, dx:dx + G3, :] += dy @ W[:, dz, dy_, dx, :]
    db = dy.sum(axis=(0, 1, 2, 3))
    return dxp[:, 1:-1, 1:-1, 1:-1, :], dW, db


def relu(x):
    return np.maximum(x, 0.0)


def pool2(x):
    B, G1, G2, G3, C = x.shape
    return x.reshape(B, G1 // 2, 2, G2 // 2, 2, G3 // 2, 2, C).mean(axis=(2, 4, 6))


def pool2_backward(dy):
    return np.repeat(np.repeat(np.repeat(dy, 2, axis=1), 2, axis=2), 2, axis=3) / 8.0


def up2(x):
    return np.repeat(np.repeat(np.repeat(x, 2, axis=1), 2, axis=2), 2, axis=3)


def up2_backward(dy):
    B, G1, G2, G3, C = dy.shape
    return dy.reshape(B, G1 // 2, 2, G2 // 2, 2, G3 // 2, 2, C).sum(axis=(2, 4, 6))


def masked_mse(y, t, m):
    """L = sum m (y - t)^2 / sum m, and dL/dy."""
    s = m.sum()
    r = (y - t) * m
    return float((r * (y - t)).sum() / s), 2.0 * r / s


# -- the network --------------------------------------------------------------
def init_params(rng, scale=1.0):
    """He-style initial weights (the GPU network seeds its own)."""
    P = {}
    for name, ci, co in LAYERS:
        P[name + ".w"] = rng.normal(0.0, scale * np.sqrt(2.0 / (27 * ci)), (co, 3, 3, 3, ci))
        P[name + ".b"] = rng.normal(0.0, 0.01, co)
    P["head.w"] = rng.normal(0.0, np.sqrt(1.0 / 32), 32)
    P["head.b"] = np.array([0.0])
    return P


def _ident(a):
    return a


def forward(P, x, q=None):
    """Returns the output [B, G, G, G] and the cache for backward."""
    q = q or _ident
    c = {"q": q}

    def cv(name, inp):
        pre = conv3(inp, P[name + ".w"], P[name + ".b"])
        c[name + ".in"] = inp
        c[name + ".out"] = q(relu(pre))
        return c[name + ".out"]

    e1 = cv("e1b", cv("e1a", x))
    e2 = cv("e2b", cv("e2a", q(pool2(e1))))
    e3 = cv("e3b", cv("e3a", q(pool2(e2))))
    cat2 = np.concatenate([up2(e3), e2], axis=-1)
    d2 = cv("d2b", cv("d2a", cat2))
    cat1 = np.concatenate([up2(d2), e1], axis=-1)
    d1 = cv("d1b", cv("d1a", cat1))
    c["d1"] = d1
    y = d1 @ P["head.w"] + P["head.b"][0]
    return y, c


def backward(P, c, dy):
    """Gradients of every parameter and of the network input."""
    q = c.get("q", _ident)
    g = {}
    d1 = c["d1"]
    g["head.w"] = np.einsum("bzyxc,bzyx->c", d1, dy)
    g["head.b"] = np.array([dy.sum()])
    dd1 = q(dy[..., None] * P["head.w"])

    def cvb(name, dout):
        dpre = dout * (c[name + ".out"] > 0)
        dx, dW, db = conv3_backward(c[name + ".in"], P[name + ".w"], dpre)
        g[name + ".w"] = dW
        g[name + ".b"] = db
        return q(dx)

    dcat1 = cvb("d1a", cvb("d1b", dd1))
    C1 = P["d1a.w"].shape[-1] - 32
    dd2 = q(up2_backward(dcat1[..., :C1]))
    de1 = dcat1[..., C1:]
    dcat2 = cvb("d2a", cvb("d2b", dd2))
    C2 = P["d2a.w"].shape[-1] - 64
    de3 = q(up2_backward(dcat2[..., :C2]))
    de2 = dcat2[..., C2:]
    dp2 = cvb("e3a", cvb("e3b", de3))
    de2 = q(de2 + pool2_backward(dp2))
    dp1 = cvb("e2a", cvb("e2b", de2))
    de1 = q(de1 + pool2_backward(dp1))
    dx = cvb("e1a", cvb("e1b", de1))
    return g, dx


def loss_and_grads(P, x, t, m, q=None):
    y, c = forward(P, x, q)
    L, dy = masked_mse(y, t, m)
    g, dx = backward(P, c, dy)
    return L, g, dx, y


def adam_step(p, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """Adam (Kingma & Ba 2015): returns new (p, m, v); step counts from 1."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
