"""Pins of the FP64 surrogate reference: definitions, library routines,
adjointness and central finite differences."""
import numpy as np
import pytest
from scipy import signal

from oracle import surrogate_ref as S


def test_conv3_matches_definition_and_scipy():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 4, 5, 3, 3))
    W = rng.normal(size=(4, 3, 3, 3, 3))
    b = rng.normal(size=4)
    y = S.conv3(x, W, b)
    # brute force from the definition on a few outputs
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (1, 1), (0, 0)))
    for (bb, z, yy, xx, co) in [(0, 0, 0, 0, 0), (1, 3, 4, 2, 3), (0, 2, 1, 1, 2)]:
        s = b[co]
        for dz in range(3):
            for dy in range(3):
                for dx in range(3):
                    for ci in range(3):
                        s += W[co, dz, dy, dx, ci] * xp[bb, z + dz, yy + dy, xx + dx, ci]
        assert abs(y[bb, z, yy, xx, co] - s) < 1e-12
    # cross-correlation per (co, ci) summed over ci, via scipy
    for bb in range(2):
        for co in range(4):
            ref = sum(signal.correlate(x[bb, ..., ci], W[co, ..., ci], mode="same",
                                       method="direct") for ci in range(3)) + b[co]
            assert np.allclose(y[bb, ..., co], ref, atol=1e-12)


def test_pool_and_upsample_adjoint():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, 4, 4, 6, 3))
    y = rng.normal(size=(2, 2, 2, 3, 3))
    assert abs((S.pool2(x) * y).sum() - (x * S.pool2_backward(y)).sum()) < 1e-12
    u = rng.normal(size=(2, 2, 2, 3, 3))
    w = rng.normal(size=(2, 4, 4, 6, 3))
    assert abs((S.up2(u) * w).sum() - (u * S.up2_backward(w)).sum()) < 1e-12
    assert np.allclose(S.pool2(S.up2(u)), u)


def test_conv3_backward_adjoint():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(1, 3, 4, 5, 2))
    W = rng.normal(size=(3, 3, 3, 3, 2))
    dy = rng.normal(size=(1, 3, 4, 5, 3))
    dx, dW, db = S.conv3_backward(x, W, dy)
    # <conv(x) - b, dy> is bilinear: equals <x, dx> and <W, dW>
    lin = (S.conv3(x, W, np.zeros(3)) * dy).sum()
    assert abs(lin - (x * dx).sum()) < 1e-10
    assert abs(lin - (W * dW).sum()) < 1e-10
    assert np.allclose(db, dy.sum(axis=(0, 1, 2, 3)))


@pytest.mark.parametrize("seed", [3, 4])
def test_network_gradients_finite_differences(seed):
    rng = np.random.default_rng(seed)
    G = 4
    P = S.init_params(rng)
    x = rng.normal(size=(1, G, G, G, S.IN_CHANNELS))
    t = rng.normal(size=(1, G, G, G))
    m = (rng.random((1, G, G, G)) < 0.8).astype(float)
    L, g, dx, _ = S.loss_and_grads(P, x, t, m)
    h = 1e-6
    checked = 0
    for name in sorted(P):
        flat = P[name].reshape(-1)
        for idx in rng.choice(flat.size, size=min(3, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            Lp = S.loss_and_grads(P, x, t, m)[0]
            flat[idx] = old - h
            Lm = S.loss_and_grads(P, x, t, m)[0]
            flat[idx] = old
            fd = (Lp - Lm) / (2 * h)
            an = g[name].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)) + 1e-9, (name, idx, fd, an)
            checked += 1
    xf = x.reshape(-1)
    for idx in rng.choice(xf.size, size=6, replace=False):
        old = xf[idx]
        xf[idx] = old + h
        Lp = S.loss_and_grads(P, x, t, m)[0]
        xf[idx] = old - h
        Lm = S.loss_and_grads(P, x, t, m)[0]
        xf[idx] = old
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - dx.reshape(-1)[idx]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9
    assert checked > 50


def test_adam_first_steps():
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -0.1, 0.0])
    m = np.zeros(3)
    v = np.zeros(3)
    p1, m1, v1 = S.adam_step(p, g, m, v, 1, 1e-2)
    # bias-corrected first step moves by lr * g / (|g| + eps)
    assert np.allclose(p1, p - 1e-2 * g / (np.abs(g) + 1e-8))
    p2, _, _ = S.adam_step(p1, g, m1, v1, 2, 1e-2)
    assert np.allclose(p2, p - 2e-2 * g / (np.abs(g) + 1e-8), atol=1e-12)
