"""Pins for the FP64 CPU reference of the surrogate network: the convolution against
scipy's correlation routine, pooling/upsampling against definitions, and the whole
backward pass against central finite differences of the forward pass."""
import numpy as np
import pytest
from scipy import signal

from oracle import unet as U


def test_conv3x3_matches_scipy_correlate():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((7, 9, 3))
    W = rng.standard_normal((9, 3, 4))
    b = rng.standard_normal(4)
    y = U.conv3x3(x, W, b)
    for o in range(4):
        ref = b[o] + sum(signal.correlate2d(x[..., c], W[:, c, o].reshape(3, 3), mode="same")
                         for c in range(3))
        np.testing.assert_allclose(y[..., o], ref, atol=1e-12)


def test_pool_and_upsample_definitions():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((4, 6, 2))
    y, arg = U.maxpool(x)
    assert y.shape == (2, 3, 2)
    assert y[1, 2, 1] == max(x[2, 4, 1], x[2, 5, 1], x[3, 4, 1], x[3, 5, 1])
    u = U.upsample(y)
    assert u.shape == x.shape and u[3, 5, 0] == y[1, 2, 0]
    # adjoint identities: <up(a), b> = <a, up^T(b)>
    b = rng.standard_normal(x.shape)
    assert abs(np.sum(U.upsample(y) * b) - np.sum(y * U.upsample_backward(b))) < 1e-12


@pytest.mark.parametrize("levels", [2, 3])
def test_backward_matches_finite_differences(levels):
    rng = np.random.default_rng(2 + levels)
    H, W, C = 8, 8, 2
    p = U.init_params(levels, 4, C, seed=levels)
    for k in p:
        if k.endswith(".b"):
            p[k] = rng.standard_normal(p[k].shape) * 0.1
    x = rng.standard_normal((H, W, C))
    t = rng.uniform(0, 1, (H, W))
    loss, g, dx = U.loss_and_grads(p, x, t, levels)
    mask0, _, _ = U.forward(p, x, levels)
    e0 = np.abs(mask0 - t)          # the second loss term's target is a constant
    h = 1e-6
    checked = 0
    for name in ["enc0a.w", "enc0b.b", f"enc{levels - 1}b.w", "dec0a.w", "dec0b.w", "head.w", "head.b"]:
        flat = p[name].reshape(-1)
        for idx in rng.choice(flat.size, size=min(4, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp, _, _ = U.loss_and_grads(p, x, t, levels, e0)
            flat[idx] = old - h
            lm, _, _ = U.loss_and_grads(p, x, t, levels, e0)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = g[name].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 + 1e-4 * abs(fd), (name, idx, fd, an)
            checked += 1
    # input gradient
    for idx in rng.choice(x.size, size=4, replace=False):
        xf = x.reshape(-1)
        old = xf[idx]
        xf[idx] = old + h
        lp, _, _ = U.loss_and_grads(p, x, t, levels, e0)
        xf[idx] = old - h
        lm, _, _ = U.loss_and_grads(p, x, t, levels, e0)
        xf[idx] = old
        assert abs((lp - lm) / (2 * h) - dx.reshape(-1)[idx]) <= 1e-6 + 1e-4 * abs(dx.reshape(-1)[idx])
    assert checked > 10
