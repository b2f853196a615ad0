"""FP64 CPU reference of the NCC-surrogate network (forward and backward).

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite may import it.  It
shares no code with the HIP kernels; its own correctness is pinned in
tests/test_unet_reference.py against scipy's correlation routine (forward) and
central finite differences of its own forward pass (backward).

Network (a U-Net): activations are NHWC arrays [H][W][C].
  encoder level l (l = 0..levels-1): conv3x3 -> ReLU -> conv3x3 -> ReLU   (skip_l)
                                     maxpool 2x2 before the next level
  decoder level l (l = levels-2..0): upsample(nearest, 2x) of the level below,
                                     concat [upsampled, skip_l] on channels,
                                     conv3x3 -> ReLU -> conv3x3 -> ReLU
  head: 1x1 conv to 2 channels: mask = sigmoid(z0), predicted error = sigmoid(z1)
Conventions: conv3x3 is a cross-correlation with zero padding,
  y[h, w, o] = b[o] + sum_{dh, dw in -1..1} sum_c x[h + dh, w + dw, c] * W[3 (dh + 1) + (dw + 1), c, o];
maxpool passes the gradient to the first maximum in the order (0,0), (0,1), (1,0), (1,1);
loss = sum_p w_p BCE(mask, t) + sum_p w_p BCE(err, stop(|mask - t|)) with w_p = 1/P by default.
"""
from __future__ import annotations

from typing import Dict, List

import numpy as np


def conv3x3(x: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    H, Wd, C = x.shape
    xp = np.zeros((H + 2, Wd + 2, C))
    xp[1:-1, 1:-1] = x
    y = np.zeros((H, Wd, W.shape[2])) + b
    for t in range(9):
        dh, dw = t // 3 - 1, t % 3 - 1
        y += xp[1 + dh:1 + dh + H, 1 + dw:1 + dw + Wd] @ W[t]
    return y


def conv3x3_backward(x: np.ndarray, W: np.ndarray, dy: np.ndarray):
    """Gradients of conv3x3 with respect to x, W and b."""
    H, Wd, C = x.shape
    xp = np.zeros((H + 2, Wd + 2, C))
    xp[1:-1, 1:-1] = x
    dxp = np.zeros_like(xp)
    dW = np.zeros_like(W)
    for t in range(9):
        dh, dw = t // 3 - 1, t % 3 - 1
        win = xp[1 + dh:1 + dh + H, 1 + dw:1 + dw + Wd]
        dW[t] = np.einsum("hwc,hwo->co", win, dy)
        dxp[1 + dh:1 + dh + H, 1 + dw:1 + dw + Wd] += dy @ W[t].T
    return dxp[1:-1, 1:-1], dW, dy.sum(axis=(0, 1))


def maxpool(x: np.ndarray):
    H, Wd, C = x.shape
    blocks = [x[0::2, 0::2], x[0::2, 1::2], x[1::2, 0::2], x[1::2, 1::2]]
    stack = np.stack(blocks)                      # [4][H/2][W/2][C]
    arg = np.argmax(stack, axis=0)                # first maximum in scan order
    return stack.max(axis=0), arg


def maxpool_backward(arg: np.ndarray, dy: np.ndarray, shape) -> np.ndarray:
    dx = np.zeros(shape)
    offs = [(0, 0), (0, 1), (1, 0), (1, 1)]
    for k, (a, c) in enumerate(offs):
        dx[a::2, c::2] += np.where(arg == k, dy, 0.0)
    return dx


def upsample(x: np.ndarray) -> np.ndarray:
    return np.repeat(np.repeat(x, 2, axis=0), 2, axis=1)


def upsample_backward(dy: np.ndarray) -> np.ndarray:
    return dy[0::2, 0::2] + dy[0::2, 1::2] + dy[1::2, 0::2] + dy[1::2, 1::2]


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def init_params(levels: int, base: int, c_in: int, seed: int = 0) -> Dict[str, np.ndarray]:
    """He-normal weights [9][C_in][C_out], zero biases; head weights [C][2]."""
    rng = np.random.default_rng(seed)
    p = {}

    def conv(name, ci, co):
        p[name + ".w"] = rng.standard_normal((9, ci, co)) * np.sqrt(2.0 / (9 * ci))
        p[name + ".b"] = np.zeros(co)

    ch = [base * 2 ** l for l in range(levels)]
    prev = c_in
    for l in range(levels):
        conv(f"enc{l}a", prev, ch[l])
        conv(f"enc{l}b", ch[l], ch[l])
        prev = ch[l]
    for l in range(levels - 2, -1, -1):
        conv(f"dec{l}a", ch[l + 1] + ch[l], ch[l])
        conv(f"dec{l}b", ch[l], ch[l])
    p["head.w"] = rng.standard_normal((ch[0], 2)) * np.sqrt(1.0 / ch[0])
    p["head.b"] = np.zeros(2)
    return p


def forward(p: Dict[str, np.ndarray], x: np.ndarray, levels: int):
    """Returns (mask, err, cache)."""
    cache = {"x": x}
    h = x
    skips: List[np.ndarray] = []
    for l in range(levels):
        if l > 0:
            h, arg = maxpool(h)
            cache[f"pool{l}"] = (arg, skips[-1].shape)
        cache[f"enc{l}a.in"] = h
        h = np.maximum(conv3x3(h, p[f"enc{l}a.w"], p[f"enc{l}a.b"]), 0.0)
        cache[f"enc{l}a.out"] = h
        cache[f"enc{l}b.in"] = h
        h = np.maximum(conv3x3(h, p[f"enc{l}b.w"], p[f"enc{l}b.b"]), 0.0)
        cache[f"enc{l}b.out"] = h
        skips.append(h)
    for l in range(levels - 2, -1, -1):
        u = upsample(h)
        cat = np.concatenate([u, skips[l]], axis=2)
        cache[f"dec{l}a.in"] = cat
        h = np.maximum(conv3x3(cat, p[f"dec{l}a.w"], p[f"dec{l}a.b"]), 0.0)
        cache[f"dec{l}a.out"] = h
        cache[f"dec{l}b.in"] = h
        h = np.maximum(conv3x3(h, p[f"dec{l}b.w"], p[f"dec{l}b.b"]), 0.0)
        cache[f"dec{l}b.out"] = h
    cache["feat"] = h
    z = h @ p["head.w"] + p["head.b"]
    cache["z"] = z
    return sigmoid(z[..., 0]), sigmoid(z[..., 1]), cache


def loss_and_grads(p: Dict[str, np.ndarray], x: np.ndarray, t: np.ndarray, levels: int, e_stop=None, wts=None):
    """Loss sum_p w_p BCE(mask, t) + sum_p w_p BCE(err, e) (w = 1/P unless given) and
    gradients, BCE(s, y) = -y log s - (1 - y) log(1 - s) evaluated from the logits; the
    error target e = |mask - t| is a constant of the second term (pass e_stop to hold it
    at given values, e.g. when differencing the loss)."""
    mask, err, cache = forward(p, x, levels)
    P = t.size
    w = np.full(t.shape, 1.0 / P) if wts is None else wts
    e = np.abs(mask - t) if e_stop is None else e_stop
    z0, z1 = cache["z"][..., 0], cache["z"][..., 1]
    sp = lambda v: np.logaddexp(0.0, v)           # softplus
    loss = np.sum(w * (t * sp(-z0) + (1 - t) * sp(z0))) + np.sum(w * (e * sp(-z1) + (1 - e) * sp(z1)))
    dz = np.zeros(cache["z"].shape)
    dz[..., 0] = (mask - t) * w
    dz[..., 1] = (err - e) * w
    g = {"head.w": np.einsum("hwc,hwo->co", cache["feat"], dz), "head.b": dz.sum(axis=(0, 1))}
    ch = [p[f"enc{l}b.w"].shape[2] for l in range(levels)]
    dskip = [None] * levels

    def conv_back(name, dh):
        dh = dh * (cache[name + ".out"] > 0)
        dx, dW, db = conv3x3_backward(cache[name + ".in"], p[name + ".w"], dh)
        g[name + ".w"], g[name + ".b"] = dW, db
        return dx

    # decoder from the output level down, mirroring the forward order in reverse
    d = dz @ p["head.w"].T
    for l in range(0, levels - 1):
        d = conv_back(f"dec{l}b", d)
        d = conv_back(f"dec{l}a", d)
        du, ds = d[..., :ch[l + 1]], d[..., ch[l + 1]:]
        dskip[l] = ds
        d = upsample_backward(du)
    # d is now the gradient at the deepest encoder output
    for l in range(levels - 1, -1, -1):
        if dskip[l] is not None and l < levels - 1:
            d = d + dskip[l]
        d = conv_back(f"enc{l}b", d)
        d = conv_back(f"enc{l}a", d)
        if l > 0:
            arg, shape = cache[f"pool{l}"]
            d = maxpool_backward(arg, d, shape)
    return loss, g, d
