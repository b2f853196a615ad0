"""Thin ctypes binding of the surrogate-network kernels (include/pam_nn.h).

Argument marshalling only: torch tensors supply device memory and streams; every
operation runs in the HIP library.
"""
from __future__ import annotations

import ctypes as C

from . import pam

_NN = None


def lib():
    global _NN
    if _NN is None:
        L = pam._lib()
        vp, i32, i64, f32 = C.c_void_p, C.c_int32, C.c_int64, C.c_float
        sig = {
            "pam_nn_conv3x3": [vp, i32, i32, i32, i32, i32, vp, vp, vp, i32, i32, i32, i32, i32, vp],
            "pam_nn_conv3x3_wgrad": [vp, i32, vp, i32, i32, i32, i32, i32, i32, vp, vp, vp],
            "pam_nn_relu_backward": [vp, i32, vp, i32, i64, i32, vp],
            "pam_nn_maxpool": [vp, i32, i32, i32, i32, i32, vp, i32, vp, vp],
            "pam_nn_maxpool_backward": [vp, i32, vp, i32, i32, i32, i32, vp, i32, i32, vp],
            "pam_nn_upsample": [vp, i32, i32, i32, i32, i32, vp, i32, vp],
            "pam_nn_upsample_backward": [vp, i32, i32, i32, i32, i32, vp, i32, vp],
            "pam_nn_head": [vp, i32, i64, vp, vp, vp, vp, vp, vp, vp, vp, i64, vp],
            "pam_nn_loss_weights": [vp, i32, i64, f32, vp, vp],
            "pam_nn_head_backward": [vp, i32, i64, vp, vp, vp, vp, vp, vp],
            "pam_nn_adam": [vp, vp, vp, vp, i64, f32, f32, f32, f32, i32, vp],
            "pam_nn_pack_weights": [vp, i32, i32, vp, vp, vp],
            "pam_nn_features": [vp, i32, i64, vp, vp],
            "pam_nn_confidence": [vp, vp, i32, i64, vp, vp],
            "pam_nn_apply_mask": [vp, vp, vp, i64, vp],
            "pam_nn_coherence_features": [vp, i32, i64, i32, i32, i32, vp, vp, vp, vp],
            "pam_nn_error_estimate": [vp, vp, vp, i32, i64, vp, vp],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = C.c_int
        _NN = L
    return _NN


def _p(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _s(stream):
    import torch
    return C.c_void_p((stream or torch.cuda.current_stream()).cuda_stream)


def _call(name, *args):
    st = getattr(lib(), name)(*args)
    if st != 0:
        raise pam.PamError(st, name)


def conv3x3(x, ldx, batch, h, w, k_in, wt, bias, y, ldy, n_out, relu=True, flip=False, accumulate=False, stream=None):
    _call("pam_nn_conv3x3", _p(x), ldx, batch, h, w, k_in, _p(wt), _p(bias), _p(y), ldy, n_out, int(relu),
          int(flip), int(accumulate), _s(stream))


def conv3x3_wgrad(x, ldx, dy, lddy, batch, h, w, c_in, c_out, dw, db, stream=None):
    _call("pam_nn_conv3x3_wgrad", _p(x), ldx, _p(dy), lddy, batch, h, w, c_in, c_out, _p(dw), _p(db), _s(stream))


def relu_backward(y, ldy, dy, lddy, pixels, c, stream=None):
    _call("pam_nn_relu_backward", _p(y), ldy, _p(dy), lddy, pixels, c, _s(stream))


def maxpool(x, ldx, batch, h, w, c, y, ldy, arg, stream=None):
    _call("pam_nn_maxpool", _p(x), ldx, batch, h, w, c, _p(y), ldy, _p(arg), _s(stream))


def maxpool_backward(dy, lddy, arg, batch, h, w, c, dx, lddx, accumulate, stream=None):
    _call("pam_nn_maxpool_backward", _p(dy), lddy, _p(arg), batch, h, w, c, _p(dx), lddx, int(accumulate), _s(stream))


def upsample(x, ldx, batch, h, w, c, y, ldy, stream=None):
    _call("pam_nn_upsample", _p(x), ldx, batch, h, w, c, _p(y), ldy, _s(stream))


def upsample_backward(dy, lddy, batch, h, w, c, dx, lddx, stream=None):
    _call("pam_nn_upsample_backward", _p(dy), lddy, batch, h, w, c, _p(dx), lddx, _s(stream))


def head(feat, c, pixels, w, b, target, weight, mask, err, dz, loss, count, stream=None):
    _call("pam_nn_head", _p(feat), c, pixels, _p(w), _p(b), _p(target), _p(weight), _p(mask), _p(err), _p(dz),
          _p(loss), count, _s(stream))


def loss_weights(energy, batch, pixels, mix, out, stream=None):
    _call("pam_nn_loss_weights", _p(energy), batch, pixels, mix, _p(out), _s(stream))


def head_backward(feat, c, pixels, w, dz, dfeat, dw, db, stream=None):
    _call("pam_nn_head_backward", _p(feat), c, pixels, _p(w), _p(dz), _p(dfeat), _p(dw), _p(db), _s(stream))


def adam(p, g, m, v, lr, beta1, beta2, eps, step, stream=None):
    _call("pam_nn_adam", _p(p), _p(g), _p(m), _p(v), p.numel(), lr, beta1, beta2, eps, step, _s(stream))


def pack_weights(w, c_in, c_out, wt, wd, stream=None):
    _call("pam_nn_pack_weights", _p(w), c_in, c_out, _p(wt), _p(wd), _s(stream))


def features(energy, batch, pixels, out, stream=None):
    _call("pam_nn_features", _p(energy), batch, pixels, _p(out), _s(stream))


def confidence(err, energy, batch, pixels, conf, stream=None):
    _call("pam_nn_confidence", _p(err), _p(energy), batch, pixels, _p(conf), _s(stream))


def apply_mask(mask, energy, image, stream=None):
    _call("pam_nn_apply_mask", _p(mask), _p(energy), _p(image), mask.numel(), _s(stream))


def coherence_features(accum, n_split, split_stride, batch, n_z, n_x, out, energy, frame_max, stream=None):
    _call("pam_nn_coherence_features", _p(accum), n_split, split_stride, batch, n_z, n_x, _p(out), _p(energy),
          _p(frame_max), _s(stream))


def error_estimate(mask, err, energy, batch, pixels, est, stream=None):
    _call("pam_nn_error_estimate", _p(mask), _p(err), _p(energy), batch, pixels, _p(est), _s(stream))
