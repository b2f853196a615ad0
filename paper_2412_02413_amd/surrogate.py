"""Learned NCC-mask surrogate for AS-TAX.

AS-TAX forms its image as I = rho_n^2 * E (Eq. 11) where E is the energy of the
summed sub-aperture fields and rho_n the normalised TAX weight (Eq. 10), which
costs three angular-spectrum propagations.  With complementary masks, E equals
the plain full-aperture AS image (Eq. 3), which costs one.  The surrogate is a
U-Net that predicts rho_n from that one propagation: its energy and the
normalised cross-spectra of adjacent pixels (how coherent the field is from
column to column and from depth to depth over the band), plus a per-pixel
estimate of its own error.  The error estimate gives a predicted relative L2
error of the frame's image; a frame whose prediction exceeds a per-geometry
threshold falls back to plain AS-TAX.  The threshold is calibrated on held-out
frames of that geometry (split conformal on the ratio of true to predicted
error) so that an accepted frame exceeds a stated image-error bound with
probability at most alpha.  Plain AS-TAX on the GPU generates the training
targets and is the reference the surrogate's images are scored against.

Every numerical step runs in the HIP library: the reconstructions through
pam_as_tax, the network through the pam_nn_* kernels.  This module owns the
parameters (FP32 master copies, BF16 packed copies for the matrix cores, Adam
moments), the activation buffers and the order of the calls.
"""
from __future__ import annotations

import math
import os
import time
from dataclasses import dataclass
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import nn, pam, synth

C_FEAT = 32   # input channels of the first convolution (N_FEAT features, zero padded)
N_FEAT = 8    # energy (2) and adjacent-pixel coherence (6) features


@dataclass
class ConvSpec:
    name: str
    c_in: int
    c_out: int


class UNet:
    """U-Net of `levels` levels with base*2^l channels at level l (see oracle conventions in
    include/pam_nn.h): two 3x3 convolutions + ReLU per level, 2x2 max pooling, nearest 2x
    upsampling with skip concatenation [upsampled, skip], a 1x1 head with two outputs."""

    def __init__(self, levels: int = 4, base: int = 32, seed: int = 0, device: str = "cuda", n_feat: int = N_FEAT):
        import torch
        self.torch = torch
        self.levels, self.base, self.n_feat = levels, base, n_feat
        self.device = torch.device(device)
        self.ch = [base * 2 ** l for l in range(levels)]
        self.specs: List[ConvSpec] = []
        prev = C_FEAT
        for l in range(levels):
            self.specs += [ConvSpec(f"enc{l}a", prev, self.ch[l]), ConvSpec(f"enc{l}b", self.ch[l], self.ch[l])]
            prev = self.ch[l]
        for l in range(levels - 2, -1, -1):
            self.specs += [ConvSpec(f"dec{l}a", self.ch[l + 1] + self.ch[l], self.ch[l]),
                           ConvSpec(f"dec{l}b", self.ch[l], self.ch[l])]
        self.spec = {s.name: s for s in self.specs}
        rng = np.random.default_rng(seed)
        host = {}
        for s in self.specs:
            live = n_feat if s.name == "enc0a" else s.c_in
            fan_in = 9 * live
            w = np.zeros((9, s.c_in, s.c_out))
            w[:, :live, :] = rng.standard_normal((9, live, s.c_out)) * math.sqrt(2.0 / fan_in)
            host[s.name + ".w"] = w
            host[s.name + ".b"] = np.zeros(s.c_out)
        host["head.w"] = rng.standard_normal((self.ch[0], 2)) * math.sqrt(1.0 / self.ch[0])
        host["head.b"] = np.zeros(2)
        self.load_host_params(host)
        self.step_count = 0
        self.cache = {}

    # -- parameters ----------------------------------------------------------------
    def load_host_params(self, host: Dict[str, np.ndarray]):
        torch = self.torch
        self.params = {k: torch.tensor(v, dtype=torch.float32, device=self.device).contiguous() for k, v in host.items()}
        self.grads = {k: torch.zeros_like(v) for k, v in self.params.items()}
        self.m = {k: torch.zeros_like(v) for k, v in self.params.items()}
        self.v = {k: torch.zeros_like(v) for k, v in self.params.items()}
        self.wt, self.wd = {}, {}
        for s in self.specs:
            self.wt[s.name] = torch.empty((s.c_out, 9, s.c_in), dtype=torch.bfloat16, device=self.device)
            self.wd[s.name] = torch.empty((s.c_in, 9, s.c_out), dtype=torch.bfloat16, device=self.device)
        self.pack()

    def pack(self):
        for s in self.specs:
            nn.pack_weights(self.params[s.name + ".w"], s.c_in, s.c_out, self.wt[s.name], self.wd[s.name])

    def host_params(self) -> Dict[str, np.ndarray]:
        return {k: v.double().cpu().numpy() for k, v in self.params.items()}

    def state_dict(self):
        return {"levels": self.levels, "base": self.base, "step": self.step_count,
                **{f"p.{k}": v for k, v in self.params.items()},
                **{f"m.{k}": v for k, v in self.m.items()}, **{f"v.{k}": v for k, v in self.v.items()}}

    @classmethod
    def from_weights(cls, path, device: str = "cuda"):
        """Network and its per-geometry calibration from an inference-weights file."""
        import json
        from safetensors import safe_open
        with safe_open(path, framework="pt") as f:
            meta = f.metadata()
            net = cls(int(meta["levels"]), int(meta["base"]), device=device, n_feat=int(meta["n_feat"]))
            for k in net.params:
                net.params[k].copy_(f.get_tensor(k))
        net.pack()
        return net, json.loads(meta["calibration"])

    def save_weights(self, path, calibration: Dict[str, dict]):
        import json
        from safetensors.torch import save_file
        save_file({k: v.detach().cpu().contiguous() for k, v in self.params.items()}, path,
                  metadata={"levels": str(self.levels), "base": str(self.base), "n_feat": str(self.n_feat),
                            "features": "energy + adjacent-pixel coherence",
                            "calibration": json.dumps(calibration)})

    def load_state_dict(self, sd):
        for k in self.params:
            self.params[k].copy_(sd[f"p.{k}"])
            self.m[k].copy_(sd[f"m.{k}"])
            self.v[k].copy_(sd[f"v.{k}"])
        self.step_count = int(sd["step"])
        self.pack()

    # -- forward ---------------------------------------------------------------------
    def _buf(self, key, shape, dtype=None):
        torch = self.torch
        dtype = dtype or torch.bfloat16
        t = self.cache.get(key)
        if t is None or tuple(t.shape) != tuple(shape) or t.dtype != dtype:
            t = torch.empty(shape, dtype=dtype, device=self.device)
            self.cache[key] = t
        return t

    def forward(self, x, B: int, H: int, W: int):
        """x: BF16 [B][H][W][C_FEAT].  Returns (mask, err) FP32 [B][H][W]; keeps activations."""
        L, ch = self.levels, self.ch
        self.shape = (B, H, W)
        self.x = x
        h, ld_h = x, C_FEAT
        for l in range(L):
            Hl, Wl = H >> l, W >> l
            if l > 0:
                Hp, Wp = H >> (l - 1), W >> (l - 1)
                src, ld_src = self.skip_view(l - 1)
                pooled = self._buf(f"pool{l}", (B, Hl, Wl, ch[l - 1]))
                arg = self._buf(f"arg{l}", (B, Hl, Wl, ch[l - 1]), self.torch.uint8)
                nn.maxpool(src, ld_src, B, Hp, Wp, ch[l - 1], pooled, ch[l - 1], arg)
                h, ld_h = pooled, ch[l - 1]
            a_out = self._buf(f"enc{l}a", (B, Hl, Wl, ch[l]))
            s = self.spec[f"enc{l}a"]
            nn.conv3x3(h, ld_h, B, Hl, Wl, s.c_in, self.wt[s.name], self.params[s.name + ".b"], a_out, ch[l],
                       ch[l], relu=True)
            out, ld_out = self.skip_view(l)
            nn.conv3x3(a_out, ch[l], B, Hl, Wl, ch[l], self.wt[f"enc{l}b"], self.params[f"enc{l}b.b"], out,
                       ld_out, ch[l], relu=True)
            h, ld_h = out, ld_out
        for l in range(L - 2, -1, -1):
            Hl, Wl = H >> l, W >> l
            cat = self._buf(f"cat{l}", (B, Hl, Wl, ch[l + 1] + ch[l]))
            nn.upsample(h, ld_h, B, Hl // 2, Wl // 2, ch[l + 1], cat, ch[l + 1] + ch[l])
            da = self._buf(f"dec{l}a", (B, Hl, Wl, ch[l]))
            nn.conv3x3(cat, ch[l + 1] + ch[l], B, Hl, Wl, ch[l + 1] + ch[l], self.wt[f"dec{l}a"],
                       self.params[f"dec{l}a.b"], da, ch[l], ch[l], relu=True)
            db = self._buf(f"dec{l}b", (B, Hl, Wl, ch[l]))
            nn.conv3x3(da, ch[l], B, Hl, Wl, ch[l], self.wt[f"dec{l}b"], self.params[f"dec{l}b.b"], db, ch[l],
                       ch[l], relu=True)
            h, ld_h = db, ch[l]
        self.feat = h
        mask = self._buf("mask", (B, H, W), self.torch.float32)
        err = self._buf("err", (B, H, W), self.torch.float32)
        nn.head(h, ch[0], B * H * W, self.params["head.w"], self.params["head.b"], None, None, mask, err, None,
                None, B * H * W)
        return mask, err

    def skip_view(self, l):
        """Output of encoder level l: a channel slice of the decoder's concat buffer
        (channels [C_{l+1}, C_{l+1} + C_l)) except at the deepest level."""
        B, H, W = self.shape
        ch = self.ch
        if l == self.levels - 1:
            return self._buf(f"enc{l}b", (B, H >> l, W >> l, ch[l])), ch[l]
        cat = self._buf(f"cat{l}", (B, H >> l, W >> l, ch[l + 1] + ch[l]))
        return cat.view(-1)[ch[l + 1]:], ch[l + 1] + ch[l]

    # -- loss and backward -------------------------------------------------------------
    def loss_backward(self, target, weight=None):
        """Head loss against target (FP32 [B][H][W]) with optional per-pixel weights (FP32
        [B][H][W]; default the mean over pixels) and gradients of every parameter."""
        torch = self.torch
        B, H, W = self.shape
        L, ch = self.levels, self.ch
        P0 = B * H * W
        mask, err = self.cache["mask"], self.cache["err"]
        dz = self._buf("dz", (P0, 2), torch.float32)
        loss = self._buf("loss", (3,), torch.float32)   # BCE mask, BCE error head, weighted mask L1
        loss.zero_()
        for g in self.grads.values():
            g.zero_()
        nn.head(self.feat, ch[0], P0, self.params["head.w"], self.params["head.b"], target, weight, mask, err, dz,
                loss, P0)
        d = self._buf("gdec0b", (B, H, W, ch[0]))
        nn.head_backward(self.feat, ch[0], P0, self.params["head.w"], dz, d, self.grads["head.w"],
                         self.grads["head.b"])

        def conv_back(name, x, ldx, y, ldy, dy, lddy, Hl, Wl, want_dx, dx=None, lddx=0):
            s = self.spec[name]
            nn.relu_backward(y, ldy, dy, lddy, B * Hl * Wl, s.c_out)
            nn.conv3x3_wgrad(x, ldx, dy, lddy, B, Hl, Wl, s.c_in, s.c_out, self.grads[name + ".w"],
                             self.grads[name + ".b"])
            if want_dx:
                nn.conv3x3(dy, lddy, B, Hl, Wl, s.c_out, self.wd[name], None, dx, lddx, s.c_in, relu=False,
                           flip=True)

        for l in range(0, L - 1):
            Hl, Wl = H >> l, W >> l
            cw = ch[l + 1] + ch[l]
            gda = self._buf(f"gdec{l}a", (B, Hl, Wl, ch[l]))
            conv_back(f"dec{l}b", self.cache[f"dec{l}a"], ch[l], self.cache[f"dec{l}b"], ch[l], d, ch[l], Hl, Wl,
                      True, gda, ch[l])
            gcat = self._buf(f"gcat{l}", (B, Hl, Wl, cw))
            conv_back(f"dec{l}a", self.cache[f"cat{l}"], cw, self.cache[f"dec{l}a"], ch[l], gda, ch[l], Hl, Wl,
                      True, gcat, cw)
            nxt = self._buf(f"gdec{l + 1}b" if l + 1 <= L - 2 else f"genc{L - 1}b",
                            (B, Hl // 2, Wl // 2, ch[l + 1]))
            nn.upsample_backward(gcat, cw, B, Hl // 2, Wl // 2, ch[l + 1], nxt, ch[l + 1])
            d = nxt
        ld_d = ch[L - 1]
        for l in range(L - 1, -1, -1):
            Hl, Wl = H >> l, W >> l
            out, ld_out = self.skip_view(l)
            gea = self._buf(f"genc{l}a", (B, Hl, Wl, ch[l]))
            conv_back(f"enc{l}b", self.cache[f"enc{l}a"], ch[l], out, ld_out, d, ld_d, Hl, Wl, True, gea, ch[l])
            if l == 0:
                conv_back("enc0a", self.x, C_FEAT, self.cache["enc0a"], ch[0], gea, ch[0], Hl, Wl, False)
            else:
                gpool = self._buf(f"gpool{l}", (B, Hl, Wl, ch[l - 1]))
                conv_back(f"enc{l}a", self.cache[f"pool{l}"], ch[l - 1], self.cache[f"enc{l}a"], ch[l], gea, ch[l],
                          Hl, Wl, True, gpool, ch[l - 1])
                # gradient at the skip output of level l-1: the decoder's share (already in
                # the skip slice of gcat{l-1}) plus the pooling path
                gcat = self._buf(f"gcat{l - 1}", (B, Hl * 2, Wl * 2, ch[l] + ch[l - 1]))
                gskip = gcat.view(-1)[ch[l]:]
                nn.maxpool_backward(gpool, ch[l - 1], self.cache[f"arg{l}"], B, Hl * 2, Wl * 2, ch[l - 1], gskip,
                                    ch[l] + ch[l - 1], True)
                d, ld_d = gskip, ch[l] + ch[l - 1]
        return loss

    def adam_step(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step_count += 1
        for k in self.params:
            nn.adam(self.params[k], self.grads[k], self.m[k], self.v[k], lr, beta1, beta2, eps, self.step_count)
        self.pack()


# ----------------------------------------------------------------------------
# Data: frames from the generator, targets from plain AS-TAX on the GPU
# ----------------------------------------------------------------------------

def _frame(seed):
    """Training workload: 64-element array, 1-20 emitters, SNR uniform in [0, 30] dB."""
    return synth.cfg4_frame(seed)[0]


def _frame_headline(seed):
    """Benchmark workload: 128-element array, 4096 samples, 3 stable + 2 inertial emitters."""
    return synth.cfg2_frame(seed)[0]


FRAME_KINDS = {"train": _frame, "headline": _frame_headline}


def generate_rf(seeds: Sequence[int], workers: int = 0, kind: str = "train") -> np.ndarray:
    fn = FRAME_KINDS[kind]
    if workers and len(seeds) > 32:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(workers) as pool:
            frames = pool.map(fn, list(seeds), chunksize=16)
    else:
        frames = [fn(s) for s in seeds]
    return np.stack(frames)


def geometry_key(geom) -> str:
    """Calibration key of an array / record / grid set-up."""
    bands = "+".join(f"{lo:.6g}-{hi:.6g}" for lo, hi in geom.bands_hz)
    return (f"L{geom.n_elements}_p{geom.pitch_m:.6g}_fs{geom.fs_hz:.6g}_nt{geom.n_samples}_b{bands}"
            f"_x{geom.n_x}{geom.lateral}_z{len(geom.depths_m)}")


class Teacher:
    """Plain AS-TAX on the GPU: the image and NNCC rho_n of each frame."""

    def __init__(self, geom, precision: str = "fp32", max_frames: int = 64):
        import torch
        self.torch = torch
        self.geom = geom
        self.plan = pam.pam_plan(geom, 0, precision)
        self.max_frames = max_frames
        self.ws = pam.alloc_workspace(self.plan, max_frames, geom.n_samples)

    def __call__(self, rf):
        torch = self.torch
        F = rf.shape[0]
        assert F <= self.max_frames
        lay = pam.pam_workspace_layout(self.plan, F, self.geom.n_samples)
        img = torch.empty((F, self.plan.n_z, self.plan.n_x), device=rf.device)
        nncc = torch.empty_like(img)
        pam.pam_as_tax(self.plan, rf, img, nncc, None, self.ws[:lay.total])
        return nncc, img

    def close(self):
        pam.pam_destroy(self.plan)


class FullAperture:
    """One full-aperture propagation with the adjacent-pixel cross-spectra (an n_sub = 1
    plan with coherence): the energy E (the plain AS image) and the accumulator channels
    S, G_x, G_z left in the workspace."""

    def __init__(self, geom, precision: str = "fp32", max_frames: int = 64):
        import torch
        self.torch = torch
        self.geom = geom.replace(n_sub=1, apod=np.ones((1, geom.n_elements), np.uint8), coherence=1)
        self.plan = pam.pam_plan(self.geom, 0, precision)
        self.max_frames = max_frames
        self.ws = pam.alloc_workspace(self.plan, max_frames, geom.n_samples)
        self.P = self.plan.n_z * self.plan.n_x

    def __call__(self, rf):
        """Returns (E [F][n_z][n_x], accum [n_split * F * 5 * P] FP32 view, n_split)."""
        torch = self.torch
        F = rf.shape[0]
        assert F <= self.max_frames
        lay = pam.pam_workspace_layout(self.plan, F, self.geom.n_samples)
        E = torch.empty((F, self.plan.n_z, self.plan.n_x), device=rf.device)
        pam.pam_as_tax(self.plan, rf, E, None, None, self.ws[:lay.total])
        assert lay.n_acc == 5
        acc = self.ws[lay.accum: lay.accum + lay.n_split * F * 5 * self.P * 4].view(torch.float32)
        return E, acc, lay.n_split

    def reduced(self, rf):
        """Accumulator channels summed over the bin splits: FP32 [F][5][n_z][n_x]."""
        E, acc, n_split = self(rf)
        F = rf.shape[0]
        a = acc.view(n_split, F, 5, self.plan.n_z, self.plan.n_x)
        return a[0].clone() if n_split == 1 else a.sum(0)

    def close(self):
        pam.pam_destroy(self.plan)


def build_dataset(seeds, geom, chunk: int = 64, workers: int = 16, log=None, kind: str = "train"):
    """Accumulator channels A (FP32 [n][5][n_z][n_x]: S = E, G_x, G_z of the full aperture)
    and NNCC targets R (FP32 [n][n_z][n_x]) of the given frames, as device tensors."""
    import torch
    t = Teacher(geom, max_frames=chunk)
    fa = FullAperture(geom, max_frames=chunk)
    A, R = [], []
    try:
        for i in range(0, len(seeds), 512):
            rf = generate_rf(seeds[i:i + 512], workers, kind)
            for j in range(0, rf.shape[0], chunk):
                x = torch.from_numpy(rf[j:j + chunk]).cuda()
                r, _ = t(x)
                A.append(fa.reduced(x))
                R.append(r.clone())
            if log:
                log(f"dataset: {min(i + 512, len(seeds))}/{len(seeds)} frames")
    finally:
        torch.cuda.synchronize()
        t.close()
        fa.close()
    return torch.cat(A), torch.cat(R)


def features(A, feats, energy, fmax):
    """Network input, energy and per-frame maximum energy of frames A (FP32 [b][5][n_z][n_x],
    one split)."""
    b, _, H, W = A.shape
    nn.coherence_features(A, 1, 0, b, H, W, feats, energy, fmax)


# ----------------------------------------------------------------------------
# Training and inference
# ----------------------------------------------------------------------------

def train(net: UNet, A, R, steps: int, batch: int = 8, lr: float = 1e-3, seed: int = 0, log=None, log_every=50,
          mix: float = 0.1, rng: Optional[np.random.Generator] = None):
    """Adam on batches drawn from (A, R); the loss weights each pixel by its share of the
    frame's energy (blended with a uniform share `mix`), where the mask shapes the image.
    The batches come from `rng` (advanced in place, so a run resumes from a checkpoint of
    the network, its Adam state and rng.bit_generator.state) or a fresh generator seeded
    with `seed`."""
    torch = net.torch
    n, _, H, W = A.shape
    feats = torch.empty((batch, H, W, C_FEAT), dtype=torch.bfloat16, device=net.device)
    e = torch.empty((batch, H, W), dtype=torch.float32, device=net.device)
    wts = torch.empty((batch, H, W), dtype=torch.float32, device=net.device)
    fmax = torch.empty(batch, dtype=torch.float32, device=net.device)
    rng = np.random.default_rng(seed) if rng is None else rng
    hist = []
    t0 = time.perf_counter()
    for it in range(steps):
        idx = torch.as_tensor(rng.choice(n, size=batch, replace=False), device=net.device)
        a = A.index_select(0, idx).contiguous()
        r = R.index_select(0, idx).contiguous()
        features(a, feats, e, fmax)
        nn.loss_weights(e, batch, H * W, mix, wts)
        net.forward(feats, batch, H, W)
        loss = net.loss_backward(r, wts)
        net.adam_step(lr=lr)
        if it % log_every == 0 or it == steps - 1:
            l = loss.cpu().numpy()
            hist.append((it, float(l[0]), float(l[1]), float(l[2])))
            if log:
                log(f"step {it}: BCE mask {l[0]:.4f} BCE err {l[1]:.4f} weighted mask L1 {l[2]:.4f} "
                    f"({time.perf_counter() - t0:.1f} s)")
    return hist


def _infer(net: UNet, feats, e, b, H, W):
    torch = net.torch
    m, er = net.forward(feats[:b], b, H, W)
    est = torch.empty(b, dtype=torch.float32, device=net.device)
    nn.error_estimate(m, er, e[:b], b, H * W, est)
    return m, er, est


def predict(net: UNet, A, batch: int = 8):
    """Mask, per-pixel predicted error and predicted image error of frames A [n][5][H][W]."""
    torch = net.torch
    n, _, H, W = A.shape
    feats = torch.empty((batch, H, W, C_FEAT), dtype=torch.bfloat16, device=net.device)
    e = torch.empty((batch, H, W), dtype=torch.float32, device=net.device)
    fmax = torch.empty(batch, dtype=torch.float32, device=net.device)
    masks, errs, ests = [], [], []
    for i in range(0, n, batch):
        b = min(batch, n - i)
        features(A[i:i + b].contiguous(), feats, e, fmax)
        m, er, est = _infer(net, feats, e, b, H, W)
        masks.append(m.clone())
        errs.append(er.clone())
        ests.append(est)
    return torch.cat(masks), torch.cat(errs), torch.cat(ests)


def calibrate(est, actual, bound: float, alpha: float) -> dict:
    """Threshold on the predicted image error for a stated bound.

    Split conformal on r = actual / predicted error over n calibration frames: q is the
    ceil((n + 1)(1 - alpha))-th smallest r, and a frame is accepted when its predicted
    error is at most tau = bound / q.  For a new frame exchangeable with the calibration
    frames, P(r <= q) >= 1 - alpha, and an accepted frame with r <= q has an image error
    of at most q * (bound / q) = bound, so the probability that a frame is accepted yet
    exceeds the bound is at most alpha."""
    est = np.asarray(est, dtype=np.float64)
    actual = np.asarray(actual, dtype=np.float64)
    n = len(est)
    r = np.sort(np.where(est > 0, actual / np.maximum(est, 1e-300), np.inf))
    k = int(math.ceil((n + 1) * (1 - alpha)))
    q = float(r[k - 1]) if k <= n else math.inf
    tau = bound / q if q > 0 else math.inf
    accepted = est <= tau
    return {"tau": tau, "q": q, "bound": bound, "alpha": alpha, "n": n,
            "calibration_accept_rate": float(accepted.mean()),
            "calibration_accepted_over_bound": float((accepted & (actual > bound)).mean())}


class SurrogatePipeline:
    """Surrogate AS-TAX: one full-aperture propagation with the pair cross-spectra + network
    mask; frames whose predicted image error exceeds tau are recomputed with plain AS-TAX
    (tau < 0: every frame; tau = inf: none)."""

    def __init__(self, geom, net: UNet, tau: float, precision: str = "fp32", max_frames: int = 64,
                 batch: int = 16):
        import torch
        self.torch = torch
        self.geom, self.net, self.tau = geom, net, tau
        self.fa = FullAperture(geom, precision, max_frames)
        self.teacher = Teacher(geom, precision, max_frames)
        self.batch = batch
        H, W = self.fa.plan.n_z, self.fa.plan.n_x
        self.feats = torch.empty((batch, H, W, C_FEAT), dtype=torch.bfloat16, device=net.device)
        self.e = torch.empty((batch, H, W), dtype=torch.float32, device=net.device)
        self.fmax = torch.empty(batch, dtype=torch.float32, device=net.device)

    def __call__(self, rf):
        torch = self.torch
        F = rf.shape[0]
        H, W = self.fa.plan.n_z, self.fa.plan.n_x
        P = H * W
        E, acc, n_split = self.fa(rf)                       # plain AS image = E
        mask = torch.empty_like(E)
        est = torch.empty(F, dtype=torch.float32, device=rf.device)
        for i in range(0, F, self.batch):
            b = min(self.batch, F - i)
            nn.coherence_features(acc[i * 5 * P:], n_split, F * 5 * P, b, H, W, self.feats, self.e, self.fmax)
            m, _, es = _infer(self.net, self.feats, self.e, b, H, W)
            mask[i:i + b].copy_(m)
            est[i:i + b].copy_(es)
        image = torch.empty_like(E)
        nn.apply_mask(mask, E, image)
        fallback = (est > self.tau).cpu().numpy()
        if fallback.any():
            idx = np.nonzero(fallback)[0]
            sel = torch.as_tensor(idx, device=rf.device)
            _, img3 = self.teacher(rf.index_select(0, sel).contiguous())
            image.index_copy_(0, sel, img3)
        return image, mask, est, fallback

    def close(self):
        self.fa.close()
        self.teacher.close()


# ----------------------------------------------------------------------------
# Evaluation (Section II-E metrics) and the training / evaluation driver
# ----------------------------------------------------------------------------

def image_metrics(I):
    """ESA in pixels (area above half the maximum) and ISNR in dB (Eq. 12) per frame."""
    torch = __import__("torch")
    mx = I.flatten(1).max(dim=1).values[:, None, None]
    inside = I > 0.5 * mx
    n_in = inside.flatten(1).sum(1).double()
    s_in = (I * inside).flatten(1).sum(1).double()
    s_out = (I * ~inside).flatten(1).sum(1).double()
    n_out = I[0].numel() - n_in
    isnr = 10 * torch.log10((s_in / n_in) / (s_out / n_out).clamp_min(1e-300))
    return n_in, isnr


def image_errors(E, R, mask):
    """Relative L2 error of each frame's image mask^2 E against AS-TAX's rho_n^2 E."""
    I_ref = R * R * E
    I = mask * mask * E
    return ((I - I_ref).flatten(1).norm(dim=1) / I_ref.flatten(1).norm(dim=1)).double()


def compare(E, R, mask, label):
    """Image error and metric differences of I = mask^2 E against AS-TAX's I = rho_n^2 E."""
    rel = image_errors(E, R, mask)
    esa_r, isnr_r = image_metrics(R * R * E)
    esa, isnr = image_metrics(mask * mask * E)
    w = E / E.flatten(1).sum(1)[:, None, None]
    ml1 = ((mask - R).abs() * w).flatten(1).sum(1).double()
    return {"form": label, "image_rel_l2_mean": float(rel.mean()), "image_rel_l2_p95": float(rel.quantile(0.95)),
            "image_rel_l2_max": float(rel.max()),
            "mask_l1_energy_weighted_mean": float(ml1.mean()),
            "mask_l1_mean": float((mask - R).abs().flatten(1).mean(1).mean()),
            "abs_d_isnr_db_mean": float((isnr - isnr_r).abs().mean()),
            "abs_d_esa_rel_mean": float(((esa - esa_r).abs() / esa_r).mean())}


def evaluate(net, A, R, cal: dict):
    """Held-out frames against a calibration: fallback rate, the fraction of frames accepted
    yet over the bound, and the images with fallback, alone and of the baselines."""
    import torch
    E = A[:, 0]
    m, _, est = predict(net, A)
    err = image_errors(E, R, m)
    fb = est > cal["tau"]
    accepted = ~fb
    m_fb = torch.where(fb[:, None, None], R, m)
    as3 = E / E.flatten(1).max(1).values[:, None, None]
    est_d = est.double()
    return {"frames": int(E.shape[0]), "tau": cal["tau"], "bound": cal["bound"], "alpha": cal["alpha"],
            "fallback_rate": float(fb.float().mean()),
            "accepted_over_bound": float((accepted & (err > cal["bound"])).float().mean()),
            "accepted_error_mean": float(err[accepted].mean()) if bool(accepted.any()) else None,
            "predicted_vs_actual_error_corr": float(torch.corrcoef(torch.stack([est_d, err]))[0, 1]),
            "results": [compare(E, R, m_fb, "surrogate with fallback"), compare(E, R, m, "surrogate alone"),
                        compare(E, R, torch.ones_like(m), "plain AS (weight 1)"),
                        compare(E, R, as3, "AS^3 self-mask (appendix)")]}


def calibration_for(net, A, R, bound, alpha):
    m, _, est = predict(net, A)
    err = image_errors(A[:, 0], R, m)
    return calibrate(est.cpu().numpy(), err.cpu().numpy(), bound, alpha)


def main(argv=None):
    import argparse
    import json
    import sys
    import torch
    ap = argparse.ArgumentParser(description="train, calibrate and evaluate the NCC-mask surrogate")
    ap.add_argument("--train", type=int, default=20000)
    ap.add_argument("--val", type=int, default=1000, help="calibration frames of the training geometry")
    ap.add_argument("--eval", type=int, default=2000)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=3e-4)
    ap.add_argument("--levels", type=int, default=4)
    ap.add_argument("--base", type=int, default=32)
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--bound", type=float, default=0.25, help="image relative L2 error bound")
    ap.add_argument("--alpha", type=float, default=0.05, help="allowed rate of accepted frames over the bound")
    ap.add_argument("--headline-train", type=int, default=0,
                    help="benchmark-workload frames (128 elements) added to the training set")
    ap.add_argument("--headline-val", type=int, default=500, help="calibration frames of the benchmark geometry")
    ap.add_argument("--headline-eval", type=int, default=128)
    ap.add_argument("--out", default="", help="training checkpoint (parameters and Adam state)")
    ap.add_argument("--weights", default="", help="inference weights (parameters and calibration, safetensors)")
    args = ap.parse_args(argv)

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    geom = synth.cfg4_geometry()
    hgeom = synth.cfg2_geometry()
    rep = {"geometry": "64 elements, 1024 samples at 20 MHz, 205 bins (1-5 MHz), 512 x 256 grid",
           "network": f"U-Net {args.levels} levels, {args.base} base channels, {N_FEAT} input features, "
                      "BF16 operands, FP32 accumulation",
           "train_frames": args.train, "headline_train_frames": args.headline_train, "val_frames": args.val,
           "headline_val_frames": args.headline_val, "eval_frames": args.eval,
           "headline_eval_frames": args.headline_eval, "steps": args.steps, "batch": args.batch, "lr": args.lr,
           "bound": args.bound, "alpha": args.alpha}
    t0 = time.perf_counter()
    A_tr, R_tr = build_dataset(list(range(args.train)), geom, workers=args.workers, log=log)
    if args.headline_train:
        Ah, Rh = build_dataset(list(range(3_000_000, 3_000_000 + args.headline_train)), hgeom,
                               workers=args.workers, log=log, kind="headline")
        A_tr, R_tr = torch.cat([A_tr, Ah]), torch.cat([R_tr, Rh])
        del Ah, Rh
    A_va, R_va = build_dataset(list(range(args.train, args.train + args.val)), geom, workers=args.workers)
    A_ev, R_ev = build_dataset(list(range(1_000_000, 1_000_000 + args.eval)), geom, workers=args.workers)
    Ah_va, Rh_va = build_dataset(list(range(5_000_000, 5_000_000 + args.headline_val)), hgeom,
                                 workers=args.workers, kind="headline")
    Ah_ev, Rh_ev = build_dataset(list(range(4_000_000, 4_000_000 + args.headline_eval)), hgeom,
                                 workers=args.workers, kind="headline")
    rep["dataset_s"] = round(time.perf_counter() - t0, 1)
    log(f"datasets in {rep['dataset_s']} s")
    net = UNet(args.levels, args.base, seed=0)
    t0 = time.perf_counter()
    hist = train(net, A_tr, R_tr, args.steps, args.batch, args.lr, log=log, log_every=max(1, args.steps // 20))
    torch.cuda.synchronize()
    rep["train_s"] = round(time.perf_counter() - t0, 1)
    rep["train_ms_per_step"] = round(1e3 * rep["train_s"] / max(1, args.steps), 2)
    rep["loss_history"] = hist
    del A_tr, R_tr
    cal = {geometry_key(geom): calibration_for(net, A_va, R_va, args.bound, args.alpha),
           geometry_key(hgeom): calibration_for(net, Ah_va, Rh_va, args.bound, args.alpha)}
    rep["calibration"] = cal
    rep["heldout"] = evaluate(net, A_ev, R_ev, cal[geometry_key(geom)])
    rep["headline"] = evaluate(net, Ah_ev, Rh_ev, cal[geometry_key(hgeom)])
    rf_h = generate_rf(list(range(4_000_000, 4_000_064)), args.workers, "headline")
    rep["ms_per_frame"] = {"train workload": timing(geom, net, generate_rf(list(range(2_000_000, 2_000_064)),
                                                                             args.workers)),
                           "benchmark workload": timing(hgeom, net, rf_h)}
    if args.out:
        os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
        torch.save(net.state_dict(), args.out)
    if args.weights:
        os.makedirs(os.path.dirname(os.path.abspath(args.weights)), exist_ok=True)
        net.save_weights(args.weights, cal)
    print(json.dumps(rep), flush=True)


def timing(geom, net, rf_host, reps: int = 5):
    """ms per frame of the surrogate pipeline (no fallback) and of plain AS-TAX, 64-frame batches."""
    import torch
    rf = torch.from_numpy(np.ascontiguousarray(rf_host)).cuda()
    F = rf.shape[0]
    pipe = SurrogatePipeline(geom, net, tau=math.inf, max_frames=F)
    teacher = Teacher(geom, max_frames=F)
    try:
        for _ in range(2):
            pipe(rf)
            teacher(rf)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            pipe(rf)
        torch.cuda.synchronize()
        t_s = (time.perf_counter() - t) / reps / F
        t = time.perf_counter()
        for _ in range(reps):
            teacher(rf)
        torch.cuda.synchronize()
        t_p = (time.perf_counter() - t) / reps / F
    finally:
        pipe.close()
        teacher.close()
    return {"surrogate (1 propagation + network)": round(1e3 * t_s, 4),
            "plain AS-TAX (3 propagations)": round(1e3 * t_p, 4)}


if __name__ == "__main__":
    main()
