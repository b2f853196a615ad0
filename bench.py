"""Benchmark of the AS-TAX hot path on one MI355X.

Workload (one step = one pam_as_tax call over a batch of 64 frames, inputs
resident in HBM): 128-element array, pitch 0.3 mm, 4096 samples at 40 MHz,
768 bins (0.5-8 MHz), image 512 depths x 256 columns, 3 stable + 2 inertial
emitters per frame at random positions, 20 dB channel noise (synthetic; the
paper's recordings are not available).

Prints ONE JSON line on stdout:
  * throughput (frames/s) and single-frame latency p50/p99 of the main form;
  * the dominant kernel (fields: propagator + two-stage inverse lateral transform +
    cross-spectra) against its roofline, timed live with HIP events on the library's
    stream: `frac` counts the method's own algorithmic flops (lateral inverse FFTs,
    propagator products, cross-spectra sums).  In FP32 the transform is a 16 x 16 FFT
    on the vector ALUs (bound "alu", FP32 vector peak); the 16-bit forms run it as
    DFT-GEMMs on the matrix cores (bound "mfma", with `mfma_util` the matrix-core
    flops they execute);
  * the other operand forms of the DFT-GEMM on the same frames;
  * the error of every form against the FP64 oracle (max and mean over 16 frames
    of this workload and 64 frames of the 64-element workload), computed by oracle
    processes on the host while the GPU legs run;
  * the mixed-record-length workload (64 frames of 2048/4096/8192 samples on one
    8192-sample plan) per form, with its error against the oracle per length;
  * the paper's comparison beamformer (FD-TEA-TAX) on the same frames;
  * the NCC-mask surrogate, the paper-shape context timings, host-copy-inclusive
    throughput, and a serving leg (Poisson arrivals at 100 / 1,000 / 5,000 frames/s
    over a fixed horizon);
  * the evaluation harness on the HIP path: apodization-pattern sweep (ISNR, NNCC
    centroid), two-source Rayleigh dips, uneven-strength regional peaks (AS, AS-TAX, AS^3);
  * the oracle timed on the host CPU (all cores and one thread; a reported
    baseline, not the target).
Diagnostics go to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "AS-TAX frames/s and p99 ms/frame (128ch, 256×512); surrogate/split vs plain"
HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"fp32": 157.3, "split_bf16": 2500.0, "split_fp16": 2500.0, "bf16": 2500.0, "fp16": 2500.0}
VALU_FP32_PEAK_TFLOPS = 157.3          # 256 CUs x 2.4 GHz x 256 FP32 flops per clock (packed FMA)
VALU_FP32_UNPACKED_TFLOPS = 78.6       # the same without packed FP32 instructions (not used in this build)
MFMA_PASSES = {"fp32": 1, "split_bf16": 3, "split_fp16": 3, "bf16": 1, "fp16": 1}
ACC_FRAMES_BENCH = 16       # frames of the benchmark workload checked against the oracle
ACC_FRAMES_SMALL = 64       # frames of the 64-element workload checked against the oracle


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ----------------------------------------------------------------------------
# work and bytes
# ----------------------------------------------------------------------------

def executed_mfma_flops(geom, n_sel: int, n_frames: int, precision: str) -> float:
    """Matrix-core flops one launch of the fields kernel executes.  N_x = 256 (factored
    transform): per (frame, bin, sub-aperture, depth) two 16-point complex DFT stages in
    real form, 2 x 32 x 32 x 2 flops per 16 outputs each, on depths padded to 16;
    otherwise the folded dense form, a real GEMM of (2 n_sub 32-padded depths) x N x N.
    Times the product passes of the operand form."""
    N, ns = geom.n_x, geom.n_sub
    if N == 256:
        per = ns * n_sel * 16 * math.ceil(geom.n_z / 16) * N * 256.0
    else:
        per = 2.0 * (2 * ns) * 32 * math.ceil(geom.n_z / 32) * N * N * n_sel
    return per * n_frames * MFMA_PASSES[precision]


def fields_algorithmic_flops(geom, n_sel: int) -> float:
    """The method's own work in the fields step per frame (complexity terms of the paper's
    run-time analysis, 5 N log2 N flops per complex FFT): the lateral inverse FFTs of every
    sub-aperture, bin and depth, the propagator products, and 12 FMAs of cross-spectra
    per pixel and bin."""
    N, nz, ns = geom.n_x, geom.n_z, geom.n_sub
    lat_ifft = ns * n_sel * nz * 5 * N * math.log2(N)
    prop = ns * n_sel * nz * N * 6
    cross = n_sel * nz * N * 24
    return lat_ifft + prop + cross


def algorithmic_flops(geom, n_sel: int) -> float:
    """Whole-path algorithmic work per frame: the fields terms plus the time and lateral
    forward FFTs."""
    N, ns = geom.n_x, geom.n_sub
    t_fft = geom.n_elements * 5 * (geom.n_samples / 2) * math.log2(geom.n_samples / 2)
    lat_fft = ns * n_sel * 5 * N * math.log2(N)
    return fields_algorithmic_flops(geom, n_sel) + t_fft + lat_fft


def algorithmic_bytes(lay, n_frames: int, n_sel: int, geom) -> float:
    """Bytes the fields kernel must move once per launch: the lateral coefficients of every
    (frame, bin, sub-aperture) in, the accumulated energy and cross-spectra sums out."""
    coeffs = n_frames * n_sel * geom.n_sub * geom.n_x * 8
    accum = lay.n_split * n_frames * lay.n_acc * geom.n_z * geom.n_x * 4
    return float(coeffs + accum)


def source_digest() -> str:
    """SHA-256 of the fields kernel's sources: traffic counters stay valid only for this code."""
    import hashlib
    h = hashlib.sha256()
    for name in ("kernels.hpp", "k3_factored.hpp", "k3_fft.hpp"):
        with open(os.path.join(ROOT, "paper_2412_02413_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def recorded_traffic(precision: str):
    """HBM bytes per launch of the fields kernel from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE scaled by a plain copy of known size), or None when the
    summary is missing or was taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", "fields_traffic_cfg2_b64.txt")
    if not os.path.exists(path):
        return None
    digest, vals = None, {}
    with open(path) as f:
        for line in f:
            parts = line.split()
            if len(parts) >= 2 and parts[0] == "source_sha256":
                digest = parts[1]
            elif parts and parts[0] == "traffic":
                kv = dict(p.split("=", 1) for p in parts[2:])
                vals[parts[1]] = int(kv["bytes_per_launch"])
    if digest != source_digest():
        return None
    return vals.get(precision)


# ----------------------------------------------------------------------------
# the oracle on the host (separate processes, started before the GPU is touched)
# ----------------------------------------------------------------------------

def _oracle_job(job: str, threads: int, conn) -> None:
    """FP64 oracle results for the accuracy check: I and rho_n per frame, plus timing."""
    from threadpoolctl import threadpool_limits
    from oracle import as_tax as O
    from paper_2412_02413_amd import synth
    out = {"job": job, "threads": threads, "frames": {}, "seconds": []}
    with threadpool_limits(threads):
        if job == "bench":
            g = synth.cfg2_geometry()
            for s in range(ACC_FRAMES_BENCH):
                rf = synth.cfg2_frame(s)[0]
                t0 = time.perf_counter()
                r = O.as_tax(rf, g)
                out["seconds"].append(time.perf_counter() - t0)
                out["frames"][s] = (r["I"], r["rho_n"])
        else:
            g = synth.cfg1_geometry()
            for s in range(ACC_FRAMES_SMALL):
                rf = synth.cfg1_frame(s)
                t0 = time.perf_counter()
                r = O.as_tax(rf, g)
                out["seconds"].append(time.perf_counter() - t0)
                out["frames"][s] = (r["I"], r["rho_n"])
            g3 = synth.cfg3_geometry()
            seen = set()
            out["mixed"] = {}
            for s in range(64):
                rf = synth.cfg3_frame(s)
                n_t = rf.shape[-1]
                if n_t in seen:
                    continue
                seen.add(n_t)
                r = O.as_tax(rf, g3.replace(n_samples=n_t))
                out["mixed"][n_t] = (s, r["I"], r["rho_n"])
    conn.send(out)
    conn.close()


def start_oracles(threads_each: int):
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    procs = []
    for job in ("bench", "small"):
        recv, send = ctx.Pipe(duplex=False)
        p = ctx.Process(target=_oracle_job, args=(job, threads_each, send), daemon=True)
        p.start()
        procs.append((job, p, recv))
    return procs


def join_oracles(procs, timeout_s: float = 600.0):
    res = {}
    for job, p, recv in procs:
        if recv.poll(timeout_s):
            res[job] = recv.recv()
        p.join(30)
    return res


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(oracle_res: dict, threads_all: int) -> dict:
    """The oracle as it stands on the host cores.  All-core figures come from the accuracy
    runs (16 benchmark frames, 64 small frames, one oracle process each); the one-thread
    figure times the oracle on one benchmark frame restricted to every 16th bin (48 of
    768 bins: the work is linear in the bin count) and scales it to the whole frame; the
    paper-shape frame (690 bins, 300 x 256) runs once on all cores."""
    from threadpoolctl import threadpool_limits
    from oracle import as_tax as O
    from paper_2412_02413_amd import synth
    out = {"kind": "oracle", "cpu_model": cpu_model(), "nproc": os.cpu_count(),
           "affinity_cpus": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None}
    b = oracle_res.get("bench")
    if b and b["seconds"]:
        sec = float(np.mean(b["seconds"]))
        out.update({"value": round(1.0 / sec, 4), "unit": "frames/s", "cores": b["threads"],
                    "sample": f"{len(b['seconds'])} frames of the benchmark workload, {b['threads']} threads "
                              f"(BLAS), {sec:.2f} s per frame"})
    s = oracle_res.get("small")
    if s and s["seconds"]:
        sec = float(np.mean(s["seconds"]))
        out["small_workload"] = {"frames_per_s": round(1.0 / sec, 3), "threads": s["threads"],
                                 "sample": f"{len(s['seconds'])} frames of the 64-element workload"}
    # one thread on a bin subset of one benchmark frame
    g = synth.cfg2_geometry()
    ks = O.bins(g.fs_hz, g.n_samples, g.bands_hz)
    sub = ks[::16]
    bands = [(k * g.fs_hz / g.n_samples, k * g.fs_hz / g.n_samples) for k in sub]
    rf = synth.cfg2_frame(0)[0]
    with threadpool_limits(1):
        t0 = time.perf_counter()
        O.as_tax(rf, g.replace(bands_hz=bands))
        dt = time.perf_counter() - t0
    per_frame = dt * len(ks) / len(sub)
    out["one_thread"] = {"value": round(1.0 / per_frame, 5), "unit": "frames/s", "cores": 1,
                         "sample": f"one benchmark frame on {len(sub)} of {len(ks)} bins: {dt:.2f} s, "
                                   f"scaled to {per_frame:.1f} s per frame"}
    # paper shape, all cores
    gp = synth.paper_geometry(690)
    rfp = synth.paper_frame(0, 690)
    with threadpool_limits(threads_all):
        t0 = time.perf_counter()
        O.as_tax(rfp, gp)
        dt = time.perf_counter() - t0
    out["paper_shape_690_bins"] = {"seconds_per_frame": round(dt, 3), "threads": threads_all,
                                   "paper_context": "Xeon 3 GHz, one thread, Matlab: 8.4 s (Table III)"}
    return out


# ----------------------------------------------------------------------------
# GPU legs
# ----------------------------------------------------------------------------

def errors_vs_oracle(images, nncc, refs) -> dict:
    """Relative L2 of the image and max |d rho_n| over all pixels, max and mean over frames."""
    e_i, e_r = [], []
    for f, (I, rho) in refs.items():
        e_i.append(float(np.linalg.norm(images[f] - I) / np.linalg.norm(I)))
        e_r.append(float(np.abs(nncc[f] - rho).max()))
    if not e_i:
        return None
    return {"rel_l2_image_max": max(e_i), "rel_l2_image_mean": float(np.mean(e_i)),
            "max_abs_nncc_max": max(e_r), "max_abs_nncc_mean": float(np.mean(e_r)), "frames": len(e_i)}


def run_frames(pam, torch, geom, rf_np, precision, dev):
    """One launch over host frames (all of one record length); images and NNCC back on the host."""
    plan = pam.pam_plan(geom, 0, precision)
    try:
        x = torch.from_numpy(np.ascontiguousarray(rf_np, np.float32)).to(dev)
        out = pam.reconstruct(plan, x, want_nncc=True)
        torch.cuda.synchronize()
        return out["image"].cpu().numpy().astype(np.float64), out["nncc"].cpu().numpy().astype(np.float64)
    finally:
        pam.pam_destroy(plan)


def mixed_lengths(pam, torch, precisions, steps, dev):
    """64 frames of the 64-element array with record lengths drawn from 2048/4096/8192 on one
    8192-sample plan (the bins of a record are every 2nd / 4th bin of the plan's), timed over
    all 64 frames as ONE grouped call (pam_as_tax_grouped: the frames packed by record length;
    the library runs the fields stage as one work-list launch where its cost estimate favours
    that, else group after group) and, for comparison, as one pam_as_tax call per record length."""
    from paper_2412_02413_amd import synth
    g = synth.cfg3_geometry()
    frames = [synth.cfg3_frame(s) for s in range(64)]
    lengths = sorted({fr.shape[-1] for fr in frames})
    groups = {n: [i for i, fr in enumerate(frames) if fr.shape[-1] == n] for n in lengths}
    glist = [(n, len(groups[n])) for n in lengths]
    dev_rf = {n: torch.from_numpy(np.stack([frames[i] for i in idx])).to(dev) for n, idx in groups.items()}
    packed = torch.cat([dev_rf[n].reshape(-1) for n in lengths]).contiguous()
    out = {"frames": 64, "record_lengths": {str(n): len(idx) for n, idx in groups.items()},
           "call": "one pam_as_tax_grouped call per 64 frames (frames packed by record length)"}
    firsts = {}
    for prec in precisions:
        plan = pam.pam_plan(g, 0, prec)
        try:
            stream = torch.cuda.current_stream(dev)
            img = torch.empty((64, g.n_z, g.n_x), device=dev)
            nn = torch.empty_like(img)
            ws = pam.alloc_workspace_grouped(plan, glist, dev)
            bufs = {}
            for n, x in dev_rf.items():
                F = x.shape[0]
                bufs[n] = (torch.empty((F, g.n_z, g.n_x), device=dev), torch.empty((F, g.n_z, g.n_x), device=dev),
                           pam.alloc_workspace(plan, F, n, dev))

            def grouped():
                pam.pam_as_tax_grouped(plan, packed, glist, img, nn, None, ws, stream)

            def per_length():
                for n, x in dev_rf.items():
                    im, nc, w = bufs[n]
                    pam.pam_as_tax(plan, x, im, nc, None, w, stream, n)

            # two rounds in alternating order, the faster of each form's two timings: neither form
            # always runs first (clock ramp, caches)
            best = {}
            for order in ((("grouped", grouped), ("per_length_calls", per_length)),
                          (("per_length_calls", per_length), ("grouped", grouped))):
                for name, fn in order:
                    fn()
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    for _ in range(steps):
                        fn()
                    torch.cuda.synchronize()
                    wall = time.perf_counter() - t0
                    best[name] = min(best.get(name, wall), wall)
            res = {name: {"frames_per_s": round(64 * steps / wall, 2), "ms_per_64_frames": round(1e3 * wall / steps, 3)}
                   for name, wall in best.items()}
            out[prec] = {**res["grouped"], "per_length_calls": res["per_length_calls"]}
            # first frame of each record length, from the grouped call (packed order)
            k, fr = 0, {}
            for n in lengths:
                fr[n] = (img[k].cpu().numpy().astype(np.float64), nn[k].cpu().numpy().astype(np.float64))
                k += len(groups[n])
            firsts[prec] = fr
        finally:
            pam.pam_destroy(plan)
    return out, firsts, groups


def surrogate_entry(geom, rf, plain_images, fps_plain, precision, steps, warmup, path):
    """The NCC-mask surrogate (one full-aperture propagation + U-Net mask, confidence
    fallback to plain AS-TAX) on the same frames: throughput, fallback rate, and its image
    against plain AS-TAX's."""
    import torch
    from paper_2412_02413_amd import surrogate as S
    net, calibration = S.UNet.from_weights(path)
    cal = calibration.get(S.geometry_key(geom))
    tau = cal["tau"] if cal else -1.0          # an uncalibrated geometry falls back on every frame
    F = rf.shape[0]
    pipe = S.SurrogatePipeline(geom, net, tau=tau, precision=precision, max_frames=F)
    try:
        for _ in range(warmup):
            pipe(rf)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fb = 0
        for _ in range(steps):
            image, _, _, fallback = pipe(rf)
            fb += int(fallback.sum())
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    finally:
        pipe.close()
    rel = ((image - plain_images).flatten(1).norm(dim=1) / plain_images.flatten(1).norm(dim=1)).double()
    _, isnr_s = S.image_metrics(image)
    _, isnr_p = S.image_metrics(plain_images)
    fps = F * steps / wall
    over = rel > cal["bound"] if cal else torch.zeros_like(rel, dtype=torch.bool)
    return {"frames_per_s": round(fps, 2), "ms_per_step": round(1e3 * wall / steps, 3),
            "speedup_vs_plain": round(fps / fps_plain, 3),
            "fallback_rule": "predicted image rel. L2 error > tau (per-geometry split-conformal calibration)",
            "tau": round(tau, 5), "bound": cal["bound"] if cal else None, "alpha": cal["alpha"] if cal else None,
            "fallback_rate": round(fb / (F * steps), 4),
            "frames_over_bound": round(float(over.float().mean()), 4),
            "image_rel_l2_vs_plain_mean": round(float(rel.mean()), 4),
            "image_rel_l2_vs_plain_p95": round(float(rel.quantile(0.95)), 4),
            "image_rel_l2_vs_plain_max": round(float(rel.max()), 4),
            "abs_d_isnr_db_mean": round(float((isnr_s - isnr_p).abs().mean()), 3),
            "network": f"U-Net {net.levels} levels, {net.base} base channels, {net.n_feat} input features "
                       "(energy, adjacent-pixel coherence), BF16 operands, FP32 accumulation",
            "weights": os.path.relpath(path, ROOT)}


def stage_rooflines(geom, n_sel: int, F: int, lay, stage_ms: dict) -> dict:
    """The smaller kernels against their own bounds, from the live stage times, by the bytes
    they must move (HBM): K1 (time FFT) the RF in and the in-band bins out; K2 (apodized
    lateral FFT into the factored order, k2_fft) the bins in and the coefficients out; K4
    (NCC / weight / image) the accumulators in, energy and weight through, image and NNCC
    out.  K2's FFT work (5 N log2 N flops per transform) is reported beside its bytes."""
    pix = geom.n_z * geom.n_x
    plane = F * pix * 4
    k1_bytes = F * geom.n_elements * geom.n_samples * 4 + F * n_sel * geom.n_elements * 8
    k2_bytes = F * n_sel * geom.n_elements * 8 + F * n_sel * geom.n_sub * geom.n_x * 8
    # accumulators in, energy + weight out; weight + energy in, image + NNCC out
    k4_bytes = lay.n_split * lay.n_acc * plane + 2 * plane + 2 * plane + 2 * plane
    out = {}
    for name, key, amount in (("time_fft", "time_fft", k1_bytes), ("lateral", "lateral", k2_bytes),
                              ("finalize", "finalize", k4_bytes)):
        ms = stage_ms[key]
        ach = amount / (ms * 1e-3) / 1e9
        out[name] = {"bound": "hbm", "achieved": round(ach, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ach / HBM_PEAK_GBS, 4), "per_launch": amount, "ms": round(ms, 4)}
    N = geom.n_x
    k2_flops = F * n_sel * geom.n_sub * 5.0 * N * math.log2(N)
    out["lateral"]["fft_flops_per_launch"] = k2_flops
    out["lateral"]["fft_tflops"] = round(k2_flops / (stage_ms["lateral"] * 1e-3) / 1e12, 2)
    return out


def paper_shape(precisions, steps: int, dev) -> dict:
    """The paper's image shape (128 elements, 2048 samples at 35.6 MHz, 2x zero-stuffing to 256
    columns, 300 depths; 690 and 128 bins): ms per frame in 64-frame launches and single-frame
    latency, to quote beside the paper's own per-image times (other hardware: context only)."""
    import torch
    from paper_2412_02413_amd import pam, synth
    out = {}
    for n_bins in (690, 128):
        g = synth.paper_geometry(n_bins)
        frames = np.stack([synth.paper_frame(s, n_bins) for s in range(8)])
        rf = torch.from_numpy(np.concatenate([frames] * 8)).to(dev)
        F = rf.shape[0]
        for prec in precisions:
            plan = pam.pam_plan(g, 0, prec)
            try:
                image = torch.empty((F, g.n_z, g.n_x), device=dev)
                ws = pam.alloc_workspace(plan, F, g.n_samples, dev)
                stream = torch.cuda.current_stream(dev)
                pam.pam_as_tax(plan, rf, image, None, None, ws, stream)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(steps):
                    pam.pam_as_tax(plan, rf, image, None, None, ws, stream)
                torch.cuda.synchronize()
                ms_frame = 1e3 * (time.perf_counter() - t0) / (steps * F)
                img1 = torch.empty((1, g.n_z, g.n_x), device=dev)
                ws1 = pam.alloc_workspace(plan, 1, g.n_samples, dev)
                lat = []
                for c in range(23):
                    torch.cuda.synchronize()
                    tw = time.perf_counter()
                    pam.pam_as_tax(plan, rf[c % F: c % F + 1], img1, None, None, ws1, stream)
                    torch.cuda.synchronize()
                    if c >= 3:
                        lat.append(1e3 * (time.perf_counter() - tw))
                out[f"{n_bins}_bins_{prec}"] = {"ms_per_frame_batched": round(ms_frame, 4),
                                                "ms_single_frame_p50_wall": round(float(np.median(lat)), 4),
                                                "bins": plan.info.n_bins}
            finally:
                pam.pam_destroy(plan)
    out["paper_context"] = "RTX 4090, CUDA: 9.8 ms (690 bins) and 1.8 ms (128 bins) per image (Table III)"
    return out


def pcie_inclusive(geom, rf_host, precision, steps, dev):
    """Throughput with the RF copied host->device (pinned) and the images copied back in
    every launch, all on one stream: the rate a caller holding frames in host memory sees."""
    import torch
    from paper_2412_02413_amd import pam
    F = rf_host.shape[0]
    plan = pam.pam_plan(geom, 0, precision)
    try:
        rf_pin = torch.from_numpy(rf_host).pin_memory()
        img_pin = torch.empty((F, geom.n_z, geom.n_x), dtype=torch.float32).pin_memory()
        rf_dev = torch.empty(rf_pin.shape, dtype=torch.float32, device=dev)
        image = torch.empty((F, geom.n_z, geom.n_x), device=dev)
        ws = pam.alloc_workspace(plan, F, geom.n_samples, dev)
        stream = torch.cuda.current_stream(dev)

        def one():
            rf_dev.copy_(rf_pin, non_blocking=True)
            pam.pam_as_tax(plan, rf_dev, image, None, None, ws, stream)
            img_pin.copy_(image, non_blocking=True)

        one()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            one()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    finally:
        pam.pam_destroy(plan)
    return {"frames_per_s": round(F * steps / wall, 2), "ms_per_step": round(1e3 * wall / steps, 3),
            "steps": steps, "copies": "RF host->device and image device->host per launch, pinned host memory"}


def fd_tea_entry(geom, rf, fps_as: float, steps: int, n_frames: int = 8) -> dict:
    """The paper's comparison beamformer (frequency-domain delay-and-sum with the same TAX
    weighting, pam_fd_tea_tax) on the first frames of the same batch, FP32, timed with
    events on the stream it runs on."""
    import torch
    from paper_2412_02413_amd import pam
    x = rf[:n_frames]
    F = x.shape[0]
    plan = pam.pam_plan(geom, 0, "fp32")
    try:
        img = torch.empty((F, geom.n_z, geom.n_x), device=x.device)
        nn_ = torch.empty_like(img)
        ws = pam.alloc_workspace(plan, F, geom.n_samples, x.device)
        pam.pam_fd_tea_tax(plan, x, img, nn_, None, ws)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            pam.pam_fd_tea_tax(plan, x, img, nn_, None, ws)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
    finally:
        pam.pam_destroy(plan)
    fps = F / (ms * 1e-3)
    return {"frames_per_s": round(fps, 2), "ms_per_frame": round(ms / F, 4), "frames_per_launch": F,
            "as_tax_fp32_over_fd_tea": round(fps_as / fps, 2),
            "paper_context": "RTX 4090: FD-TEA-TAX 17.3 ms vs AS-TAX 9.8 ms per image (Appendix, Table III)"}


def serving_entry(precision: str, horizon_s: float, loads=(100.0, 1000.0, 5000.0)) -> dict:
    """Continuous-batching server under Poisson arrivals: for each offered load, requests
    arrive over `horizon_s` seconds; batches are admitted until horizon + 2 s, after which
    the queued remainder counts as unserved and only batches in flight drain.  The mix is
    64/128/256-element arrays (128x256 / 256x512 / 512x1024 grids) at 20/40 MHz with records
    of 1024-16384 samples."""
    from paper_2412_02413_amd import serving as SV
    t = time.perf_counter()
    pool = SV.make_pool()
    log(f"serving pool of {len(pool)} frames in {time.perf_counter() - t:.1f} s")
    srv = SV.Server(max_batch=16, n_streams=4, precision=precision, hbm_budget=32 << 30)
    out = {"precision": precision, "horizon_s": horizon_s, "admission_deadline_s": horizon_s + 2.0,
           "max_batch": 16, "streams": 4, "hbm_budget_gib": 32,
           "mix": "64/128/256 elements x 20/40 MHz x 1024-16384 samples", "loads": []}
    try:
        srv.run(SV.poisson_requests(pool, 1e6, len(pool), seed=99), realtime=False)     # plans + warm-up
        for rate in loads:
            srv.batch_sizes.clear()
            srv.stats.clear()
            reqs = SV.poisson_requests(pool, rate, max(1, int(rate * horizon_s)), seed=int(rate))
            srv.run(reqs, deadline_s=horizon_s + 2.0)
            s = SV.summarize(reqs, rate)
            s["mean_batch"] = round(float(np.mean(srv.batch_sizes)), 2) if srv.batch_sizes else 0
            s["admission_stalls"] = srv.stats["admission_stalls"]
            out["loads"].append(s)
            log(f"serving: {s}")
    finally:
        srv.close()
    return out


def copy_calibration(dev, mib: int = 1024, reps: int = 3):
    """Plain device copies of a known size (outside any timed region): the per-dispatch
    FETCH_SIZE / WRITE_SIZE counters of these copies scale the fields kernel's counters."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    log(f"copy calibration: {reps} device copies of {mib} MiB")
    del src, dst


# ----------------------------------------------------------------------------

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--frames", type=int, default=64, help="frames per launch")
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--latency-calls", type=int, default=1000)
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle (accuracy check and CPU baseline)")
    ap.add_argument("--oracle-threads", type=int, default=7, help="BLAS threads of each of the two oracle processes")
    ap.add_argument("--variants", default="split_bf16,split_fp16,bf16,fp16",
                    help="other precision forms measured beside the main one (comma list, '' for none)")
    ap.add_argument("--surrogate", default=os.path.join(ROOT, "paper_2412_02413_amd", "weights",
                                                        "surrogate_l4_b32_coh.safetensors"),
                    help="surrogate weights measured beside plain AS-TAX ('' for none)")
    ap.add_argument("--no-paper-shape", dest="paper_shape", action="store_false",
                    help="skip the paper-shape (690 / 128 bins, 300 x 256) context timing")
    ap.add_argument("--no-mixed", dest="mixed", action="store_false", help="skip the mixed-record-length leg")
    ap.add_argument("--serving-horizon", type=float, default=1.5,
                    help="seconds of Poisson arrivals per offered load (0 skips the serving leg)")
    ap.add_argument("--no-evaluation", dest="evaluation", action="store_false",
                    help="skip the pattern-selection / resolution / uneven-strength harness")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="finish with plain device copies of 1 GiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); frames are independent, "
              "so a multi-GPU run would shard frames across devices with no exchange.", file=sys.stderr)
        sys.exit(2)

    # the oracle processes start before anything touches the GPU
    procs = start_oracles(args.oracle_threads) if not args.no_cpu_baseline else []

    import torch
    from paper_2412_02413_amd import pam, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    geom = synth.cfg2_geometry()
    F = args.frames
    t0 = time.perf_counter()
    rf_host = np.stack([synth.cfg2_frame(i)[0] for i in range(F)])
    log(f"generated {F} frames in {time.perf_counter() - t0:.1f} s")

    rf = torch.from_numpy(rf_host).to(dev)
    stream = torch.cuda.current_stream(dev)
    ev = pam.HipEvents()
    n_acc = min(ACC_FRAMES_BENCH, F)

    def measure(precision: str, latency_calls: int):
        """Throughput over `steps` launches, stage times from HIP events on the library's
        stream, optional single-frame latency; returns a dict with the first frames' outputs."""
        plan = pam.pam_plan(geom, 0, precision)
        image = torch.empty((F, geom.n_z, geom.n_x), device=dev)
        nncc = torch.empty_like(image)
        ws = pam.alloc_workspace(plan, F, geom.n_samples, dev)
        for _ in range(args.warmup):
            pam.pam_as_tax(plan, rf, image, nncc, None, ws, stream)
        torch.cuda.synchronize()
        events = [ev.create(pam.N_STAGE_EVENTS) for _ in range(args.steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            pam.pam_as_tax_events(plan, rf, image, events[k], nncc, None, ws, stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        stage_ms = {s: 0.0 for s in pam.STAGES}
        for k in range(args.steps):
            for i, s in enumerate(pam.STAGES):
                stage_ms[s] += ev.elapsed_ms(events[k][i], events[k][i + 1]) / args.steps
        lat_gpu, lat_wall, lat_graph = [], [], []
        if latency_calls > 0:
            img1 = torch.empty((1, geom.n_z, geom.n_x), device=dev)
            ws1 = pam.alloc_workspace(plan, 1, geom.n_samples, dev)
            e1 = ev.create(pam.N_STAGE_EVENTS)
            for c in range(latency_calls + 3):
                x = rf[c % F: c % F + 1]
                torch.cuda.synchronize()
                tw = time.perf_counter()
                pam.pam_as_tax_events(plan, x, img1, e1, None, None, ws1, stream)
                torch.cuda.synchronize()
                if c >= 3:
                    lat_wall.append(1e3 * (time.perf_counter() - tw))
                    lat_gpu.append(ev.elapsed_ms(e1[0], e1[-1]))
            # the same single-frame call replayed from a graph captured once on a side stream
            # (the library's launches only; each frame is copied into the captured input first,
            # outside the timed region)
            gs = torch.cuda.Stream(device=dev)
            x1 = rf[0:1].clone()
            img_g = torch.empty_like(img1)
            ws_g = pam.alloc_workspace(plan, 1, geom.n_samples, dev)
            with torch.cuda.stream(gs):
                pam.pam_as_tax(plan, x1, img_g, None, None, ws_g, gs)
            gs.synchronize()
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph, stream=gs):
                pam.pam_as_tax(plan, x1, img_g, None, None, ws_g, gs)
            torch.cuda.synchronize()
            for c in range(latency_calls + 3):
                x1.copy_(rf[c % F: c % F + 1])
                torch.cuda.synchronize()
                g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                with torch.cuda.stream(gs):
                    g0.record(gs)
                    graph.replay()
                    g1.record(gs)
                g1.synchronize()
                if c >= 3:
                    lat_graph.append(g0.elapsed_time(g1))
            del graph
        n_sel = plan.info.n_bins
        lay = pam.pam_workspace_layout(plan, F, geom.n_samples)
        pam.pam_destroy(plan)
        res = {"precision": precision, "ms_per_step": 1e3 * wall / args.steps,
               "frames_per_s": F * args.steps / wall, "stage_ms": stage_ms, "n_sel": n_sel,
               "lat_gpu": lat_gpu, "lat_wall": lat_wall, "lat_graph": lat_graph, "layout": lay, "images": image,
               "acc_images": image[:n_acc].cpu().numpy().astype(np.float64),
               "acc_nncc": nncc[:n_acc].cpu().numpy().astype(np.float64)}
        log(f"{precision}: {res['ms_per_step']:.2f} ms/step, {res['frames_per_s']:.1f} frames/s, "
            f"stages {stage_ms}")
        return res

    def fields_roofline(r, precision):
        k3_ms = r["stage_ms"]["fields"]
        alg = fields_algorithmic_flops(geom, r["n_sel"]) * F
        ach = alg / (k3_ms * 1e-3) / 1e12
        if precision == "fp32":
            # 16 x 16 FFT on the vector ALUs: no matrix-core work
            peak = VALU_FP32_PEAK_TFLOPS
            return {"kernel": "fields (propagator + 16 x 16 vector FFT + cross-spectra, k3fft)", "bound": "alu",
                    "achieved": round(ach, 3), "peak": peak, "unit": "TFLOP/s", "frac": round(ach / peak, 4),
                    "frac_of_unpacked_fp32": round(ach / VALU_FP32_UNPACKED_TFLOPS, 4),
                    "ms": round(k3_ms, 3), "algorithmic_flops_per_launch": alg}
        exe = executed_mfma_flops(geom, r["n_sel"], F, precision)
        peak = MFMA_PEAK_TFLOPS[precision]
        util = exe / (k3_ms * 1e-3) / 1e12
        return {"kernel": "fields (propagator + two-stage DFT-GEMM + cross-spectra, k3ff)", "bound": "mfma",
                "achieved": round(ach, 3), "peak": peak, "unit": "TFLOP/s", "frac": round(ach / peak, 4),
                "ms": round(k3_ms, 3), "algorithmic_flops_per_launch": alg,
                "mfma_executed_flops_per_launch": exe, "mfma_tflops": round(util, 2),
                "mfma_util": round(util / peak, 4)}

    main_res = measure(args.precision, args.latency_calls)
    fps, ms_per_step, stage_ms, n_sel = (main_res["frames_per_s"], main_res["ms_per_step"],
                                         main_res["stage_ms"], main_res["n_sel"])
    lat_gpu, lat_wall = main_res["lat_gpu"], main_res["lat_wall"]
    if lat_gpu:
        log(f"latency: p50 {np.percentile(lat_gpu, 50):.3f} ms p99 {np.percentile(lat_gpu, 99):.3f} ms (GPU); "
            f"graph replay p50 {np.percentile(main_res['lat_graph'], 50):.3f} p99 "
            f"{np.percentile(main_res['lat_graph'], 99):.3f} ms")
    roof = fields_roofline(main_res, args.precision)
    roof["traffic"] = recorded_traffic(args.precision)
    roof["algorithmic_bytes_per_launch"] = algorithmic_bytes(main_res["layout"], F, n_sel, geom)
    roof["traffic_unit"] = "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)"

    precisions = [args.precision] + [v for v in args.variants.split(",") if v and v != args.precision]
    variants, acc_out = {}, {args.precision: (main_res["acc_images"], main_res["acc_nncc"])}
    for prec in precisions[1:]:
        r = measure(prec, 0)
        acc_out[prec] = (r["acc_images"], r["acc_nncc"])
        rv = fields_roofline(r, prec)
        variants[prec] = {"frames_per_s": round(r["frames_per_s"], 2), "ms_per_step": round(r["ms_per_step"], 3),
                          "speedup_vs_plain": round(r["frames_per_s"] / fps, 3), "fields": rv}
        del r

    # the 64-element workload on the GPU (accuracy against the oracle)
    g1 = synth.cfg1_geometry()
    rf1 = np.stack([synth.cfg1_frame(s) for s in range(ACC_FRAMES_SMALL)])
    small_out = {p: run_frames(pam, torch, g1, rf1, p, dev) for p in precisions}

    mixed = None
    if args.mixed:
        mixed, mixed_first, mixed_groups = mixed_lengths(pam, torch, [p for p in precisions if p in
                                                                      ("fp32", "split_bf16", "split_fp16")],
                                                         max(3, args.steps // 4), dev)
        log(f"mixed record lengths: {mixed}")

    sur = None
    if args.surrogate:
        if os.path.exists(args.surrogate):
            sur = surrogate_entry(geom, rf, main_res["images"], fps, args.precision, args.steps, args.warmup,
                                  args.surrogate)
            log(f"surrogate: {sur}")
            if args.precision != "split_bf16":
                sur["with_split_bf16_propagation"] = surrogate_entry(
                    geom, rf, main_res["images"], fps, "split_bf16", args.steps, args.warmup, args.surrogate)
                log(f"surrogate, split BF16 propagation: {sur['with_split_bf16_propagation']}")
        else:
            log(f"surrogate weights not found at {args.surrogate}: no surrogate entry")
    fdt = fd_tea_entry(geom, rf, fps, max(2, args.steps // 10))
    log(f"FD-TEA-TAX: {fdt}")
    pcie = pcie_inclusive(geom, rf_host, args.precision, max(3, args.steps // 4), dev)
    log(f"with host copies: {pcie}")
    stages_roof = stage_rooflines(geom, n_sel, F, main_res["layout"], stage_ms)
    pshape = paper_shape([args.precision, "split_bf16"], 5, dev) if args.paper_shape else None
    if pshape:
        log(f"paper shape: {pshape}")
    serving = serving_entry(args.precision, args.serving_horizon) if args.serving_horizon > 0 else None
    evaluation = None
    if args.evaluation:
        from paper_2412_02413_amd import evaluate as EV
        t0 = time.perf_counter()
        evaluation = {"pattern_sweep": EV.pattern_sweep(n_frames=8, precision=args.precision),
                      "resolution": EV.resolution(n_frames=4, precision=args.precision),
                      "uneven_strength": EV.uneven_strength(n_frames=4, precision=args.precision)}
        log(f"evaluation harness in {time.perf_counter() - t0:.1f} s: chosen patterns "
            f"{[v['chosen_m'] for v in evaluation['pattern_sweep']['methods'].values()]}")
    if args.copy_calibration:
        copy_calibration(dev)
    ev.close()

    # accuracy against the oracle, then the oracle's own speed (nothing else running)
    accuracy, cpu = None, None
    if procs:
        t0 = time.perf_counter()
        ores = join_oracles(procs)
        log(f"oracle results after a further {time.perf_counter() - t0:.1f} s")
        accuracy = {}
        for prec in precisions:
            ent = {}
            if "bench" in ores:
                ent["benchmark_workload"] = errors_vs_oracle(acc_out[prec][0], acc_out[prec][1],
                                                             ores["bench"]["frames"])
            if "small" in ores:
                ent["small_workload"] = errors_vs_oracle(small_out[prec][0], small_out[prec][1],
                                                         ores["small"]["frames"])
                if mixed is not None and prec in mixed_first:
                    per = {}
                    for n_t, (s, I, rho) in ores["small"]["mixed"].items():
                        k = mixed_groups[n_t].index(s)
                        assert k == 0
                        img, rn = mixed_first[prec][n_t]
                        per[str(n_t)] = {"rel_l2_image": float(np.linalg.norm(img - I) / np.linalg.norm(I)),
                                         "max_abs_nncc": float(np.abs(rn - rho).max()), "seed": s}
                    ent["mixed_lengths_first_frame_per_length"] = per
            accuracy[prec] = ent
        log(f"accuracy: {json.dumps(accuracy)}")
        cpu = cpu_baseline(ores, 2 * args.oracle_threads)
        log(f"cpu baseline: {cpu}")

    rec = {
        "metric": METRIC,
        "value": round(fps, 2),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else args.precision,
        "data": "synthetic",
        "config": {"workload": "128 elements, 4096 samples at 40 MHz, 768 bins 0.5-8 MHz, "
                               "512x256 image, 3 sub-apertures (Pattern-16), 64 frames per launch",
                   "frames_per_step": F, "precision": args.precision, "parallelism": "none (1 GPU)"},
        "latency_ms_per_frame": ({"p50": round(float(np.percentile(lat_gpu, 50)), 4),
                                  "p99": round(float(np.percentile(lat_gpu, 99)), 4),
                                  "p99_host_wall": round(float(np.percentile(lat_wall, 99)), 4),
                                  "graph_p50": round(float(np.percentile(main_res["lat_graph"], 50)), 4),
                                  "graph_p99": round(float(np.percentile(main_res["lat_graph"], 99)), 4),
                                  "calls": len(lat_gpu), "frames_per_call": 1} if lat_gpu else None),
        "stage_ms_per_step": {k: round(v, 4) for k, v in stage_ms.items()},
        "stage_rooflines": stages_roof,
        "roofline": roof,
        "algorithmic_gflop_per_frame": round(algorithmic_flops(geom, n_sel) / 1e9, 3),
        "algorithmic_tflops": round(algorithmic_flops(geom, n_sel) * fps / 1e12, 3),
        "error_vs_oracle": accuracy,
        "cpu_baseline": cpu,
        "variants": variants,
        "mixed_record_lengths": mixed,
        "fd_tea_tax": fdt,
        "surrogate": sur,
        "pcie_inclusive": pcie,
        "paper_shape": pshape,
        "serving": serving,
        "evaluation": evaluation,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
