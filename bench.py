"""Benchmark of the AS-TAX hot path on one MI355X.

Workload (one step = one pam_as_tax call over a batch of 64 frames, inputs
resident in HBM): 128-element array, pitch 0.3 mm, 4096 samples at 40 MHz,
768 bins (0.5-8 MHz), image 512 depths x 256 columns, 3 stable + 2 inertial
emitters per frame at random positions, 20 dB channel noise (synthetic; the
paper's recordings are not available).

Prints ONE JSON line on stdout: throughput (frames/s), per-frame latency
p50/p99 of single-frame calls, the dominant kernel's roofline figures measured
live with HIP events on the library's stream, the error of the GPU result against
the FP64 oracle on one frame, and the oracle itself timed on the host CPU
(a reported baseline, not the target).  Beside the main form: the other precision
forms of the DFT-GEMM, and the NCC-mask surrogate (committed weights) on the same
frames, with its fallback rate and its image against plain AS-TAX's.
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
MFMA_PASSES = {"fp32": 1, "split_bf16": 3, "split_fp16": 3, "bf16": 1, "fp16": 1}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def executed_mfma_flops(geom, n_sel: int, n_frames: int, precision: str) -> float:
    """Matrix-core flops one launch of the fields kernel executes: per (frame, bin) a
    real GEMM of (2 n_sub * 32-padded depths) x N_x x N_x (folded real basis), times the
    number of product passes of the precision mode."""
    n_z_pad = 32 * math.ceil(geom.n_z / 32)
    return 2.0 * (2 * geom.n_sub) * n_z_pad * geom.n_x * geom.n_x * n_sel * n_frames * MFMA_PASSES[precision]


def algorithmic_flops(geom, n_sel: int) -> float:
    """FFT-equivalent work of one frame (5 N log2 N per complex FFT): lateral inverse FFTs,
    propagator products, 12 FMAs of cross-spectra per pixel and bin, time and lateral FFTs."""
    N, nz, ns = geom.n_x, geom.n_z, geom.n_sub
    lat_ifft = ns * n_sel * nz * 5 * N * math.log2(N)
    prop = ns * n_sel * nz * N * 6
    cross = n_sel * nz * N * 24
    t_fft = geom.n_elements * 5 * (geom.n_samples / 2) * math.log2(geom.n_samples / 2)
    lat_fft = ns * n_sel * 5 * N * math.log2(N)
    return lat_ifft + prop + cross + t_fft + lat_fft


def make_frames(n: int, base_seed: int = 0) -> np.ndarray:
    from paper_2412_02413_amd import synth
    return np.stack([synth.cfg2_frame(base_seed + i)[0] for i in range(n)])


def err(img, rho, ref):
    return {"rel_l2_image": float(np.linalg.norm(img - ref["I"]) / np.linalg.norm(ref["I"])),
            "max_abs_nncc": float(np.abs(rho - ref["rho_n"]).max()), "frames": 1}


def cpu_baseline(rf0: np.ndarray, geom):
    """FP64 oracle on one full cfg2 frame on the host cores."""
    from oracle import as_tax as O
    try:
        from threadpoolctl import threadpool_info
        threads = max([int(i.get("num_threads", 1)) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    t0 = time.perf_counter()
    ref = O.as_tax(rf0, geom)
    dt = time.perf_counter() - t0
    return ref, {"value": 1.0 / dt, "unit": "frames/s", "cores": threads, "kind": "oracle",
                 "sample": f"1 full frame of the benchmark workload (seed 0): {dt:.1f} s"}


def source_digest() -> str:
    """SHA-256 of the fields kernel's sources: traffic counters stay valid only for this code."""
    import hashlib
    h = hashlib.sha256()
    for name in ("kernels.hpp", "k3_fields.hpp", "k3_fields16.hpp", "k3_fields_fused.hpp"):
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


def algorithmic_bytes(lay, n_frames: int, n_sel: int, geom) -> float:
    """Bytes the fields kernel must move once per launch: the lateral coefficients of every
    (frame, bin, sub-aperture) in, the accumulated energy and cross-spectra sums out."""
    coeffs = n_frames * n_sel * geom.n_sub * geom.n_x * 8
    accum = lay.n_split * n_frames * lay.n_acc * geom.n_z * geom.n_x * 4
    return float(coeffs + accum)


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


def surrogate_entry(geom, rf, plain_images, fps_plain, precision, steps, warmup, path):
    """The NCC-mask surrogate (one full-aperture propagation + U-Net mask, confidence
    fallback to plain AS-TAX) on the same frames: throughput, fallback rate, and its image
    against plain AS-TAX's."""
    import torch
    from paper_2412_02413_amd import surrogate as S
    net, tau = S.UNet.from_weights(path)
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
    return {"frames_per_s": round(fps, 2), "ms_per_step": round(1e3 * wall / steps, 3),
            "speedup_vs_plain": round(fps / fps_plain, 3), "tau": round(tau, 4),
            "fallback_rate": round(fb / (F * steps), 4),
            "image_rel_l2_vs_plain_mean": round(float(rel.mean()), 4),
            "image_rel_l2_vs_plain_p95": round(float(rel.quantile(0.95)), 4),
            "abs_d_isnr_db_mean": round(float((isnr_s - isnr_p).abs().mean()), 3),
            "network": f"U-Net {net.levels} levels, {net.base} base channels, BF16 operands, FP32 accumulation",
            "weights": os.path.relpath(path, ROOT)}


def stage_rooflines(geom, n_sel: int, F: int, lay, stage_ms: dict) -> dict:
    """The smaller kernels against their own bounds, from the live stage times:
    K1 (time FFT) and K4 (NCC / weight / image) against HBM bandwidth by the bytes they
    must move, K2 (apodized lateral DFT) against the FP32 vector rate (non-packed FMA,
    78.6 TFLOP/s) by its direct-DFT flops."""
    pix = geom.n_z * geom.n_x
    plane = F * pix * 4
    k1_bytes = F * geom.n_elements * geom.n_samples * 4 + F * n_sel * geom.n_elements * 8
    # accumulators in, energy + weight out; weight + energy in, image + NNCC out
    k4_bytes = lay.n_split * lay.n_acc * plane + 2 * plane + 2 * plane + 2 * plane
    k2_flops = F * n_sel * geom.n_sub * geom.n_x * geom.n_elements * 8.0
    out = {}
    for name, key, amount, peak, unit, scale in (
            ("time_fft", "time_fft", k1_bytes, HBM_PEAK_GBS, "GB/s", 1e9),
            ("finalize", "finalize", k4_bytes, HBM_PEAK_GBS, "GB/s", 1e9),
            ("lateral", "lateral", k2_flops, 78.6, "TFLOP/s", 1e12)):
        ms = stage_ms[key]
        ach = amount / (ms * 1e-3) / scale
        out[name] = {"bound": "hbm" if unit == "GB/s" else "valu", "achieved": round(ach, 2), "peak": peak,
                     "unit": unit, "frac": round(ach / peak, 4), "per_launch": amount, "ms": round(ms, 4)}
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--frames", type=int, default=64, help="frames per launch")
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--latency-calls", type=int, default=1000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--variants", default="split_bf16,split_fp16,bf16,fp16",
                    help="other precision forms measured beside the main one (comma list, '' for none)")
    ap.add_argument("--surrogate", default=os.path.join(ROOT, "paper_2412_02413_amd", "weights",
                                                        "surrogate_l4_b32.safetensors"),
                    help="surrogate weights measured beside plain AS-TAX ('' for none)")
    ap.add_argument("--no-paper-shape", dest="paper_shape", action="store_false",
                    help="skip the paper-shape (690 / 128 bins, 300 x 256) context timing")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="finish with plain device copies of 1 GiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); frames are independent, "
              "so a multi-GPU run would shard frames across devices with no exchange.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2412_02413_amd import pam, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    geom = synth.cfg2_geometry()
    F = args.frames
    t0 = time.perf_counter()
    rf_host = make_frames(F)
    log(f"generated {F} frames in {time.perf_counter() - t0:.1f} s")

    rf = torch.from_numpy(rf_host).to(dev)
    stream = torch.cuda.current_stream(dev)
    ev = pam.HipEvents()

    def measure(precision: str, latency_calls: int):
        """Throughput over `steps` 64-frame launches, stage times from HIP events on the
        library's stream, optional single-frame latency; returns a dict and frame 0's output."""
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
        lat_gpu, lat_wall = [], []
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
        n_sel = plan.info.n_bins
        lay = pam.pam_workspace_layout(plan, F, geom.n_samples)
        pam.pam_destroy(plan)
        res = {"precision": precision, "ms_per_step": 1e3 * wall / args.steps,
               "frames_per_s": F * args.steps / wall, "stage_ms": stage_ms, "n_sel": n_sel,
               "lat_gpu": lat_gpu, "lat_wall": lat_wall, "layout": lay, "images": image}
        log(f"{precision}: {res['ms_per_step']:.2f} ms/step, {res['frames_per_s']:.1f} frames/s, "
            f"stages {stage_ms}")
        return res, image[0].cpu().numpy().astype(np.float64), nncc[0].cpu().numpy().astype(np.float64)

    main_res, img0, rho0 = measure(args.precision, args.latency_calls)
    fps, ms_per_step, stage_ms, n_sel = (main_res["frames_per_s"], main_res["ms_per_step"],
                                         main_res["stage_ms"], main_res["n_sel"])
    lat_gpu, lat_wall = main_res["lat_gpu"], main_res["lat_wall"]
    if lat_gpu:
        log(f"latency: p50 {np.percentile(lat_gpu, 50):.3f} ms p99 {np.percentile(lat_gpu, 99):.3f} ms (GPU)")

    # roofline of the dominant kernel (fields: propagate + DFT-GEMM + cross-spectra)
    k3_ms = stage_ms["fields"]
    flops = executed_mfma_flops(geom, n_sel, F, args.precision)
    achieved = flops / (k3_ms * 1e-3) / 1e12
    peak = MFMA_PEAK_TFLOPS[args.precision]
    alg = algorithmic_flops(geom, n_sel)
    traffic = recorded_traffic(args.precision)
    alg_bytes = algorithmic_bytes(main_res["layout"], F, n_sel, geom)

    # accuracy on frame 0 against the oracle, and the oracle's own speed on the host
    out = {}
    ref = None
    if not args.no_cpu_baseline:
        ref, cpu = cpu_baseline(rf_host[0], geom)
        out["error_vs_oracle"] = err(img0, rho0, ref)
        log(f"oracle: {cpu['sample']}; error {out['error_vs_oracle']}")
    else:
        cpu = None

    variants = {}
    for prec in [v for v in args.variants.split(",") if v and v != args.precision]:
        r, im, rh = measure(prec, 0)
        del r["images"]
        k3v = r["stage_ms"]["fields"]
        fl = executed_mfma_flops(geom, r["n_sel"], F, prec)
        variants[prec] = {"frames_per_s": round(r["frames_per_s"], 2), "ms_per_step": round(r["ms_per_step"], 3),
                          "speedup_vs_plain": round(r["frames_per_s"] / fps, 3),
                          "fields_ms": round(k3v, 3),
                          "mfma_tflops": round(fl / (k3v * 1e-3) / 1e12, 2), "mfma_peak": MFMA_PEAK_TFLOPS[prec],
                          "error_vs_oracle": err(im, rh, ref) if ref is not None else None}

    sur = None
    if args.surrogate:
        if os.path.exists(args.surrogate):
            sur = surrogate_entry(geom, rf, main_res["images"], fps, args.precision, args.steps, args.warmup,
                                  args.surrogate)
            log(f"surrogate: {sur}")
            if args.precision != "split_bf16":
                # the same network on a split-BF16 full-aperture propagation (fallback in split BF16)
                sur["with_split_bf16_propagation"] = surrogate_entry(
                    geom, rf, main_res["images"], fps, "split_bf16", args.steps, args.warmup, args.surrogate)
                log(f"surrogate, split BF16 propagation: {sur['with_split_bf16_propagation']}")
        else:
            log(f"surrogate weights not found at {args.surrogate}: no surrogate entry")
    pcie = pcie_inclusive(geom, rf_host, args.precision, max(3, args.steps // 4), dev)
    log(f"with host copies: {pcie}")
    stages_roof = stage_rooflines(geom, n_sel, F, main_res["layout"], stage_ms)
    pshape = paper_shape([args.precision, "split_bf16"], 5, dev) if args.paper_shape else None
    if pshape:
        log(f"paper shape: {pshape}")
    if args.copy_calibration:
        copy_calibration(dev)

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
                                  "calls": len(lat_gpu), "frames_per_call": 1} if lat_gpu else None),
        "stage_ms_per_step": {k: round(v, 4) for k, v in stage_ms.items()},
        "stage_rooflines": stages_roof,
        "roofline": {"kernel": "fields (propagate + DFT-GEMM + cross-spectra)", "bound": "mfma",
                     "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
                     "frac": round(achieved / peak, 4), "traffic": traffic,
                     "flops_per_launch": flops, "algorithmic_bytes_per_launch": alg_bytes,
                     "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)"},
        "algorithmic_gflop_per_frame": round(alg / 1e9, 3),
        "algorithmic_tflops": round(alg * fps / 1e12, 3),
        "cpu_baseline": cpu,
        "variants": variants,
        "surrogate": sur,
        "pcie_inclusive": pcie,
        "paper_shape": pshape,
    }
    rec.update(out)
    ev.close()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
