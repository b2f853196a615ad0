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
(a reported baseline, not the target).  Diagnostics go to stderr.
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--frames", type=int, default=64, help="frames per launch")
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--latency-calls", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--variants", default="split_bf16,split_fp16,bf16,fp16",
                    help="other precision forms measured beside the main one (comma list, '' for none)")
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
        pam.pam_destroy(plan)
        res = {"precision": precision, "ms_per_step": 1e3 * wall / args.steps,
               "frames_per_s": F * args.steps / wall, "stage_ms": stage_ms, "n_sel": n_sel,
               "lat_gpu": lat_gpu, "lat_wall": lat_wall}
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
        k3v = r["stage_ms"]["fields"]
        fl = executed_mfma_flops(geom, r["n_sel"], F, prec)
        variants[prec] = {"frames_per_s": round(r["frames_per_s"], 2), "ms_per_step": round(r["ms_per_step"], 3),
                          "speedup_vs_plain": round(r["frames_per_s"] / fps, 3),
                          "fields_ms": round(k3v, 3),
                          "mfma_tflops": round(fl / (k3v * 1e-3) / 1e12, 2), "mfma_peak": MFMA_PEAK_TFLOPS[prec],
                          "error_vs_oracle": err(im, rh, ref) if ref is not None else None}

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
        "roofline": {"kernel": "fields (propagate + DFT-GEMM + cross-spectra)", "bound": "mfma",
                     "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
                     "frac": round(achieved / peak, 4), "traffic": None,
                     "flops_per_launch": flops},
        "algorithmic_gflop_per_frame": round(alg / 1e9, 3),
        "algorithmic_tflops": round(alg * fps / 1e12, 3),
        "cpu_baseline": cpu,
        "variants": variants,
    }
    rec.update(out)
    ev.close()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
