"""Evaluation harness on the HIP path: apodization-pattern selection, two-source
resolution and uneven source strength.

Every image comes from the library (pam_as_tax through the binding); this module only
builds the inputs, post-processes the images on the host and tabulates:

* pattern_sweep - Pattern-m (m = 2..32) for AS-DAX and AS-TAX on frames of a cavitating
  tunnel (the selection experiment of Section III-A): image SNR (Eq. 12), energy spread
  area (A_0.5) and the centroid of the NNCC map above 0.9 (Eq. 13 with rho_n in place of
  I), its axial distance from the frame's mean source depth, and the pattern chosen by the
  rule "highest ISNR among the patterns whose NNCC centroid lies within `tol_mm` of the
  reference depth"
  (Section III-A picks Pattern-16 on the same two criteria);
* resolution - two bubbles 0.35 mm apart laterally and 4 mm apart axially (Appendix,
  "Spatial resolution"): the depth of the trough of the profile through the two
  sources, relative to the lower of the two peaks, for AS, AS-DAX and AS-TAX; Rayleigh's
  criterion resolves them when the trough is at least 26.3 % below the peak;
* uneven_strength - two coherent sources at (+-5 mm, 40 mm) with amplitudes 1 : 2 (Appendix,
  "Noise and uneven cavitation strength") at several SNRs: the regional peak intensity of
  each source for AS, AS-TAX and AS^3 (the AS image weighted by its own normalised square),
  all normalised to the maximum of the AS image.

Inputs are synthetic (synth.tunnel_frame, synth.bubble_pair_frame,
synth.coherent_pair_frame): the paper's phantom recordings and k-Wave / Marmottant
simulations are not available.
"""
from __future__ import annotations

import argparse
import json
import sys
from typing import Dict, Sequence

import numpy as np

from . import pam, synth

MM = 1e-3
RAYLEIGH_DIP = 0.263


# ----------------------------------------------------------------------------
# image metrics (Section II-E)
# ----------------------------------------------------------------------------

def a05(I: np.ndarray) -> np.ndarray:
    """A_0.5: pixels strictly above half the image maximum."""
    return I > 0.5 * I.max()


def esa_mm2(I: np.ndarray, dx_m: float, dz_m: float) -> float:
    return float(np.count_nonzero(a05(I)) * dx_m * dz_m / MM ** 2)


def isnr_db(I: np.ndarray) -> float:
    """Eq. 12: mean inside A_0.5 over mean outside, in dB."""
    m = a05(I)
    return float(10.0 * np.log10(I[m].mean() / I[~m].mean()))


def centroid(I: np.ndarray, x: np.ndarray, z: np.ndarray, alpha: float):
    """Eq. 13: intensity-weighted centroid (x, z) of the pixels above alpha times the maximum."""
    m = I > alpha * I.max()
    w = I[m]
    Z, X = np.meshgrid(z, x, indexing="ij")
    return float(np.sum(w * X[m]) / w.sum()), float(np.sum(w * Z[m]) / w.sum())


def grid_x(geom) -> np.ndarray:
    """Lateral coordinates of the image columns (array centre at x = 0)."""
    L, N = geom.n_elements, geom.n_x
    if geom.lateral == "pad":
        o, dx = (N - L) // 2, geom.pitch_m
        centre = o + (L - 1) / 2.0
    else:
        s = N // L
        dx, centre = geom.pitch_m / s, s * (L - 1) / 2.0
    return (np.arange(N) - centre) * dx


# ----------------------------------------------------------------------------
# running the library
# ----------------------------------------------------------------------------

def reconstruct(geom, rf: np.ndarray, precision: str = "fp32", batch: int = 16):
    """Images and NNCC maps of host frames [F][L][n_t] through pam_as_tax."""
    import torch
    plan = pam.pam_plan(geom, 0, precision)
    try:
        imgs, nnccs = [], []
        for b0 in range(0, rf.shape[0], batch):
            x = torch.from_numpy(np.ascontiguousarray(rf[b0:b0 + batch], np.float32)).cuda()
            out = pam.reconstruct(plan, x, want_nncc=True)
            torch.cuda.synchronize()
            imgs.append(out["image"].cpu().numpy().astype(np.float64))
            nnccs.append(out["nncc"].cpu().numpy().astype(np.float64))
        return np.concatenate(imgs), np.concatenate(nnccs)
    finally:
        pam.pam_destroy(plan)


# ----------------------------------------------------------------------------
# Section III-A: selection of the apodization pattern
# ----------------------------------------------------------------------------

def pattern_sweep(n_frames: int = 16, ms: Sequence[int] = (2, 4, 8, 16, 32), z_ref_mm: float = 40.0,
                  tol_mm: float = 1.0, precision: str = "fp32", seed0: int = 0) -> Dict:
    g0 = synth.paper_geometry(690)
    scenes = [synth.tunnel_frame(seed0 + s, g0, z_mm=z_ref_mm) for s in range(n_frames)]
    rf = np.stack([sc[0] for sc in scenes])
    # reference depth of each frame: the mean depth of its emitters (the tunnel's sources)
    z_true = np.array([np.mean([e.z_m for e in sc[1]]) / MM for sc in scenes])
    x, z = grid_x(g0), np.asarray(g0.depths_m)
    dx, dz = x[1] - x[0], z[1] - z[0]
    out = {"frames": n_frames, "tunnel_depth_mm": z_ref_mm, "rule_tolerance_mm": tol_mm,
           "reference": "mean emitter depth of each frame",
           "scene": "6 stable/inertial emitters in a 5 mm tunnel at 40 mm depth, |x| <= 2.5 mm, 20 dB; "
                    "128 elements, 0.178 mm pitch, 35.6 MHz, 2048 samples, 690 bins, 2x stuffing, 300 x 256",
           "methods": {}}
    for name, n_sub in (("AS-DAX", 2), ("AS-TAX", 3)):
        rows = []
        for m in ms:
            g = g0.replace(n_sub=n_sub, pattern_m=m)
            I, rho = reconstruct(g, rf, precision)
            isnr = [isnr_db(I[f]) for f in range(n_frames)]
            esa = [esa_mm2(I[f], dx, dz) for f in range(n_frames)]
            cz = [centroid(rho[f], x, z, 0.9)[1] / MM for f in range(n_frames)]
            rows.append({"m": m, "isnr_db_mean": round(float(np.mean(isnr)), 3),
                         "isnr_db_std": round(float(np.std(isnr)), 3),
                         "esa_mm2_mean": round(float(np.mean(esa)), 4),
                         "nncc_centroid_z_mm_mean": round(float(np.mean(cz)), 3),
                         "nncc_centroid_abs_err_mm_mean": round(float(np.mean(np.abs(np.array(cz) - z_true))), 3)})
        ok = [r for r in rows if r["nncc_centroid_abs_err_mm_mean"] <= tol_mm]
        chosen = max(ok, key=lambda r: r["isnr_db_mean"])["m"] if ok else None
        out["methods"][name] = {"patterns": rows, "chosen_m": chosen}
    return out


# ----------------------------------------------------------------------------
# Appendix: spatial resolution (Rayleigh's criterion)
# ----------------------------------------------------------------------------

def profile_dip(I: np.ndarray, x: np.ndarray, z: np.ndarray, p1_mm, p2_mm, search_mm: float = 0.5) -> Dict:
    """Trough depth of the profile through two sources: the peak of each source is the
    profile maximum within `search_mm` of its true position, on its own side of the
    midpoint, the trough the profile minimum between the two peaks, and the dip
    1 - trough / min(peak1, peak2)."""
    (x1, z1), (x2, z2) = p1_mm, p2_mm
    search_mm = min(search_mm, 0.5 * max(abs(x2 - x1), abs(z2 - z1)))
    lateral = abs(z1 - z2) < 1e-9
    if lateral:
        d = int(np.argmin(np.abs(z / MM - z1)))
        prof, coord, a, b = I[d, :], x / MM, x1, x2
    else:
        j = int(np.argmin(np.abs(x / MM - x1)))
        prof, coord, a, b = I[:, j], z / MM, z1, z2

    mid = 0.5 * (a + b)

    def peak(c):
        sel = np.where((np.abs(coord - c) <= search_mm) & ((coord - mid) * (c - mid) > 0))[0]
        k = sel[np.argmax(prof[sel])]
        return k, prof[k]

    (k1, v1), (k2, v2) = peak(a), peak(b)
    lo, hi = sorted((k1, k2))
    trough = float(prof[lo:hi + 1].min()) if hi > lo else float(min(v1, v2))
    dip = 1.0 - trough / float(min(v1, v2))
    return {"dip": round(dip, 4), "resolved": bool(dip >= RAYLEIGH_DIP),
            "peak_positions_mm": [round(float(coord[k1]), 4), round(float(coord[k2]), 4)]}


def resolution(n_frames: int = 8, precision: str = "fp32") -> Dict:
    g0 = synth.paper_geometry(690)
    x, z = grid_x(g0), np.asarray(g0.depths_m)
    cases = {"lateral": ((-0.175, 40.0), (0.175, 40.0)), "axial": ((0.0, 38.0), (0.0, 42.0))}
    out = {"frames": n_frames, "rayleigh_dip": RAYLEIGH_DIP,
           "scene": "two bubbles radiating harmonics of a 1 MHz drive (3-15 MHz band), 20 dB; paper-shape array",
           "cases": {}}
    for cname, (p1, p2) in cases.items():
        rf = np.stack([synth.bubble_pair_frame(100 + s, p1, p2, g0) for s in range(n_frames)])
        res = {}
        for name, n_sub in (("AS", 1), ("AS-DAX", 2), ("AS-TAX", 3)):
            I, _ = reconstruct(g0.replace(n_sub=n_sub), rf, precision)
            dips = [profile_dip(I[f], x, z, p1, p2)["dip"] for f in range(n_frames)]
            res[name] = {"dip_mean": round(float(np.mean(dips)), 4), "dip_std": round(float(np.std(dips)), 4),
                         "resolved_fraction": round(float(np.mean([d >= RAYLEIGH_DIP for d in dips])), 3)}
        out["cases"][cname] = {"sources_mm": [p1, p2], **res}
    return out


# ----------------------------------------------------------------------------
# Appendix: noise and uneven cavitation strength
# ----------------------------------------------------------------------------

def regional_peaks(I: np.ndarray, x: np.ndarray, z: np.ndarray, p1_mm, p2_mm, half_mm: float = 2.0):
    """Regional peak intensity: the local maximum within +-half_mm of each source."""
    out = []
    for (xs, zs) in (p1_mm, p2_mm):
        cols = np.abs(x / MM - xs) <= half_mm
        rows = np.abs(z / MM - zs) <= half_mm
        out.append(float(I[np.ix_(rows, cols)].max()))
    return out


def uneven_strength(snrs_db: Sequence[float] = (15.0, 10.0, 5.0, -5.0), n_frames: int = 8,
                    precision: str = "fp32") -> Dict:
    g0 = synth.paper_geometry(690)
    x, z = grid_x(g0), np.asarray(g0.depths_m)
    p1, p2 = (-5.0, 40.0), (5.0, 40.0)
    out = {"frames": n_frames, "sources_mm": [p1, p2], "amplitudes": [1.0, 2.0],
           "scene": "one broadband waveform (3-15 MHz) from both sources, same phase, amplitudes 1 : 2; "
                    "paper-shape array", "snr": {}}
    for snr in snrs_db:
        rf = np.stack([synth.coherent_pair_frame(200 + s, 5.0, 40.0, 2.0, snr, geom=g0) for s in range(n_frames)])
        I_as, _ = reconstruct(g0.replace(n_sub=1), rf, precision)
        I_tax, _ = reconstruct(g0.replace(n_sub=3), rf, precision)
        rpi = {"AS": [], "AS-TAX": [], "AS^3": []}
        for f in range(n_frames):
            ref = I_as[f].max()
            as3 = (I_as[f] / ref) ** 2 * I_as[f]
            for name, img in (("AS", I_as[f]), ("AS-TAX", I_tax[f]), ("AS^3", as3)):
                rpi[name].append(regional_peaks(img / ref, x, z, p1, p2))
        out["snr"][str(snr)] = {k: {"rpi_weak_mean": round(float(np.mean([v[0] for v in vals])), 4),
                                    "rpi_strong_mean": round(float(np.mean([v[1] for v in vals])), 4)}
                                for k, vals in rpi.items()}
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description="Pattern selection, resolution and uneven-strength evaluation")
    ap.add_argument("--frames", type=int, default=16)
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--only", default="sweep,resolution,uneven")
    args = ap.parse_args(argv)
    want = set(args.only.split(","))
    out = {}
    if "sweep" in want:
        out["pattern_sweep"] = pattern_sweep(args.frames, precision=args.precision)
    if "resolution" in want:
        out["resolution"] = resolution(max(2, args.frames // 2), args.precision)
    if "uneven" in want:
        out["uneven_strength"] = uneven_strength(n_frames=max(2, args.frames // 2), precision=args.precision)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    sys.exit(main())
