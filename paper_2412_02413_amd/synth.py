"""Seeded synthetic channel-RF generator and the imaging geometries it is used with.

This module is input generation only. It holds none of the reconstruction's
arithmetic (no bin selection, no apodization, no transforms of the method), so
both the HIP path and the FP64 oracle may take their inputs from it.

Physical setting (Section II-A, Fig. 1 of the paper): a linear array on the
plane z = 0 whose centre is the lateral origin; element l sits at
x_l = (l - (L-1)/2) * pitch.  Sources are points in the (x, z > 0) half plane;
each channel receives the source signal delayed by the exact geometric time of
flight r / c (unit amplitude, no 1/sqrt(r) spreading).

Workloads follow the paper's shapes (Section II-D: 128 elements, 2048 samples at
35.6 MHz, 3-15 MHz band, 300 x 256 image) and five synthetic configurations:

  cfg1  64 elements, pitch 0.3 mm, fs 20 MHz, c 1540 m/s, 1024 samples, one
        broadband emitter at (0, 30 mm), 20 dB channel noise; PAD to 128,
        depths 20-50 mm at 0.2 mm (151), band 1-5 MHz (205 bins).
  cfg2  128 elements, pitch 0.3 mm, fs 40 MHz, 4096 samples; 3 stable
        (harmonic) and 2 inertial (broadband burst) emitters at random
        positions; PAD to 256, depths 15.0 + 0.1 d mm (512), band 0.5-8 MHz
        (768 bins).
  cfg3  cfg1 geometry, record lengths drawn from {2048, 4096, 8192}, 1-10
        emitters of mixed type.
  cfg4  cfg1 array and band on a 256 x 512 grid (0.1 mm from 15 mm), 1-20
        emitters, SNR uniform in [0, 30] dB.
  cfg5  serving mix: 64/128/256 elements (pitch 0.3/0.3/0.2 mm), grids
        128x256 / 256x512 / 512x1024, fs 20 or 40 MHz, 1024-16384 samples.
  paper the paper's own shape: 128 elements, pitch 0.178 mm, fs 35.6 MHz,
        2048 samples, c 1500 m/s, 2x zero-stuffing to 256 columns, 300 depths
        at 0.2 mm, 3-15 MHz (690 bins).

Every draw comes from numpy's PCG64 seeded per frame, so a frame is a pure
function of (config, seed).
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

MM = 1e-3
MHZ = 1e6


@dataclass
class Geometry:
    """Plain description of one imaging set-up (mirrors pam_geometry_t)."""

    n_elements: int
    pitch_m: float
    fs_hz: float
    c_mps: float
    n_samples: int
    bands_hz: List[Tuple[float, float]]
    depths_m: np.ndarray
    n_x: int
    lateral: str = "pad"          # "pad" or "stuff"
    n_sub: int = 3
    pattern_m: int = 16
    apod: Optional[np.ndarray] = None   # explicit (n_sub, L) 0/1 masks, overrides pattern_m
    eps: float = 1e-3
    evanescent: str = "decay"     # "decay" or "zero"
    coherence: int = 0            # 1: adjacent-pixel cross-spectra with the full-aperture sums

    def replace(self, **kw) -> "Geometry":
        return dataclasses.replace(self, **kw)

    @property
    def n_z(self) -> int:
        return int(len(self.depths_m))

    def element_x(self) -> np.ndarray:
        L = self.n_elements
        return (np.arange(L) - (L - 1) / 2.0) * self.pitch_m


def _depths(z0_mm: float, dz_mm: float, n: int) -> np.ndarray:
    return (z0_mm + dz_mm * np.arange(n, dtype=np.float64)) * MM


def cfg1_geometry() -> Geometry:
    return Geometry(n_elements=64, pitch_m=0.3 * MM, fs_hz=20 * MHZ, c_mps=1540.0,
                    n_samples=1024, bands_hz=[(1 * MHZ, 5 * MHZ)],
                    depths_m=_depths(20.0, 0.2, 151), n_x=128, lateral="pad")


def cfg2_geometry() -> Geometry:
    return Geometry(n_elements=128, pitch_m=0.3 * MM, fs_hz=40 * MHZ, c_mps=1540.0,
                    n_samples=4096, bands_hz=[(0.5 * MHZ, 8 * MHZ)],
                    depths_m=_depths(15.0, 0.1, 512), n_x=256, lateral="pad")


def cfg3_geometry() -> Geometry:
    """cfg1 array and band; the plan serves records up to 8192 samples."""
    return cfg1_geometry().replace(n_samples=8192)


def cfg4_geometry() -> Geometry:
    return cfg1_geometry().replace(depths_m=_depths(15.0, 0.1, 512), n_x=256)


def paper_geometry(n_bins: int = 690) -> Geometry:
    """The paper's acquisition and image shape (Sections II-D and III-D).

    690 bins is the 3-15 MHz wideband set.  The 128-bin variant keeps a
    contiguous 128-bin band starting at 3 MHz (the paper's harmonic windows
    are not reproducible as 128 bins, so a plain band of that size stands in).
    """
    fs = 35.6 * MHZ
    n_t = 2048
    if n_bins == 690:
        bands = [(3 * MHZ, 15 * MHZ)]
    else:
        df = fs / n_t
        k0 = int(np.ceil(3 * MHZ / df))
        bands = [((k0 - 0.25) * df, (k0 + n_bins - 1 + 0.25) * df)]
    return Geometry(n_elements=128, pitch_m=0.178 * MM, fs_hz=fs, c_mps=1500.0,
                    n_samples=n_t, bands_hz=bands, depths_m=_depths(10.0, 0.2, 300),
                    n_x=256, lateral="stuff")


CFG5_ARRAYS = {
    64: dict(pitch_m=0.3 * MM, n_x=128, n_z=256),
    128: dict(pitch_m=0.3 * MM, n_x=256, n_z=512),
    256: dict(pitch_m=0.2 * MM, n_x=512, n_z=1024),
}


def cfg5_geometry(n_elements: int, fs_hz: float, n_samples: int) -> Geometry:
    a = CFG5_ARRAYS[n_elements]
    band = (1 * MHZ, 5 * MHZ) if fs_hz < 30 * MHZ else (0.5 * MHZ, 8 * MHZ)
    # depth grid spans roughly 15-66 mm whatever the row count
    dz = 51.2 / a["n_z"]
    return Geometry(n_elements=n_elements, pitch_m=a["pitch_m"], fs_hz=fs_hz, c_mps=1540.0,
                    n_samples=n_samples, bands_hz=[band], depths_m=_depths(15.0, dz, a["n_z"]),
                    n_x=a["n_x"], lateral="pad")


# ----------------------------------------------------------------------------
# Emitters
# ----------------------------------------------------------------------------

@dataclass
class Emitter:
    x_m: float
    z_m: float
    kind: str                  # "broadband", "stable" or "inertial"
    amplitude: float = 1.0
    params: dict = field(default_factory=dict)


def _delays(geom: Geometry, em: Emitter) -> np.ndarray:
    xl = geom.element_x()
    return np.sqrt((xl - em.x_m) ** 2 + em.z_m ** 2) / geom.c_mps


def _band_mask(n: int, fs: float, lo: float, hi: float) -> np.ndarray:
    f = np.arange(n // 2 + 1) * fs / n
    return (f >= lo) & (f <= hi)


def _delay_periodic(spec: np.ndarray, n: int, fs: float, tau: np.ndarray) -> np.ndarray:
    """Delay a one-sided spectrum by tau (per channel) with a phase ramp; real output."""
    f = np.arange(n // 2 + 1) * fs / n
    ramp = np.exp(-2j * np.pi * f[None, :] * tau[:, None])
    return np.fft.irfft(spec[None, :] * ramp, n=n, axis=1)


def _broadband_periodic(geom: Geometry, em: Emitter, rng: np.random.Generator,
                        n_t: int, band: Tuple[float, float]) -> np.ndarray:
    """Periodic band-limited Gaussian noise, delayed exactly per channel."""
    fs = geom.fs_hz
    m = _band_mask(n_t, fs, *band)
    spec = np.zeros(n_t // 2 + 1, np.complex128)
    nb = int(m.sum())
    spec[m] = rng.standard_normal(nb) + 1j * rng.standard_normal(nb)
    sig = _delay_periodic(spec, n_t, fs, _delays(geom, em))
    rms = np.sqrt(np.mean(sig ** 2))
    return em.amplitude * sig / max(rms, 1e-300)


def _stable(geom: Geometry, em: Emitter, rng: np.random.Generator, n_t: int,
            f_max: float) -> np.ndarray:
    """Harmonics of a jittered 1.5 MHz fundamental, evaluated at t - tau_l."""
    f0 = 1.5 * MHZ * (1.0 + 0.001 * rng.standard_normal())
    n_h = int(np.floor(f_max / (1.5 * MHZ)))
    a = 1.0 + rng.uniform(-0.05, 0.05, n_h)
    ph = rng.uniform(0, 2 * np.pi, n_h)
    t = np.arange(n_t) / geom.fs_hz
    tau = _delays(geom, em)
    sig = np.zeros((geom.n_elements, n_t))
    for h in range(n_h):
        sig += a[h] * np.cos(2 * np.pi * (h + 1) * f0 * (t[None, :] - tau[:, None]) + ph[h])
    rms = np.sqrt(np.mean(sig ** 2))
    return em.amplitude * sig / max(rms, 1e-300)


def _inertial(geom: Geometry, em: Emitter, rng: np.random.Generator, n_t: int,
              band: Tuple[float, float]) -> np.ndarray:
    """Band-limited noise burst of 2-20 us, delayed on a 2x padded record then cropped."""
    fs = geom.fs_hz
    n2 = 2 * n_t
    dur = rng.uniform(2e-6, 20e-6)
    n_on = max(1, int(round(dur * fs)))
    tau = _delays(geom, em)
    span = n_t - n_on - int(np.ceil((tau.max() - tau.min()) * fs)) - 1
    start = int(rng.integers(0, max(span, 1)))
    x = np.zeros(n2)
    x[start:start + n_on] = rng.standard_normal(n_on)
    X = np.fft.rfft(x)
    X[~_band_mask(n2, fs, *band)] = 0.0
    sig = _delay_periodic(X, n2, fs, tau - tau.min())[:, :n_t]
    act = sig[:, start:start + n_on]
    rms = np.sqrt(np.mean(act ** 2)) if act.size else 1.0
    return em.amplitude * sig / max(rms, 1e-300)


def _add_noise(sig: np.ndarray, snr_db: Optional[float], rng: np.random.Generator) -> np.ndarray:
    if snr_db is None:
        return sig
    p_sig = np.mean(sig ** 2)
    p_noise = p_sig / (10.0 ** (snr_db / 10.0))
    return sig + rng.standard_normal(sig.shape) * np.sqrt(p_noise)


def render(geom: Geometry, emitters: Sequence[Emitter], rng: np.random.Generator,
           n_t: Optional[int] = None, snr_db: Optional[float] = 20.0,
           band: Optional[Tuple[float, float]] = None) -> np.ndarray:
    """Sum of emitter signals at each element plus white channel noise -> float32 [L][n_t]."""
    n_t = geom.n_samples if n_t is None else n_t
    band = geom.bands_hz[0] if band is None else band
    sig = np.zeros((geom.n_elements, n_t))
    for em in emitters:
        if em.kind == "broadband":
            sig += _broadband_periodic(geom, em, rng, n_t, band)
        elif em.kind == "stable":
            sig += _stable(geom, em, rng, n_t, band[1])
        elif em.kind == "inertial":
            sig += _inertial(geom, em, rng, n_t, band)
        else:
            raise ValueError(em.kind)
    return _add_noise(sig, snr_db, rng).astype(np.float32)


def _random_emitters(rng, n, x_rng_mm, z_rng_mm, kinds):
    out = []
    for i in range(n):
        out.append(Emitter(x_m=rng.uniform(*x_rng_mm) * MM, z_m=rng.uniform(*z_rng_mm) * MM,
                           kind=kinds[i] if i < len(kinds) else rng.choice(["stable", "inertial"])))
    return out


# ----------------------------------------------------------------------------
# Per-config frame generators: frame = f(config, seed)
# ----------------------------------------------------------------------------

def cfg1_frame(seed: int, snr_db: Optional[float] = 20.0,
               source_mm: Tuple[float, float] = (0.0, 30.0)) -> np.ndarray:
    g = cfg1_geometry()
    rng = np.random.default_rng(seed)
    em = [Emitter(source_mm[0] * MM, source_mm[1] * MM, "broadband")]
    return render(g, em, rng, snr_db=snr_db)


def coherent_pair_frame(seed: int, x_mm: float = 5.0, z_mm: float = 40.0, ratio: float = 2.0,
                        snr_db: Optional[float] = 15.0, geom: Optional[Geometry] = None) -> np.ndarray:
    """Two sources at (-x, z) and (+x, z) radiating the same broadband waveform with
    amplitudes 1 : ratio (same phase, uneven strength), cfg1 array by default."""
    g = cfg1_geometry() if geom is None else geom
    rng = np.random.default_rng(seed)
    n_t = g.n_samples
    m = _band_mask(n_t, g.fs_hz, *g.bands_hz[0])
    spec = np.zeros(n_t // 2 + 1, np.complex128)
    spec[m] = rng.standard_normal(int(m.sum())) + 1j * rng.standard_normal(int(m.sum()))
    sig = np.zeros((g.n_elements, n_t))
    for amp, xs in ((1.0, -x_mm), (ratio, x_mm)):
        em = Emitter(xs * MM, z_mm * MM, "broadband")
        sig += amp * _delay_periodic(spec, n_t, g.fs_hz, _delays(g, em))
    return _add_noise(sig, snr_db, rng).astype(np.float32)


def cfg2_frame(seed: int, snr_db: Optional[float] = 20.0) -> Tuple[np.ndarray, List[Emitter]]:
    g = cfg2_geometry()
    rng = np.random.default_rng(seed)
    em = _random_emitters(rng, 5, (-15, 15), (20, 60), ["stable"] * 3 + ["inertial"] * 2)
    return render(g, em, rng, snr_db=snr_db), em


def cfg3_frame(seed: int) -> np.ndarray:
    g = cfg3_geometry()
    rng = np.random.default_rng(seed)
    n_t = int(rng.choice([2048, 4096, 8192]))
    n_em = int(rng.integers(1, 11))
    em = _random_emitters(rng, n_em, (-9, 9), (20, 50), [])
    return render(g, em, rng, n_t=n_t, snr_db=20.0)


def cfg4_frame(seed: int) -> Tuple[np.ndarray, List[Emitter]]:
    g = cfg4_geometry()
    rng = np.random.default_rng(seed)
    n_em = int(rng.integers(1, 21))
    em = _random_emitters(rng, n_em, (-9, 9), (18, 64), [])
    snr = float(rng.uniform(0.0, 30.0))
    return render(g, em, rng, snr_db=snr), em


def cfg5_request(seed: int) -> Tuple[Geometry, np.ndarray]:
    rng = np.random.default_rng(seed)
    L = int(rng.choice([64, 128, 256]))
    fs = float(rng.choice([20 * MHZ, 40 * MHZ]))
    n_t = int(2 ** rng.integers(10, 15))
    g = cfg5_geometry(L, fs, n_t)
    half = L * g.pitch_m / 2 / MM
    em = _random_emitters(rng, int(rng.integers(1, 6)), (-0.8 * half, 0.8 * half), (20, 60), [])
    return g, render(g, em, rng, snr_db=20.0)


def paper_frame(seed: int, n_bins: int = 690) -> np.ndarray:
    g = paper_geometry(n_bins)
    rng = np.random.default_rng(seed)
    em = [Emitter(0.0, 40 * MM, "stable"), Emitter(-3 * MM, 35 * MM, "inertial")]
    return render(g, em, rng, band=(3 * MHZ, 15 * MHZ), snr_db=20.0)


def tunnel_frame(seed: int, geom: Optional[Geometry] = None, snr_db: Optional[float] = 20.0,
                 z_mm: float = 40.0, half_width_mm: float = 2.5, diameter_mm: float = 5.0,
                 n_sources: int = 6) -> Tuple[np.ndarray, List[Emitter]]:
    """Cavitation in a tunnel lying in the image plane (stand-in for a wall-less flow phantom
    imaged with the array parallel to the tunnel): stable and inertial emitters inside the
    tunnel's cross-section under the focal region, |x| <= half_width, |z - z_mm| <= d/2.
    Paper-shape array by default."""
    g = paper_geometry(690) if geom is None else geom
    rng = np.random.default_rng(seed)
    em = [Emitter(rng.uniform(-half_width_mm, half_width_mm) * MM,
                  (z_mm + rng.uniform(-diameter_mm / 2, diameter_mm / 2)) * MM,
                  str(rng.choice(["stable", "inertial"])))
          for _ in range(n_sources)]
    return render(g, em, rng, snr_db=snr_db), em


def bubble_pair_frame(seed: int, p1_mm: Tuple[float, float], p2_mm: Tuple[float, float],
                      geom: Optional[Geometry] = None, snr_db: Optional[float] = 20.0,
                      f_drive_hz: float = 1.0 * MHZ, f_centre_hz: float = 8.9 * MHZ,
                      frac_bw: float = 0.67) -> np.ndarray:
    """Two bubbles driven by one excitation (stand-in for the Marmottant-model pair of the
    resolution appendix): each radiates harmonics of the drive frequency inside the
    geometry's band with its own random amplitudes and phases (slightly different bubble
    sizes), delayed exactly per channel and shaped by a Gaussian receive response of the
    array (centre 8.9 MHz, 67 % fractional bandwidth at half amplitude, the CL15-7 figures
    the appendix states).  Paper-shape array by default."""
    g = paper_geometry(690) if geom is None else geom
    rng = np.random.default_rng(seed)
    n_t = g.n_samples
    lo, hi = g.bands_hz[0]
    t = np.arange(n_t) / g.fs_hz
    sig = np.zeros((g.n_elements, n_t))
    hs = [h for h in range(1, int(hi // f_drive_hz) + 1) if lo <= h * f_drive_hz <= hi]
    sigma = frac_bw * f_centre_hz / 2.0 / np.sqrt(2.0 * np.log(2.0))
    resp = np.exp(-((np.array(hs, float) * f_drive_hz - f_centre_hz) ** 2) / (2.0 * sigma ** 2))
    for (x, z) in (p1_mm, p2_mm):
        tau = _delays(g, Emitter(x * MM, z * MM, "stable"))
        amp = resp * rng.uniform(0.5, 1.0, len(hs))
        ph = rng.uniform(0, 2 * np.pi, len(hs))
        for a, p_, h in zip(amp, ph, hs):
            sig += a * np.cos(2 * np.pi * h * f_drive_hz * (t[None, :] - tau[:, None]) + p_)
    return _add_noise(sig, snr_db, rng).astype(np.float32)


def batch(gen, seeds: Sequence[int]) -> np.ndarray:
    frames = []
    for s in seeds:
        r = gen(s)
        frames.append(r[0] if isinstance(r, tuple) else r)
    return np.stack(frames)
