"""FP64 CPU oracle for the cross-correlated angular-spectrum (AS-TAX) reconstruction.

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite, the package smoke
check and the CPU-baseline leg of the benchmark may import or run anything in
this directory.  It shares no code with the HIP path: every table (frequency
bins, apodization masks, lateral grid, wavenumbers, DFT matrices, propagators)
is rebuilt here from the paper's definitions.

Plain, slow and direct: every transform is a dense DFT written out as a matrix
product in complex128, with twiddle arguments taken from exact integer products
reduced modulo the transform length.  Nothing is blocked, folded or fused beyond
chunking over frequency bins to bound memory.

Steps (paper Section II-A unless noted; equation numbers are the paper's):
  O1 bins        frequency set Omega: bins 0 < k < n_t/2 whose frequency lies in a
                 closed band (Eq. 3's Omega; the wideband 3-15 MHz set of Section
                 II-E has 690 bins at 2048 samples and 35.6 MHz).
  O2 time DFT    F_t of each channel (Eq. 1), forward kernel exp(-i w t).
  O3 placement   apodize (Pattern-m, Sections II-A and II-C) and place on the
                 lateral grid: centred zero padding, or s-fold zero-stuffing
                 (Section II-E) with the apodization indexed on physical elements.
  O4 lateral DFT F_x of each sub-aperture (Eq. 1).
  O5 propagator  exp(i z sqrt(w^2/c^2 - kx^2)) from the array plane (Eq. 2),
                 principal square root (evanescent components decay).
  O6 inverse     inverse lateral DFT with the 1/N factor -> monochromatic fields.
  O7 sums        S_i = sum_w |p_i|^2, C_ij = sum_w Re(conj(p_i) p_j) (Eq. 4 with the
                 negative frequencies taken as conjugates, Appendix A), and
                 E = sum_w |p_1 + p_2 + p_3|^2 (Eq. 11).
  O8 NCC         rho_ij = C_ij / (sqrt(S_i) sqrt(S_j)), floored at eps (Eq. 4 text),
                 capped at 1; TAX weight = cube root of the product of the three
                 pairs (Eq. 10); DAX (n = 2) uses the single pair; plain AS (n = 1)
                 has weight 1.
  O9 normalize   rho_n = weight / its maximum over the image (NNCC, Section II-A),
                 image I = rho_n^2 * E (Eq. 11 / Eq. 5).

Every function's output is pinned in tests/test_oracle.py against facts that do
not come from this file (printed examples, library FFTs, closed forms,
invariants, brute force).
"""
from __future__ import annotations

from typing import Dict, Optional, Sequence, Tuple

import numpy as np

TWO_PI = 2.0 * np.pi


# ----------------------------------------------------------------------------
# O1  frequency bins
# ----------------------------------------------------------------------------

def bins(fs_hz: float, n_t: int, bands_hz: Sequence[Tuple[float, float]]) -> np.ndarray:
    """Bins k, 0 < k < n_t/2, with lo <= k*fs/n_t <= hi for some band (Eq. 3's Omega).

    DC and Nyquist are excluded; band edges are closed.
    """
    out = []
    for k in range(1, (n_t + 1) // 2):
        f = (k * fs_hz) / n_t
        if any(lo <= f <= hi for lo, hi in bands_hz):
            out.append(k)
    return np.asarray(out, dtype=np.int64)


# ----------------------------------------------------------------------------
# O2  time DFT (Eq. 1, F_t)
# ----------------------------------------------------------------------------

def time_dft(rf: np.ndarray, ks: np.ndarray) -> np.ndarray:
    """X[l, b] = sum_n s[l, n] exp(-2 pi i ((k_b n) mod n_t) / n_t), complex128 [L][n_bins]."""
    s = np.asarray(rf, dtype=np.float64)
    n_t = s.shape[-1]
    n = np.arange(n_t, dtype=np.int64)
    idx = (ks[None, :].astype(np.int64) * n[:, None]) % n_t          # [n_t][n_bins]
    W = np.exp(-1j * TWO_PI * idx / n_t)
    return s @ W


# ----------------------------------------------------------------------------
# O3  apodization and lateral placement
# ----------------------------------------------------------------------------

def pattern_masks(n_elements: int, m: int, n_sub: int) -> np.ndarray:
    """Pattern-m with n complementary sub-apertures: a_i[l] = 1 iff floor(l/m) mod n == i.

    Blocks of m active elements separated by (n-1)m inactive ones (Section II-A
    for n = 2, Section II-C for n = 3).
    """
    a = np.zeros((n_sub, n_elements), dtype=np.uint8)
    for l in range(n_elements):
        a[(l // m) % n_sub, l] = 1
    return a


def lateral_layout(n_elements: int, pitch_m: float, n_x: int, mode: str) -> Tuple[np.ndarray, float, np.ndarray]:
    """Grid column j of each element, the grid spacing dx and the grid x coordinates.

    pad:   j = o + l with o = floor((N_x - L)/2), dx = pitch.
    stuff: j = s*l with s = N_x / L, dx = pitch / s (zero-stuffed channels between
           elements, Section II-E).
    Grid coordinate: the array centre is the origin (Fig. 1), so
    x_j = (j - j_centre) * dx with j_centre the (fractional) column of the array centre.
    """
    L = n_elements
    if mode == "pad":
        o = (n_x - L) // 2
        cols = o + np.arange(L)
        dx = pitch_m
        centre = o + (L - 1) / 2.0
    elif mode == "stuff":
        s = n_x // L
        cols = s * np.arange(L)
        dx = pitch_m / s
        centre = s * (L - 1) / 2.0
    else:
        raise ValueError(mode)
    x = (np.arange(n_x) - centre) * dx
    return cols.astype(np.int64), dx, x


def place(X: np.ndarray, masks: np.ndarray, cols: np.ndarray, n_x: int) -> np.ndarray:
    """u[i, b, j]: apodized channel spectra on the lateral grid, zeros elsewhere."""
    n_sub = masks.shape[0]
    n_b = X.shape[1]
    u = np.zeros((n_sub, n_b, n_x), dtype=np.complex128)
    for i in range(n_sub):
        u[i][:, cols] = (masks[i][:, None] * X).T
    return u


# ----------------------------------------------------------------------------
# O4 / O6  lateral DFT pair
# ----------------------------------------------------------------------------

def dft_matrix(n: int, sign: int) -> np.ndarray:
    """W[a, b] = exp(sign * 2 pi i ((a b) mod n) / n)."""
    a = np.arange(n, dtype=np.int64)
    return np.exp(sign * 1j * TWO_PI * ((a[:, None] * a[None, :]) % n) / n)


def lateral_dft(u: np.ndarray) -> np.ndarray:
    """P[..., q] = sum_j u[..., j] exp(-2 pi i q j / N) (Eq. 1, F_x)."""
    n = u.shape[-1]
    return u @ dft_matrix(n, -1).T


def inverse_lateral_dft(P: np.ndarray) -> np.ndarray:
    """p[..., j] = (1/N) sum_q P[..., q] exp(+2 pi i q j / N)."""
    n = P.shape[-1]
    return (P @ dft_matrix(n, +1).T) / n


# ----------------------------------------------------------------------------
# O5  propagator (Eq. 2)
# ----------------------------------------------------------------------------

def kx_grid(n_x: int, dx: float) -> np.ndarray:
    """kx_q = 2 pi qs / (N dx), qs = q for q < N/2 else q - N (the DFT's own frequencies)."""
    q = np.arange(n_x)
    qs = np.where(q < n_x / 2, q, q - n_x)
    return TWO_PI * qs / (n_x * dx)


def kz(k: np.ndarray, kx: np.ndarray) -> np.ndarray:
    """Principal complex root sqrt(k^2 - kx^2): real when propagating, +i*sqrt(kx^2-k^2) otherwise."""
    d = k[..., None] ** 2 - kx[None, :] ** 2
    return np.where(d >= 0, np.sqrt(np.abs(d)) + 0j, 1j * np.sqrt(np.abs(d)))


def propagator(kz_: np.ndarray, z: np.ndarray, mode: str = "decay") -> np.ndarray:
    """H[b, d, q] = exp(i z_d kz[b, q]); mode 'zero' drops evanescent components."""
    H = np.exp(1j * z[None, :, None] * kz_[:, None, :])
    if mode == "zero":
        H = np.where((np.imag(kz_) > 0)[:, None, :], 0.0, H)
    elif mode != "decay":
        raise ValueError(mode)
    return H


# ----------------------------------------------------------------------------
# Whole pipeline
# ----------------------------------------------------------------------------

def geometry_tables(geom) -> Dict[str, np.ndarray]:
    """Everything the reconstruction needs that depends on the geometry only."""
    ks = bins(geom.fs_hz, geom.n_samples, geom.bands_hz)
    cols, dx, x = lateral_layout(geom.n_elements, geom.pitch_m, geom.n_x, geom.lateral)
    if geom.apod is not None:
        masks = np.asarray(geom.apod, dtype=np.uint8)
    else:
        masks = pattern_masks(geom.n_elements, geom.pattern_m, geom.n_sub)
    f = ks * geom.fs_hz / geom.n_samples
    kk = TWO_PI * f / geom.c_mps
    return dict(ks=ks, f=f, k=kk, cols=cols, dx=np.float64(dx), x=x, masks=masks,
                kx=kx_grid(geom.n_x, dx))


def fields(rf: np.ndarray, geom, chunk: int = 16):
    """Yield (bin slice, p[i, b, d, j]) for chunks of bins: the monochromatic fields (O2-O6)."""
    t = geometry_tables(geom)
    n_t = rf.shape[-1]
    if n_t != geom.n_samples:
        raise ValueError("record length must equal the geometry's n_samples")
    X = time_dft(rf, t["ks"])                                  # [L][n_b]
    u = place(X, t["masks"], t["cols"], geom.n_x)              # [n_sub][n_b][N]
    P = lateral_dft(u)                                         # [n_sub][n_b][N]
    z = np.asarray(geom.depths_m, dtype=np.float64)
    KZ = kz(t["k"], t["kx"])                                   # [n_b][N]
    for b0 in range(0, len(t["ks"]), chunk):
        sl = slice(b0, min(b0 + chunk, len(t["ks"])))
        H = propagator(KZ[sl], z, geom.evanescent)            # [c][n_z][N]
        p = inverse_lateral_dft(H[None, :, :, :] * P[:, sl, None, :])   # [n_sub][c][n_z][N]
        yield sl, p


def cross_spectra(rf: np.ndarray, geom, chunk: int = 16) -> Dict[str, np.ndarray]:
    """O7: S_i, C_ij (pairs (1,2), (2,3), (3,1)) and E, each [n_z][N_x] float64."""
    n = geom.n_sub
    nz, nx = len(geom.depths_m), geom.n_x
    S = np.zeros((n, nz, nx))
    pairs = [(0, 1), (1, 2), (2, 0)] if n == 3 else ([(0, 1)] if n == 2 else [])
    C = np.zeros((len(pairs), nz, nx))
    E = np.zeros((nz, nx))
    for _, p in fields(rf, geom, chunk):
        S += np.sum(np.abs(p) ** 2, axis=1)
        for c, (i, j) in enumerate(pairs):
            C[c] += np.sum(np.real(np.conj(p[i]) * p[j]), axis=0)
        E += np.sum(np.abs(np.sum(p, axis=0)) ** 2, axis=0)
    return dict(S=S, C=C, E=E, pairs=np.asarray(pairs))


def ncc(S: np.ndarray, C: np.ndarray, pairs: np.ndarray) -> np.ndarray:
    """rho_ij = C_ij / (sqrt(S_i) sqrt(S_j)); 0 where a denominator vanishes (Eq. 4)."""
    out = np.zeros_like(C)
    for c, (i, j) in enumerate(pairs):
        den = np.sqrt(S[i]) * np.sqrt(S[j])
        ok = den > 0
        out[c][ok] = C[c][ok] / den[ok]
    return out


def weight(rho: np.ndarray, eps: float, n_sub: int) -> np.ndarray:
    """Clamp each pair to [eps, 1], then the TAX cube root (Eq. 10) / DAX pair / AS one."""
    r = np.clip(rho, eps, 1.0)
    if n_sub == 3:
        return np.cbrt(r[0] * r[1] * r[2])
    if n_sub == 2:
        return r[0]
    return np.ones(rho.shape[1:] if rho.ndim == 3 else rho.shape)


def as_tax(rf: np.ndarray, geom, chunk: int = 16) -> Dict[str, np.ndarray]:
    """Full reconstruction of one frame: I, rho_n, rho pairs, weight, E, S, C (O1-O9)."""
    cs = cross_spectra(rf, geom, chunk)
    S, C, E = cs["S"], cs["C"], cs["E"]
    if geom.n_sub >= 2:
        rho = ncc(S, C, cs["pairs"])
        w = weight(rho, geom.eps, geom.n_sub)
    else:
        rho = np.zeros((0,) + E.shape)
        w = np.ones_like(E)
    rho_n = w / np.max(w)
    I = rho_n ** 2 * E
    return dict(I=I, rho_n=rho_n, rho=rho, w=w, E=E, S=S, C=C)


def pair_cross_spectra(rf: np.ndarray, geom, chunk: int = 16) -> Dict[str, np.ndarray]:
    """Full-aperture field sums with adjacent-pixel partners (inputs of the surrogate's
    phase-coherence features): with p the full-aperture field (plain AS, Eq. 3),
    S = sum_w |p|^2, G_x[z, x] = sum_w p[z, x] conj(p[z, x ^ 1]) over pairs of adjacent
    columns (2j, 2j + 1) and G_z[z, x] = sum_w p[z, x] conj(p[z ^ 1, x]) over pairs of
    adjacent depths (2i, 2i + 1).  Needs an even number of columns and of depths."""
    g = geom.replace(n_sub=1, apod=np.ones((1, geom.n_elements), np.uint8))
    nz, nx = len(geom.depths_m), geom.n_x
    if nz % 2 or nx % 2:
        raise ValueError("pairs need an even number of depths and of columns")
    xi = np.arange(nx) ^ 1
    zi = np.arange(nz) ^ 1
    S = np.zeros((nz, nx))
    Gx = np.zeros((nz, nx), dtype=np.complex128)
    Gz = np.zeros((nz, nx), dtype=np.complex128)
    for _, p in fields(rf, g, chunk):
        q = p[0]                                            # [c][n_z][N]
        S += np.sum(np.abs(q) ** 2, axis=0)
        Gx += np.sum(q * np.conj(q[:, :, xi]), axis=0)
        Gz += np.sum(q * np.conj(q[:, zi, :]), axis=0)
    return dict(S=S, Gx=Gx, Gz=Gz)


def as_image(rf: np.ndarray, geom, chunk: int = 16) -> np.ndarray:
    """Plain AS image of Eq. 3 with the full aperture: sum over bins of |p|^2."""
    g = geom.replace(n_sub=1, apod=np.ones((1, geom.n_elements), np.uint8))
    return cross_spectra(rf, g, chunk)["S"][0]


def stage_outputs(rf: np.ndarray, geom) -> Dict[str, np.ndarray]:
    """Intermediate results for stage-by-stage parity: X (time DFT at the bins) and P."""
    t = geometry_tables(geom)
    X = time_dft(rf, t["ks"])
    u = place(X, t["masks"], t["cols"], geom.n_x)
    return dict(X=X, u=u, P=lateral_dft(u), ks=t["ks"])


# ----------------------------------------------------------------------------
# Image metrics (Section II-E: ESA, ISNR of Eq. 12, centroid of Eq. 13)
# ----------------------------------------------------------------------------

def esa(I: np.ndarray, dx: float, dz: float) -> float:
    """Energy spread area: area of pixels above half of the image maximum."""
    return float(np.count_nonzero(I > 0.5 * I.max()) * dx * dz)


def isnr_db(I: np.ndarray) -> float:
    """10 log10(mean inside A_0.5 / mean outside A_0.5) (Eq. 12)."""
    m = I > 0.5 * I.max()
    return float(10.0 * np.log10(I[m].mean() / I[~m].mean()))


def centroid(I: np.ndarray, x: np.ndarray, z: np.ndarray, alpha: float = 0.7) -> Tuple[float, float]:
    """Intensity-weighted centroid of pixels above alpha * max (Eq. 13)."""
    m = I > alpha * I.max()
    Z, Xg = np.meshgrid(z, x, indexing="ij")
    w = I[m]
    return float(np.sum(w * Xg[m]) / w.sum()), float(np.sum(w * Z[m]) / w.sum())
