"""FP64 CPU oracle for frequency-domain delay-and-sum with triple apodization (FD-TEA-TAX).

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite and the benchmark's
CPU legs may import or run anything in this directory.  It shares no code with
the HIP path.

The paper compares AS-TAX with delay-and-sum beamformers (Appendix, "PAM with DAX
and TAX").  Time exposure acoustics sums the element signals advanced by their
travel time from the pixel (Eq. 6) and integrates the square over time (Eq. 7).
Its frequency-domain form (the appendix's equation for the harmonic field of
FD-TEA) gives the monochromatic field at pixel r directly:

    p(r, w) = sum_l F_t{s_l}(w) exp(+i w tau_l(r)),   tau_l(r) = |r - r_l| / c,

which is the Fourier transform of Eq. 6 with unit distance weights (the
frequency-domain equation carries no d_l factor; that reading is taken here).
With the apodization sets of AS-TAX the sub-aperture fields p_i feed the same
cross-spectra, NCC, TAX weight, normalisation and image as the angular-spectrum
path (Eq. 4, Eq. 10, Eq. 11), so those steps are taken from oracle/as_tax.py.

Steps: bins and time DFT (as_tax O1, O2); delays tau_l(r) for every pixel of the
image grid (the same lateral grid and depths as AS: array centre at x = 0);
fields p_i[b, d, j] = sum_l a_i[l] X[l, b] exp(2 pi i f_b tau_l(d, j)); sums over
the bins of |p_i|^2, Re(conj(p_i) p_j) and |sum_i p_i|^2; NCC, TAX, NNCC, image.
"""
from __future__ import annotations

from typing import Dict

import numpy as np

from . import as_tax as A

TWO_PI = 2.0 * np.pi


def delays(geom) -> np.ndarray:
    """tau[l, d, j] = sqrt((x_j - x_l)^2 + z_d^2) / c: travel time from pixel (x_j, z_d) to
    element l on the array plane z = 0 (element l sits at grid column cols[l])."""
    t = A.geometry_tables(geom)
    x = t["x"]
    xl = x[t["cols"]]
    z = np.asarray(geom.depths_m, dtype=np.float64)
    dx = x[None, None, :] - xl[:, None, None]
    return np.sqrt(dx ** 2 + z[None, :, None] ** 2) / geom.c_mps


def fields(rf: np.ndarray, geom, chunk: int = 16):
    """Yield (bin slice, p[i, b, d, j]): the FD-TEA field of every sub-aperture."""
    t = A.geometry_tables(geom)
    n_t = rf.shape[-1]
    if n_t != geom.n_samples:
        raise ValueError("record length must equal the geometry's n_samples")
    X = A.time_dft(rf, t["ks"])                      # [L][n_b]
    tau = delays(geom)                                # [L][n_z][N]
    masks = t["masks"].astype(np.float64)             # [n_sub][L]
    f = t["f"]
    L, nz, nx = tau.shape
    for b0 in range(0, len(t["ks"]), chunk):
        sl = slice(b0, min(b0 + chunk, len(t["ks"])))
        p = np.zeros((masks.shape[0], sl.stop - sl.start, nz, nx), dtype=np.complex128)
        for c, b in enumerate(range(sl.start, sl.stop)):
            ph = np.exp(1j * TWO_PI * f[b] * tau).reshape(L, nz * nx)       # [L][pixels]
            wX = masks * X[None, :, b]                                       # [n_sub][L]
            p[:, c] = (wX @ ph).reshape(-1, nz, nx)
        yield sl, p


def cross_spectra(rf: np.ndarray, geom, chunk: int = 16) -> Dict[str, np.ndarray]:
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


def fd_tea_tax(rf: np.ndarray, geom, chunk: int = 16) -> Dict[str, np.ndarray]:
    """FD-TEA with the TAX weighting (n_sub = 3), DAX (2) or plain FD-TEA (1): I, rho_n, ..."""
    cs = cross_spectra(rf, geom, chunk)
    S, C, E = cs["S"], cs["C"], cs["E"]
    if geom.n_sub >= 2:
        rho = A.ncc(S, C, cs["pairs"])
        w = A.weight(rho, geom.eps, geom.n_sub)
    else:
        rho = np.zeros((0,) + E.shape)
        w = np.ones_like(E)
    rho_n = w / np.max(w)
    return dict(I=rho_n ** 2 * E, rho_n=rho_n, rho=rho, w=w, E=E, S=S, C=C)
