"""Pins for the FD-TEA-TAX oracle (oracle/fd_tea.py), each from outside the oracle:

* an integer-sample delay: a pixel straight below an element at depth m c / fs sees that
  element's spectrum with the phase of an m-sample advance, i.e. numpy's rfft of the
  circularly shifted channel;
* Parseval against time-domain delay-and-sum (Eq. 6 and Eq. 7): the channels projected
  on the bins of Omega, delayed by the exact travel time through a band-limited
  interpolation kernel and summed in pure-Python loops, carry the energy and
  cross-correlations of the frequency-domain fields times 2 / n_t;
* a point emitter focuses at its true position;
* identical sub-apertures give rho = 1 (Eq. 4 with Cauchy-Schwarz equality).
"""
import math

import numpy as np

from oracle import as_tax as A
from oracle import fd_tea as T
from paper_2412_02413_amd import synth

MM = 1e-3


def tiny(**kw):
    g = synth.Geometry(n_elements=3, pitch_m=0.3 * MM, fs_hz=20e6, c_mps=1540.0, n_samples=16,
                       bands_hz=[(2.4e6, 7.6e6)], depths_m=np.array([0.4, 1.3]) * MM, n_x=8,
                       lateral="pad", n_sub=3, apod=np.eye(3, dtype=np.uint8))
    return g.replace(**kw)


def test_integer_delay_is_a_circular_shift():
    m, n_t = 5, 64
    g = synth.Geometry(n_elements=4, pitch_m=0.3 * MM, fs_hz=20e6, c_mps=1540.0, n_samples=n_t,
                       bands_hz=[(1e6, 9e6)], depths_m=np.array([m * 1540.0 / 20e6]), n_x=8,
                       lateral="pad", n_sub=1, apod=np.array([[0, 1, 0, 0]], np.uint8))
    rng = np.random.default_rng(3)
    rf = rng.standard_normal((4, n_t))
    t = A.geometry_tables(g)
    j = int(t["cols"][1])                         # the pixel column of element 1
    (sl, p), = list(T.fields(rf, g, chunk=64))
    want = np.fft.rfft(np.roll(rf[1], -m))[t["ks"]]
    np.testing.assert_allclose(p[0, :, 0, j], want, atol=1e-9 * np.abs(want).max())


def _td_das(rf, g):
    """Pure-Python time-domain delay-and-sum of the band-limited channels: returns
    p[i][pixel][n] for every sub-aperture, pixel and sample."""
    n_t, L = g.n_samples, g.n_elements
    ks = [k for k in range(1, n_t // 2) if any(lo <= k * g.fs_hz / n_t <= hi for lo, hi in g.bands_hz)]

    def kernel(u):     # projection of a unit sample on the bins of Omega, evaluated at lag u
        return sum(2.0 * math.cos(2.0 * math.pi * k * u / n_t) for k in ks) / n_t

    o = (g.n_x - L) // 2
    centre = o + (L - 1) / 2.0
    out = []
    for i in range(g.n_sub):
        rows = []
        for z in g.depths_m:
            for j in range(g.n_x):
                x = (j - centre) * g.pitch_m
                sig = [0.0] * n_t
                for l in range(L):
                    if not g.apod[i][l]:
                        continue
                    xl = (o + l - centre) * g.pitch_m
                    shift = math.sqrt((x - xl) ** 2 + z ** 2) / g.c_mps * g.fs_hz
                    for n in range(n_t):
                        sig[n] += sum(rf[l][q] * kernel(n + shift - q) for q in range(n_t))
                rows.append(sig)
        out.append(np.array(rows))
    return out


def test_parseval_against_time_domain_delay_and_sum():
    g = tiny()
    rng = np.random.default_rng(4)
    rf = rng.standard_normal((3, 16))
    p_td = _td_das(rf, g)                                     # [i][pixel][n]
    cs = T.cross_spectra(rf, g)
    scale = 2.0 / g.n_samples
    S_td = np.array([np.sum(p ** 2, axis=1) for p in p_td])
    np.testing.assert_allclose(S_td, scale * cs["S"].reshape(3, -1), rtol=1e-10)
    for c, (i, j) in enumerate(cs["pairs"]):
        np.testing.assert_allclose(np.sum(p_td[i] * p_td[j], axis=1), scale * cs["C"][c].ravel(),
                                   atol=1e-10 * S_td.max())
    E_td = np.sum(sum(p_td) ** 2, axis=1)
    np.testing.assert_allclose(E_td, scale * cs["E"].ravel(), rtol=1e-10)


def test_point_emitter_focus():
    g = synth.cfg1_geometry().replace(depths_m=(24.0 + 0.2 * np.arange(61)) * MM)
    for snr in (None, 20.0):
        rf = synth.cfg1_frame(21, snr_db=snr)
        r = T.fd_tea_tax(rf, g)
        d, j = np.unravel_index(np.argmax(r["I"]), r["I"].shape)
        t = A.geometry_tables(g)
        assert abs(t["x"][j]) <= 0.3 * MM + 1e-12
        assert abs(g.depths_m[d] - 30 * MM) <= 1.0 * MM
        assert np.all(np.abs(r["rho"]) <= 1 + 1e-12)


def test_identical_subapertures():
    g = synth.cfg1_geometry().replace(depths_m=(28.0 + 0.4 * np.arange(9)) * MM, apod=np.ones((3, 64), np.uint8))
    rf = synth.cfg1_frame(22)
    r = T.fd_tea_tax(rf, g)
    np.testing.assert_allclose(r["rho"], 1.0, atol=1e-12)
    np.testing.assert_allclose(r["rho_n"], 1.0, atol=1e-12)
    np.testing.assert_allclose(r["E"], 9 * r["S"][0], rtol=1e-12)
