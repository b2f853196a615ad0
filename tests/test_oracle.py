"""Pins for the FP64 oracle: each check comes from outside the oracle itself.

Sources of truth used here: values printed in the paper (tests/golden), numpy's
FFT routines, closed forms (single tone, plane wave), mathematical identities of
Eq. 2 and Eq. 4 (z = 0 identity, semigroup, Cauchy-Schwarz, Appendix A's
time/frequency equivalence, linearity), a brute-force circular-convolution
formulation written with pure-Python loops, and the point-emitter focus.
"""
import cmath
import math
import os

import numpy as np
import pytest

from oracle import as_tax as O
from paper_2412_02413_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
MM = 1e-3


def _golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def tiny_geometry(**kw):
    g = synth.Geometry(n_elements=4, pitch_m=0.3 * MM, fs_hz=20e6, c_mps=1540.0, n_samples=32,
                       bands_hz=[(2e6, 5e6)], depths_m=np.array([0.0, 0.7, 1.9, 3.2, 5.0]) * MM,
                       n_x=8, lateral="pad", n_sub=2, pattern_m=1)
    return g.replace(**kw)


def small_cfg1(n_depths=41, z0_mm=26.0, dz_mm=0.2):
    g = synth.cfg1_geometry()
    return g.replace(depths_m=(z0_mm + dz_mm * np.arange(n_depths)) * MM)


# ---------------------------------------------------------------- O1, O3: printed values

def test_bins_reproduce_wideband_count():
    for row in _golden("counts.txt"):
        if row[0] != "wideband_bins":
            continue
        kv = dict(p.split("=") for p in row[2:])
        ks = O.bins(float(kv["fs_hz"]), int(kv["n_t"]), [(float(kv["lo_hz"]), float(kv["hi_hz"]))])
        assert len(ks) == int(row[1])
        assert ks[0] == 173 and ks[-1] == 862


def test_band_union_is_the_union_of_its_bands():
    """Eq. 3's Omega as a union of closed windows (frequency-selective maps): the bin set
    is the disjoint union of each window's bins, and every sum over Omega (S_i, C_ij, E)
    is the sum of the per-window sums."""
    g = small_cfg1(n_depths=9)
    bands = [(1.2e6, 1.8e6), (2.8e6, 3.4e6)]
    k_union = O.bins(g.fs_hz, g.n_samples, bands)
    k_parts = [O.bins(g.fs_hz, g.n_samples, [b]) for b in bands]
    assert len(set(k_parts[0]) & set(k_parts[1])) == 0
    np.testing.assert_array_equal(k_union, np.sort(np.concatenate(k_parts)))
    rf = synth.cfg1_frame(3)
    ru = O.as_tax(rf, g.replace(bands_hz=bands))
    r1 = O.as_tax(rf, g.replace(bands_hz=[bands[0]]))
    r2 = O.as_tax(rf, g.replace(bands_hz=[bands[1]]))
    for key in ("E", "S", "C"):
        np.testing.assert_allclose(ru[key], r1[key] + r2[key], rtol=1e-12, atol=1e-12 * np.abs(ru[key]).max())


def test_propagator_table_sizes_match_printed_memory():
    # complex64 n_w x n_z x n_x tables: the printed MB figures are MiB of 8-byte entries
    for row in _golden("counts.txt"):
        if row[0] == "propagator_table_mib":
            kv = dict(p.split("=") for p in row[2:])
            n = int(kv["n_w"]) * int(kv["n_z"]) * int(kv["n_x"]) * int(kv["bytes"])
            assert round(n / 2 ** 20) == int(row[1])
        if row[0] == "image_pixels":
            kv = dict(p.split("=") for p in row[2:])
            assert int(kv["n_z"]) * int(kv["n_x"]) == int(row[1])


def test_pattern_masks_match_printed_examples():
    for label, L, m, n, i, digits in _golden("apodization_examples.txt"):
        a = O.pattern_masks(int(L), int(m), int(n))
        want = np.array([int(c) for c in digits], dtype=np.uint8)
        np.testing.assert_array_equal(a[int(i) - 1], want)
    a = O.pattern_masks(128, 16, 3)
    assert np.all(a.sum(axis=0) == 1)          # complementary


def test_cfg_bin_counts():
    assert len(O.bins(20e6, 1024, [(1e6, 5e6)])) == 205
    assert len(O.bins(40e6, 4096, [(0.5e6, 8e6)])) == 768
    # a coarse record's bins are the fine record's bins at every 4th index
    fine = O.bins(20e6, 8192, [(1e6, 5e6)])
    coarse = O.bins(20e6, 2048, [(1e6, 5e6)])
    np.testing.assert_array_equal(4 * coarse, fine[fine % 4 == 0])


# ---------------------------------------------------------------- O2: library FFT and a closed form

def test_time_dft_matches_numpy_rfft():
    rng = np.random.default_rng(1)
    rf = rng.standard_normal((5, 256))
    ks = np.array([1, 7, 64, 100, 127])
    X = O.time_dft(rf, ks)
    np.testing.assert_allclose(X, np.fft.rfft(rf, axis=1)[:, ks], rtol=0, atol=1e-11)


def test_time_dft_single_tone_closed_form():
    n_t, k0, phi = 512, 37, 0.7
    n = np.arange(n_t)
    rf = np.cos(2 * np.pi * k0 * n / n_t + phi)[None, :]
    X = O.time_dft(rf, np.array([k0 - 1, k0, k0 + 1]))
    assert abs(X[0, 1] - n_t / 2 * np.exp(1j * phi)) < 1e-10
    assert abs(X[0, 0]) < 1e-10 and abs(X[0, 2]) < 1e-10


# ---------------------------------------------------------------- O4/O6: library FFT

def test_lateral_dft_pair_matches_numpy_fft():
    rng = np.random.default_rng(2)
    u = rng.standard_normal((3, 4, 16)) + 1j * rng.standard_normal((3, 4, 16))
    np.testing.assert_allclose(O.lateral_dft(u), np.fft.fft(u, axis=-1), atol=1e-12)
    np.testing.assert_allclose(O.inverse_lateral_dft(u), np.fft.ifft(u, axis=-1), atol=1e-13)


def test_layout_pad_and_stuff():
    cols, dx, x = O.lateral_layout(64, 0.3e-3, 128, "pad")
    assert cols[0] == 32 and dx == 0.3e-3
    assert abs(x[32] + 31.5 * 0.3e-3) < 1e-15 and abs(x[95] - 31.5 * 0.3e-3) < 1e-15
    cols, dx, x = O.lateral_layout(128, 0.178e-3, 256, "stuff")
    assert cols[1] == 2 and abs(dx - 0.089e-3) < 1e-18
    assert abs(x[0] + 63.5 * 0.178e-3) < 1e-12   # element 0 at -(L-1)/2 pitch


# ---------------------------------------------------------------- O5: Eq. 2 identities

def test_z0_returns_input_spectrum():
    g = tiny_geometry(depths_m=np.array([0.0, 1e-3]))
    rng = np.random.default_rng(3)
    rf = rng.standard_normal((4, 32))
    st = O.stage_outputs(rf, g)
    for sl, p in O.fields(rf, g, chunk=64):
        np.testing.assert_allclose(p[:, :, 0, :], st["u"][:, sl, :], atol=1e-12)


def test_zero_mode_keeps_only_propagating_at_z0():
    g = tiny_geometry(depths_m=np.array([0.0]), evanescent="zero")
    t = O.geometry_tables(g)
    KZ = O.kz(t["k"], t["kx"])
    H = O.propagator(KZ, np.array([0.0]), "zero")[:, 0, :]
    prop = np.imag(KZ) == 0
    assert np.any(~prop) and np.any(prop)
    np.testing.assert_array_equal(H[prop], 1.0)
    np.testing.assert_array_equal(H[~prop], 0.0)


@pytest.mark.parametrize("mode", ["decay", "zero"])
def test_propagator_semigroup(mode):
    g = tiny_geometry()
    t = O.geometry_tables(g)
    KZ = O.kz(t["k"], t["kx"])
    z1, z2 = np.array([1.3e-3]), np.array([2.9e-3])
    H1 = O.propagator(KZ, z1, mode)
    H2 = O.propagator(KZ, z2, mode)
    H12 = O.propagator(KZ, z1 + z2, mode)
    np.testing.assert_allclose(H1 * H2, H12, atol=1e-13)


def test_field_repropagation_semigroup():
    # p(z1 + z2) equals the field at z1 re-propagated by z2 with numpy's own FFT
    g = tiny_geometry(depths_m=np.array([1.1e-3, 3.6e-3]))
    rng = np.random.default_rng(4)
    rf = rng.standard_normal((4, 32))
    t = O.geometry_tables(g)
    KZ = O.kz(t["k"], t["kx"])
    for sl, p in O.fields(rf, g, chunk=64):
        spec = np.fft.fft(p[:, :, 0, :], axis=-1)
        step = np.exp(1j * 2.5e-3 * KZ[sl])
        again = np.fft.ifft(spec * step[None], axis=-1)
        np.testing.assert_allclose(again, p[:, :, 1, :], atol=1e-10)


def test_plane_wave_closed_form():
    # N_x = L (no padding), one tone on bin k0 whose element phases follow a grid kx0:
    # p[k0, d, j] = u[j] exp(i z_d sqrt(k^2 - kx0^2)) exactly (Eq. 2 applied to one kx).
    L, n_t, fs, c, pitch = 16, 128, 20e6, 1540.0, 0.3e-3
    k0, q0 = 20, 3
    g = synth.Geometry(n_elements=L, pitch_m=pitch, fs_hz=fs, c_mps=c, n_samples=n_t,
                       bands_hz=[(k0 * fs / n_t, k0 * fs / n_t)], depths_m=np.array([0.0, 4e-3, 9e-3]),
                       n_x=L, lateral="pad", n_sub=1, apod=np.ones((1, L), np.uint8))
    kx0 = 2 * np.pi * q0 / (L * pitch)
    xl = (np.arange(L) - (L - 1) / 2) * pitch
    n = np.arange(n_t)
    rf = np.cos(2 * np.pi * k0 * n[None, :] / n_t + kx0 * xl[:, None])
    kk = 2 * np.pi * (k0 * fs / n_t) / c
    kzv = math.sqrt(kk ** 2 - kx0 ** 2)
    u = (n_t / 2) * np.exp(1j * kx0 * xl)
    (sl, p), = list(O.fields(rf, g, chunk=8))
    for d, z in enumerate(g.depths_m):
        np.testing.assert_allclose(p[0, 0, d, :], u * np.exp(1j * z * kzv), atol=1e-9)
    E = O.cross_spectra(rf, g)["S"][0]
    np.testing.assert_allclose(E, E[0, 0], rtol=1e-12)     # constant over the image


def _brute_force_fields(rf, g):
    """Pure-Python circular-convolution form of O2-O6 (tiny sizes only)."""
    L, n_t, N = g.n_elements, g.n_samples, g.n_x
    fs, c = g.fs_hz, g.c_mps
    ks = [k for k in range(1, n_t // 2) if any(lo <= k * fs / n_t <= hi for lo, hi in g.bands_hz)]
    masks = g.apod if g.apod is not None else [[1 if (l // g.pattern_m) % g.n_sub == i else 0
                                                 for l in range(L)] for i in range(g.n_sub)]
    o = (N - L) // 2
    out = np.zeros((g.n_sub, len(ks), len(g.depths_m), N), complex)
    for b, k in enumerate(ks):
        X = [sum(rf[l][n] * cmath.exp(-2j * math.pi * k * n / n_t) for n in range(n_t)) for l in range(L)]
        kk = 2 * math.pi * k * fs / n_t / c
        for d, z in enumerate(g.depths_m):
            # spatial kernel g[m] = (1/N) sum_q exp(i z kz_q) exp(2 pi i q m / N)
            ker = []
            for mm in range(N):
                acc = 0j
                for q in range(N):
                    qs = q if q < N / 2 else q - N
                    kx = 2 * math.pi * qs / (N * g.pitch_m)
                    acc += cmath.exp(1j * z * cmath.sqrt(kk * kk - kx * kx)) * cmath.exp(2j * math.pi * q * mm / N)
                ker.append(acc / N)
            for i in range(g.n_sub):
                for j in range(N):
                    out[i, b, d, j] = sum(masks[i][l] * X[l] * ker[(j - (o + l)) % N] for l in range(L))
    return out


def test_brute_force_convolution_form():
    g = tiny_geometry()
    rng = np.random.default_rng(5)
    rf = rng.standard_normal((4, 32))
    ref = _brute_force_fields(rf, g)
    (sl, p), = list(O.fields(rf, g, chunk=64))
    np.testing.assert_allclose(p, ref, atol=1e-10 * np.abs(ref).max())


# ---------------------------------------------------------------- O7/O8: Eq. 4 and Appendix A

@pytest.fixture(scope="module")
def cfg1_small():
    g = small_cfg1()
    rf = synth.cfg1_frame(11)
    return g, rf, O.as_tax(rf, g)


def test_cauchy_schwarz(cfg1_small):
    g, rf, r = cfg1_small
    assert np.all(np.abs(r["rho"]) <= 1 + 1e-12)
    assert r["rho"].min() < 0.5      # the bound is not vacuous on this frame


def test_energy_identity(cfg1_small):
    _, _, r = cfg1_small
    np.testing.assert_allclose(r["E"], r["S"].sum(0) + 2 * r["C"].sum(0), rtol=1e-10)


def test_identical_subapertures():
    g = small_cfg1(n_depths=11)
    full = np.ones((3, 64), np.uint8)
    rf = synth.cfg1_frame(12)
    r = O.as_tax(rf, g.replace(apod=full))
    ok = r["S"][0] > 0
    np.testing.assert_allclose(r["rho"][:, ok], 1.0, atol=1e-12)
    np.testing.assert_allclose(r["rho_n"], 1.0, atol=1e-12)
    E_as = O.as_image(rf, g)
    np.testing.assert_allclose(r["I"], 9 * E_as, rtol=1e-11)


def test_complementary_masks_energy_is_plain_as_image(cfg1_small):
    g, rf, r = cfg1_small
    np.testing.assert_allclose(r["E"], O.as_image(rf, g), rtol=1e-11)


def test_scale_invariance():
    g = small_cfg1(n_depths=9)
    rf = synth.cfg1_frame(13).astype(np.float64)
    a = O.as_tax(rf, g)
    b = O.as_tax(3.5 * rf, g)
    np.testing.assert_allclose(b["rho"], a["rho"], atol=1e-12)
    np.testing.assert_allclose(b["E"], 3.5 ** 2 * a["E"], rtol=1e-11)


def test_appendix_a_time_domain_ncc_equals_frequency_domain(cfg1_small):
    # Eq. 8 (mean removed, time domain) on the band-limited time signals equals Eq. 4
    g, rf, r = cfg1_small
    pix = [(3, 60), (20, 63), (30, 10), (40, 100)]
    n_t = g.n_samples
    t = O.geometry_tables(g)
    spec = {pp: np.zeros((3, n_t // 2 + 1), complex) for pp in pix}
    for sl, p in O.fields(rf, g):
        for (d, j) in pix:
            spec[(d, j)][:, t["ks"][sl]] = p[:, :, d, j]
    for (d, j) in pix:
        x = np.fft.irfft(spec[(d, j)], n=n_t, axis=-1)
        x = x - x.mean(axis=-1, keepdims=True)
        for c, (a, b) in enumerate([(0, 1), (1, 2), (2, 0)]):
            rho_td = x[a] @ x[b] / math.sqrt((x[a] @ x[a]) * (x[b] @ x[b]))
            assert abs(rho_td - r["rho"][c, d, j]) < 1e-12
        # The weighted image in its time-domain form (Eq. 9 structure, TEA-TAX): the sum over
        # time of the squared NNCC-weighted beamformed signal equals the frequency-domain image
        # up to Parseval's factor n_t / 2 (positive bins only, DC and Nyquist excluded).
        i_td = np.sum((r["rho_n"][d, j] * x.sum(axis=0)) ** 2) * n_t / 2
        assert abs(i_td - r["I"][d, j]) < 1e-9 * r["I"][d, j]


def test_tax_weight_is_cube_root_via_dax():
    # a1 == a2, a3 different: rho_12 = 1 and rho_23 = rho_31 = DAX(a2, a3), so the
    # TAX weight (Eq. 10) is the DAX weight to the power 2/3.
    g = small_cfg1(n_depths=9)
    rf = synth.cfg1_frame(14)
    m = O.pattern_masks(64, 16, 2)
    tax = O.as_tax(rf, g.replace(n_sub=3, apod=np.stack([m[0], m[0], m[1]])))
    dax = O.as_tax(rf, g.replace(n_sub=2, apod=m))
    np.testing.assert_allclose(tax["w"], np.clip(dax["w"], 1e-3, 1) ** (2.0 / 3.0), rtol=1e-10)


def test_eps_floor_and_normalisation(cfg1_small):
    g, _, r = cfg1_small
    assert np.any(r["rho"] < g.eps)                     # some pairs are floored
    assert r["w"].min() >= g.eps - 1e-15
    assert abs(r["rho_n"].max() - 1.0) < 1e-15
    assert r["rho_n"].min() >= g.eps / r["w"].max() - 1e-15


# ---------------------------------------------------------------- end to end: point emitter

@pytest.mark.parametrize("snr", [None, 20.0])
def test_point_emitter_focus(snr):
    g = synth.cfg1_geometry().replace(depths_m=(24.0 + 0.2 * np.arange(61)) * MM)
    rf = synth.cfg1_frame(21, snr_db=snr)
    r = O.as_tax(rf, g)
    d, j = np.unravel_index(np.argmax(r["I"]), r["I"].shape)
    t = O.geometry_tables(g)
    assert abs(t["x"][j]) <= 0.3 * MM + 1e-12
    assert abs(g.depths_m[d] - 30 * MM) <= 1.0 * MM
    cx, cz = O.centroid(r["I"], t["x"], g.depths_m, 0.7)
    assert abs(cx) < 0.5 * MM and abs(cz - 30 * MM) < 1.0 * MM


def test_uneven_sources_soft():
    """Soft analogue of the paper's uneven-strength test (Appendix, Section C-2):
    AS-TAX keeps the weaker source's regional peak near the AS value; AS^3 crushes it."""
    g = synth.cfg1_geometry().replace(depths_m=(34.0 + 0.2 * np.arange(61)) * MM)
    rf = synth.coherent_pair_frame(31, x_mm=5.0, z_mm=40.0, ratio=2.0, snr_db=15.0)
    r = O.as_tax(rf, g)
    E_as = O.as_image(rf, g)
    t = O.geometry_tables(g)
    left, right = t["x"] < 0, t["x"] > 0
    n_as = E_as / E_as.max()
    rpi_as = n_as[:, left].max()
    rpi_tax = (r["I"] / E_as.max())[:, left].max()
    rpi_as3 = (n_as ** 2 * n_as)[:, left].max()
    assert 0.15 < rpi_as < 0.4
    assert 0.6 * rpi_as < rpi_tax <= rpi_as * 1.0001
    assert rpi_as3 < 0.3 * rpi_as


# ---------------------------------------------------------------- hand-worked values (reading of Eq. 4 text, Eq. 10, Eq. 12-13)

def test_bins_exclude_dc_and_nyquist():
    # a closed band covering [0, fs/2] keeps every bin except DC (k = 0) and Nyquist (k = n_t/2)
    for n_t in (32, 1024):
        ks = O.bins(20e6, n_t, [(0.0, 10e6)])
        assert len(ks) == n_t // 2 - 1
        assert ks[0] == 1 and ks[-1] == n_t // 2 - 1
    # a band holding only the Nyquist frequency is empty
    assert len(O.bins(20e6, 64, [(10e6, 10e6)])) == 0


def test_weight_floor_and_cap_hand_values():
    # every pair clamped to [eps, 1] before the cube root of Eq. 10:
    #   (0.5, 0.25, 5e-4) -> (0.5, 0.25, 1e-3): cube root of 1.25e-4 = 0.05
    #   (1.2, 0.5, 0.8)   -> (1, 0.5, 0.8):     cube root of 0.4
    rho = np.array([[0.5, 1.2], [0.25, 0.5], [5e-4, 0.8]])
    w = O.weight(rho, 1e-3, 3)
    assert abs(w[0] - 0.05) < 1e-15
    assert abs(w[1] - 0.7368062997280773) < 1e-15
    # one pair (n = 2): capped, floored (also a negative pair), passed through
    np.testing.assert_array_equal(O.weight(np.array([[1.5, -0.3, 0.42]]), 1e-3, 2), [1.0, 1e-3, 0.42])


def test_ncc_zero_denominator_hand_values():
    # pixel 0: S_1 = 0, so the pairs holding sub-aperture 1 are 0 (then floored to eps);
    #          rho_23 = 2 / (sqrt(2) sqrt(8)) = 0.5
    # pixel 1: 3 / (2 * 3) = 0.5, -1.5 / (3 * 1) = -0.5, 1 / (1 * 2) = 0.5
    S = np.array([[0.0, 4.0], [2.0, 9.0], [8.0, 1.0]])
    C = np.array([[0.0, 3.0], [2.0, -1.5], [0.0, 1.0]])
    rho = O.ncc(S, C, np.array([(0, 1), (1, 2), (2, 0)]))
    assert np.all(np.isfinite(rho))
    np.testing.assert_allclose(rho, [[0.0, 0.5], [0.5, -0.5], [0.0, 0.5]], rtol=0, atol=1e-15)


def test_dead_subaperture_closed_form():
    """a_1 = a_2 = every element, a_3 = none.  S_3 = 0, so rho_23 = rho_31 = 0 and both are
    floored to eps; rho_12 = 1 wherever S_1 > 0.  The TAX weight is (1 eps eps)^(1/3) =
    eps^(2/3) = 0.01 at every pixel, rho_n = 1, and I = E = sum |2 p|^2 = 4 E_AS."""
    g = small_cfg1(n_depths=9)
    rf = synth.cfg1_frame(15)
    apod = np.stack([np.ones(64), np.ones(64), np.zeros(64)]).astype(np.uint8)
    r = O.as_tax(rf, g.replace(apod=apod))
    assert np.all(r["S"][2] == 0.0)
    np.testing.assert_array_equal(r["rho"][1:], 0.0)
    np.testing.assert_allclose(r["rho"][0], 1.0, atol=1e-12)
    np.testing.assert_allclose(r["w"], 0.01, rtol=1e-12)
    np.testing.assert_allclose(r["rho_n"], 1.0, rtol=1e-12)
    np.testing.assert_allclose(r["I"], 4 * O.as_image(rf, g), rtol=1e-11)


def test_esa_isnr_centroid_hand_image():
    I = np.array([[4.0, 1.0, 0.0, 0.0],
                  [3.0, 2.5, 0.0, 0.0],
                  [0.0, 0.0, 0.0, 1.0],
                  [2.0, 0.0, 0.0, 1.0]])
    # A_0.5 = pixels strictly above half the maximum (2): {4, 3, 2.5}; the pixel equal to 2 is outside
    assert O.esa(I, 0.1e-3, 0.2e-3) == pytest.approx(3 * 0.1e-3 * 0.2e-3, rel=1e-14)
    # Eq. 12: inside mean 9.5 / 3, outside mean (1 + 1 + 1 + 2) / 13 -> 10 log10(9.5 * 13 / 15)
    assert abs(O.isnr_db(I) - 9.155756985400032) < 1e-12
    # Eq. 13 with alpha = 0.7: pixels above 7 are (z0, x1) = 10 and (z0, x2) = 8
    J = np.array([[0.0, 10.0, 8.0], [0.0, 0.0, 0.0]])
    cx, cz = O.centroid(J, np.array([0.0, 1.0, 2.0]), np.array([5.0, 6.0]), 0.7)
    assert abs(cx - 1.4444444444444444) < 1e-15 and cz == 5.0


# ---------------------------------------------------------------- pair cross-spectra (surrogate features)

def test_pair_cross_spectra_plane_wave_closed_form():
    # the plane wave of test_plane_wave_closed_form: p[d, j] = (n_t/2) e^{i kx0 x_j} e^{i z_d kz}, so
    # G_x = (n_t/2)^2 e^{i kx0 (x_j - x_{j^1})} and G_z = (n_t/2)^2 e^{i kz (z_d - z_{d^1})}
    L, n_t, fs, c, pitch = 16, 128, 20e6, 1540.0, 0.3e-3
    k0, q0 = 20, 3
    z = np.array([0.0, 4e-3, 9e-3, 9.5e-3])
    g = synth.Geometry(n_elements=L, pitch_m=pitch, fs_hz=fs, c_mps=c, n_samples=n_t,
                       bands_hz=[(k0 * fs / n_t, k0 * fs / n_t)], depths_m=z, n_x=L, lateral="pad", n_sub=1)
    kx0 = 2 * np.pi * q0 / (L * pitch)
    xl = (np.arange(L) - (L - 1) / 2) * pitch
    n = np.arange(n_t)
    rf = np.cos(2 * np.pi * k0 * n[None, :] / n_t + kx0 * xl[:, None])
    kzv = math.sqrt((2 * np.pi * (k0 * fs / n_t) / c) ** 2 - kx0 ** 2)
    r = O.pair_cross_spectra(rf, g)
    a2 = (n_t / 2) ** 2
    j = np.arange(L)
    want_x = a2 * np.exp(1j * kx0 * (xl[j] - xl[j ^ 1]))
    d = np.arange(len(z))
    want_z = a2 * np.exp(1j * kzv * (z[d] - z[d ^ 1]))
    np.testing.assert_allclose(r["Gx"], np.broadcast_to(want_x, r["Gx"].shape), atol=1e-8 * a2)
    np.testing.assert_allclose(r["Gz"], np.broadcast_to(want_z[:, None], r["Gz"].shape), atol=1e-8 * a2)
    np.testing.assert_allclose(r["S"], a2, rtol=1e-10)


def test_pair_cross_spectra_pairing_and_bound():
    g = small_cfg1(n_depths=10)
    rf = synth.cfg1_frame(16)
    r = O.pair_cross_spectra(rf, g)
    S, Gx, Gz = r["S"], r["Gx"], r["Gz"]
    x1 = np.arange(g.n_x) ^ 1
    z1 = np.arange(10) ^ 1
    np.testing.assert_allclose(Gx[:, x1], np.conj(Gx), rtol=1e-12, atol=1e-12 * S.max())
    np.testing.assert_allclose(Gz[z1, :], np.conj(Gz), rtol=1e-12, atol=1e-12 * S.max())
    assert np.all(np.abs(Gx) ** 2 <= S * S[:, x1] * (1 + 1e-12))
    assert np.all(np.abs(Gz) ** 2 <= S * S[z1, :] * (1 + 1e-12))
    np.testing.assert_allclose(S, O.as_image(rf, g), rtol=1e-12)
