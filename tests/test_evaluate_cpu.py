"""The evaluation harness's host-side measures against independent values: its image
metrics against the oracle's (pinned by hand-worked images in test_oracle.py), its
lateral grid against the oracle's layout, the Rayleigh dip and regional peaks on
analytic profiles."""
import numpy as np

from oracle import as_tax as O
from paper_2412_02413_amd import evaluate as E
from paper_2412_02413_amd import synth

MM = 1e-3


def test_metrics_match_oracle():
    rng = np.random.default_rng(0)
    x = (np.arange(64) - 31.5) * 0.1 * MM
    z = (30 + 0.2 * np.arange(40)) * MM
    for _ in range(5):
        I = rng.gamma(0.5, 1.0, (40, 64))
        assert E.isnr_db(I) == O.isnr_db(I)
        assert abs(E.esa_mm2(I, 0.1 * MM, 0.2 * MM) - O.esa(I, 0.1 * MM, 0.2 * MM) / MM ** 2) < 1e-12
        assert np.allclose(E.centroid(I, x, z, 0.7), O.centroid(I, x, z, 0.7), rtol=0, atol=1e-15)


def test_grid_matches_oracle_layout():
    for g in (synth.paper_geometry(690), synth.cfg1_geometry(), synth.cfg2_geometry()):
        _, _, x = O.lateral_layout(g.n_elements, g.pitch_m, g.n_x, g.lateral)
        np.testing.assert_allclose(E.grid_x(g), x, rtol=0, atol=1e-15)


def test_profile_dip_analytic():
    # two Gaussians of width w at +-s: the midpoint value is 2 exp(-(s/w)^2), the peaks
    # (on the sampling grid, near +-s) close to 1 + exp(-(2s/w)^2)
    x = np.arange(-400, 401) * 0.001 * MM
    z = np.array([40.0 * MM])
    for s, w in ((0.175, 0.12), (0.175, 0.25), (0.3, 0.2)):
        prof = np.exp(-((x / MM - s) / w) ** 2) + np.exp(-((x / MM + s) / w) ** 2)
        r = E.profile_dip(prof[None, :], x, z, (-s, 40.0), (s, 40.0))
        want = 1.0 - prof[400] / prof.max() if prof[400] < prof.max() else 0.0
        assert abs(r["dip"] - want) < 1e-4, (s, w, r, want)
        assert r["resolved"] == (want >= E.RAYLEIGH_DIP)
    # axial profile: same function of depth
    zz = (38 + np.arange(0, 4001) * 0.001) * MM
    prof = np.exp(-((zz / MM - 39.0) / 0.6) ** 2) + np.exp(-((zz / MM - 41.0) / 0.6) ** 2)
    r = E.profile_dip(prof[:, None], np.array([0.0]), zz, (0.0, 39.0), (0.0, 41.0))
    assert abs(r["dip"] - (1 - prof[2000] / prof.max())) < 1e-4


def test_regional_peaks():
    x = (np.arange(21) - 10) * 1.0 * MM
    z = (30 + np.arange(21)) * MM
    I = np.zeros((21, 21))
    I[10, 5] = 0.3      # (-5 mm, 40 mm)
    I[10, 15] = 1.0     # (+5 mm, 40 mm)
    I[0, 0] = 5.0       # far away: outside both regions
    assert E.regional_peaks(I, x, z, (-5.0, 40.0), (5.0, 40.0)) == [0.3, 1.0]
