"""Host logic of the surrogate's fallback calibration (no GPU)."""
import math

import numpy as np

from paper_2412_02413_amd import surrogate as S
from paper_2412_02413_amd import synth


def test_calibration_quantile_by_hand():
    # 19 frames with ratios 1..19 (actual = r * est): k = ceil(20 * 0.9) = 18, q = 18, tau = bound / 18
    est = np.full(19, 0.01)
    actual = est * np.arange(1, 20)
    c = S.calibrate(est, actual, bound=0.36, alpha=0.1)
    assert c["q"] == 18 and math.isclose(c["tau"], 0.02)
    # too few frames for the level: nothing is accepted
    c = S.calibrate(est[:5], actual[:5], bound=0.36, alpha=0.1)
    assert c["q"] == math.inf and c["tau"] == 0.0 and c["calibration_accept_rate"] == 0.0


def test_calibration_guarantee_on_exchangeable_frames():
    """Frames drawn from one distribution: the fraction of new frames accepted yet over the
    bound stays at or below alpha (averaged over calibration draws)."""
    rng = np.random.default_rng(0)
    bound, alpha = 0.25, 0.05

    def draw(n):
        est = rng.lognormal(-2.0, 0.6, n)
        actual = est * rng.lognormal(0.3, 0.5, n)
        return est, actual

    viol = []
    for _ in range(50):
        c = S.calibrate(*draw(500), bound, alpha)
        est, actual = draw(20000)
        viol.append(np.mean((est <= c["tau"]) & (actual > bound)))
    assert np.mean(viol) <= alpha
    assert 0.0 < c["calibration_accept_rate"] < 1.0


def test_geometry_key_distinguishes_setups():
    a, b = synth.cfg4_geometry(), synth.cfg2_geometry()
    assert S.geometry_key(a) != S.geometry_key(b)
    assert S.geometry_key(a) == S.geometry_key(synth.cfg4_geometry())
    assert S.geometry_key(a) != S.geometry_key(a.replace(n_x=128))
