"""Pins of the oracle's field statistics (oracle/stats.py)."""
import numpy as np
import pytest
from scipy import stats as sps

from oracle import stats


def test_smoothing_plane_wave_closed_form():
    """W(kR) on a single Fourier pair: cos(k.x) -> exp(-k^2 R^2 / 2) cos(k.x)."""
    n, box, R = 16, 100.0, 7.0
    x = np.arange(n) * box / n
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    kv = 2 * np.pi / box * np.array([2, -1, 3])
    f = np.cos(kv[0] * X + kv[1] * Y + kv[2] * Z)
    fk = np.fft.rfftn(f) / n ** 3
    got = stats.smooth([fk], [1.0], R, box)[0]
    want = np.exp(-0.5 * (kv @ kv) * R * R) * f
    assert np.max(np.abs(got - want)) < 1e-14


def test_smoothing_cumulative_is_linear():
    n, box, R = 12, 60.0, 3.0
    rng = np.random.default_rng(0)
    fs = [np.fft.rfftn(rng.standard_normal((n, n, n))) / n ** 3 for _ in range(3)]
    c = [0.5, 0.25, 0.125]
    cum = stats.smooth(fs, c, R, box, cumulative=True)
    sep = stats.smooth(fs, c, R, box, cumulative=False)
    for j in range(3):
        assert np.allclose(cum[j], sum(sep[: j + 1]), atol=1e-14)
    # R = 0 gives the unsmoothed field back
    raw = stats.smooth([fs[0]], [1.0], 0.0, box)[0]
    assert np.allclose(np.fft.rfftn(raw) / n ** 3, fs[0], atol=1e-15)


def test_moments_and_correlation_against_library():
    rng = np.random.default_rng(1)
    a = rng.gamma(2.0, size=(8, 8, 8)) - 1.0
    b = 0.3 * a + rng.standard_normal((8, 8, 8))
    m = stats.moments([a, b])
    for f, row in zip((a, b), m):
        x = f.ravel()
        assert np.isclose(row[0], x.mean(), rtol=1e-14)
        assert np.isclose(row[1], x.var(), rtol=1e-13)
        assert np.isclose(row[2], sps.skew(x), rtol=1e-12)
        assert np.isclose(row[3], sps.kurtosis(x), rtol=1e-12)
    r = stats.correlation([a, b, -a])
    assert np.isclose(r[0, 1], sps.pearsonr(a.ravel(), b.ravel())[0], rtol=1e-12)
    assert np.isclose(r[0, 2], -1.0, atol=1e-15) and np.isclose(r[1, 1], 1.0, atol=1e-15)
    # a small example by hand: {-1, 0, 0, 1, 5}
    v = np.array([-1.0, 0.0, 0.0, 1.0, 5.0])
    mm = stats.moments([v])[0]
    assert np.isclose(mm[0], 1.0) and np.isclose(mm[1], (4 + 1 + 1 + 0 + 16) / 5)


def test_histograms_by_counting():
    rng = np.random.default_rng(2)
    x = rng.uniform(-1.5, 1.5, size=500)
    x[:4] = [-1.0, 1.0, -1.0 + 0.25, 0.999999999]  # on the lower edge, on hi, on an inner edge, just below hi
    lo, hi, nb = -1.0, 1.0, 8
    h = stats.histogram(x, lo, hi, nb)
    want = np.zeros(nb)
    for v in x:
        if lo <= v < hi:
            want[int((v - lo) // 0.25)] += 1
    assert np.array_equal(h, want)
    y = rng.uniform(-1.5, 1.5, size=500)
    j = stats.joint_histogram(x, y, lo, hi, 4)
    want = np.zeros((4, 4))
    for u, v in zip(x, y):
        if lo <= u < hi and lo <= v < hi:
            want[int((u - lo) // 0.5), int((v - lo) // 0.5)] += 1
    assert np.array_equal(j, want)
