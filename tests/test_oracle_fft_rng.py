"""Pins of the oracle's transform, generator and cosmology helpers.

Each check compares the oracle with something other than itself: the
definition evaluated by brute force, numpy's FFT and Philox, scipy quadrature,
closed-form limits, and numbers printed in the paper (tests/golden).
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate, stats

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")


@pytest.mark.parametrize("n", [6, 8])
def test_fft3d_bruteforce_definition(n):
    """O(N^6) sum of Eq. 17's definition (three axes) against the oracle DFT."""
    rng = np.random.default_rng(n)
    a = rng.standard_normal((n, n, n)) + 1j * rng.standard_normal((n, n, n))
    j = np.arange(n)
    X = np.stack(np.meshgrid(j, j, j, indexing="ij"), -1).reshape(-1, 3)
    phase = np.exp(-2j * np.pi * (X @ X.T) / n)           # [k, x]
    want = (phase @ a.reshape(-1)).reshape(n, n, n)
    got = oracle.fft3d(a, -1)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
    back = oracle.fft3d(got, +1) / n ** 3
    assert np.abs(back - a).max() <= 1e-14 * np.abs(a).max() * n


@pytest.mark.parametrize("n", [10, 12, 32])
def test_fft3d_matches_numpy(n):
    rng = np.random.default_rng(100 + n)
    a = rng.standard_normal((n, n, n)) + 1j * rng.standard_normal((n, n, n))
    assert np.allclose(oracle.fft3d(a, -1), np.fft.fftn(a), rtol=0, atol=1e-11 * n ** 1.5)
    assert np.allclose(oracle.fft3d(a, +1), np.fft.ifftn(a) * n ** 3, rtol=0, atol=1e-11 * n ** 1.5)


def test_parseval_and_half_layout():
    n = 16
    f = np.random.default_rng(3).standard_normal((n, n, n))
    F = oracle.forward(f)
    assert F.shape == (n, n, n // 2 + 1)
    w = np.full(F.shape, 2.0)
    w[:, :, 0] = 1.0
    w[:, :, n // 2] = 1.0
    # sum_x f^2 = N^3 sum_k |F|^2 for the N^-3 forward normalisation
    assert math.isclose((f * f).sum(), n ** 3 * (w * np.abs(F) ** 2).sum(), rel_tol=1e-12)
    assert np.allclose(F, np.fft.rfftn(f) / n ** 3, atol=1e-15)


@pytest.mark.parametrize("ctr,key", [(0, 0), (5, 2 ** 64 - 1), ([2 ** 64 - 2, 7, 9, 2 ** 63], [123456789, 987654321])])
def test_philox_matches_numpy(ctr, key):
    """numpy's Philox bit generator (4x64, 10 rounds) increments its counter
    before each block, so its first block is Philox(counter + 1, key)."""
    c = list(ctr) if isinstance(ctr, list) else [ctr]
    c += [0] * (4 - len(c))
    k = list(key) if isinstance(key, list) else [key]
    k += [0] * (2 - len(k))
    bg = np.random.Philox(counter=np.array(c, dtype=np.uint64), key=np.array(k, dtype=np.uint64))
    want = bg.random_raw(4)
    # counter + 1 with carry across the four 64-bit words
    v = sum(c[i] << (64 * i) for i in range(4)) + 1
    c1 = [(v >> (64 * i)) & (2 ** 64 - 1) for i in range(4)]
    got = oracle.philox4x64_10(c1, k)
    assert [int(x) for x in got] == [int(x) for x in want]


def test_unit_gaussian_statistics():
    """Box-Muller on Philox uniforms: N(0, 1) by a KS test, and cells of
    different seeds or streams are independent (no correlation)."""
    m = 40000
    g = np.array([oracle.unit_gaussian(11, 0, c) for c in range(m)])
    assert stats.kstest(g, "norm").pvalue > 1e-3
    h = np.array([oracle.unit_gaussian(12, 0, c) for c in range(m)])
    s = np.array([oracle.unit_gaussian(11, 1, c) for c in range(m)])
    assert abs(np.corrcoef(g, h)[0, 1]) < 5.0 / math.sqrt(m)
    assert abs(np.corrcoef(g, s)[0, 1]) < 5.0 / math.sqrt(m)


def test_bbks_limits():
    # small-q expansion: T = 1 - (2.34 / 2 + 3.89 / 4) q + O(q^2)
    for q in (1e-9, 1e-7):
        assert abs(oracle.bbks(q) - (1.0 - (1.17 + 0.9725) * q)) < 100 * q * q + 1e-15
    qs = np.logspace(-4, 3, 50)
    t = np.array([oracle.bbks(q) for q in qs])
    assert np.all(np.diff(t) < 0)
    # large-q asymptote: ln(2.34 q) / (2.34 q) (6.71 q)^-1
    q = 1e6
    assert math.isclose(oracle.bbks(q), math.log(1 + 2.34 * q) / (2.34 * q) / (6.71 * q), rel_tol=1e-4)


def test_sigma_r_matches_scipy():
    amp, ns, gam = 1.0, 0.96, 0.21

    def integrand(lnk):
        k = math.exp(lnk)
        x = k * 8.0
        w = 3.0 * (math.sin(x) - x * math.cos(x)) / x ** 3
        return k ** 3 * oracle.p0(k, amp, ns, gam) * w * w / (2 * math.pi ** 2)

    val, _ = integrate.quad(integrand, math.log(1e-6), math.log(1e4), limit=2000, epsabs=0, epsrel=1e-11)
    assert math.isclose(oracle.sigma_r(8.0, amp, ns, gam), math.sqrt(val), rel_tol=1e-9)
    a8 = oracle.sigma8_amp(0.8, ns, gam)
    assert math.isclose(oracle.sigma_r(8.0, a8, ns, gam), 0.8, rel_tol=1e-12)


def test_growth_eds_and_lcdm():
    for z in (0.0, 1.0, 3.0):
        assert math.isclose(oracle.growth(1.0, 0.0, z), 1.0 / (1.0 + z), rel_tol=1e-10)
    om, ol = 0.279, 0.721

    def d(a):
        e = lambda x: math.sqrt(om / x ** 3 + ol)
        v, _ = integrate.quad(lambda x: 1.0 / (x * e(x)) ** 3, 0, a, epsabs=0, epsrel=1e-12)
        return e(a) * v

    assert math.isclose(oracle.growth(om, ol, 1.0), d(0.5) / d(1.0), rel_tol=1e-9)


def test_paper_printed_constants():
    g = json.load(open(GOLDEN))
    kc = g["k_crit"]
    assert round(2 * math.pi / kc["L"] * kc["N"] / 3, 2) == kc["value"]
    km = g["k_min"]
    assert float("%.3g" % (2 * math.pi / km["L"])) == km["value"]
    kn = g["k_nyq_particles"]
    assert round(math.pi / (kn["L"] / kn["N"]), 3) == kn["value"]
    # the paper's cut k_cut2 exceeds k_crit, so the default cut aliases
    cuts = g["cuts_default"]
    n2_crit = oracle.cut_n2max_strict(cuts["N"])
    assert oracle.cut_n2max_abs(cuts["N"], cuts["L"], cuts["k_cut2"]) > n2_crit
    assert oracle.cut_n2max_abs(cuts["N"], cuts["L"], cuts["k_cut1"]) < n2_crit


def test_strict_cut_and_edges_integer_rules():
    for n in (6, 8, 64, 192, 256, 1024):
        c = oracle.cut_n2max_strict(n)
        # largest n^2 strictly below (N/3)^2, exact rationals
        assert 9 * c < n * n <= 9 * (c + 1)
    e = oracle.linear_edges(32, 64, 3, oracle.cut_n2max_strict(64))
    assert e[0] == 1 and e[-1] == oracle.cut_n2max_strict(64) + 1
    assert np.all(np.diff(e) >= 0)
    # edge b is the smallest integer n^2 with sqrt(n^2) >= b * dk / kF, exactly
    from fractions import Fraction
    for b in range(1, 32):
        t = Fraction(b * 64, 3 * 32) ** 2
        assert e[b] >= t and e[b] - 1 < t
