"""Pins of the oracle's linear field (step 1 of Sec. II C) and estimators
(Eq. 19-23): independent numpy routes to the same definitions, closed-form
triangles, and seed-ensemble statistics."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from tests import inputs


def full_spectrum(f):
    n = f.shape[0]
    return np.fft.fftn(f) / n ** 3


def signed_n2(n):
    i = np.fft.fftfreq(n, 1.0 / n)
    X, Y, Z = np.meshgrid(i, i, i, indexing="ij")
    return (X * X + Y * Y + Z * Z).astype(np.int64)


def test_power_matches_full_grid_route():
    """Half-layout weights (1 on the iz = 0, N/2 planes, else 2) against a
    plain sum over every mode of the full grid, via numpy's FFT."""
    n, box = 16, 120.0
    fs = [inputs.white(n, s) for s in (1, 2, 3)]
    fks = [oracle.forward(f) for f in fs]
    edges = np.array([1, 3, 9, 20, 40, 64, 90], dtype=np.int64)
    pairs = [(0, 0), (0, 1), (1, 0), (2, 1), (2, 2)]
    pk, km, nm = oracle.power(fks, box, pairs, edges)
    n2 = signed_n2(n)
    full = [full_spectrum(f) for f in fs]
    kF = 2 * np.pi / box
    for b in range(len(edges) - 1):
        sel = (n2 >= edges[b]) & (n2 < edges[b + 1])
        assert nm[b] == sel.sum()
        assert math.isclose(km[b], kF * np.sqrt(n2[sel]).mean(), rel_tol=1e-13)
        for p, (i, j) in enumerate(pairs):
            want = box ** 3 * np.real(full[i][sel] * np.conj(full[j][sel])).mean()
            assert math.isclose(pk[p, b], want, rel_tol=1e-11, abs_tol=1e-14 * box ** 3)
    assert np.allclose(pk[1], pk[2], rtol=1e-15, atol=0)


def _numpy_gaussian(seed, stream, cell):
    """Box-Muller on words from numpy's Philox at counter (cell // 4, stream, 0, 0):
    word pair cell % 4 // 2, cosine branch for even cells, sine for odd."""
    v = (cell >> 2) + (stream << 64) - 1   # numpy steps the counter once before drawing
    v %= 1 << 256
    ctr = np.array([(v >> (64 * i)) & (2 ** 64 - 1) for i in range(4)], dtype=np.uint64)
    w = np.random.Philox(counter=ctr, key=np.array([seed, 0], dtype=np.uint64)).random_raw(4)
    pair, branch = (cell >> 1) & 1, cell & 1
    u1 = ((int(w[2 * pair]) >> 11) + 0.5) * 2.0 ** -53
    u2 = ((int(w[2 * pair + 1]) >> 11) + 0.5) * 2.0 ** -53
    r = math.sqrt(-2.0 * math.log(u1))
    return r * (math.sin(2.0 * math.pi * u2) if branch else math.cos(2.0 * math.pi * u2))


def test_linear_field_noise_and_amplitude():
    """delta_1(k) = W1 sqrt(P0 N^3 / L^3) D w(k) with w(x) rebuilt from numpy's
    Philox and transformed by numpy's FFT."""
    n, box, seed, stream = 8, 100.0, 77, 3
    amp, ns, gam, dz = 2.0e4, 0.96, 0.21, 0.7
    cut = oracle.cut_n2max_strict(n) + 2
    d1 = oracle.linear_field(n, box, amp, ns, gam, dz, cut, seed, stream)
    w = np.array([_numpy_gaussian(seed, stream, c) for c in range(n ** 3)]).reshape(n, n, n)
    wk = full_spectrum(w)
    n2 = signed_n2(n)
    k = 2 * np.pi / box * np.sqrt(n2)
    p0 = np.vectorize(lambda x: oracle.p0(x, amp, ns, gam))(k)
    want = np.where((n2 > 0) & (n2 <= cut), wk * np.sqrt(p0 * n ** 3 / box ** 3) * dz, 0)
    got = full_spectrum(d1)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def test_linear_field_power_statistics():
    """Seed ensemble: L^3 |delta_1(k)|^2 / (D^2 P0) is Exp(1) distributed on
    every kept mode, so its shell means are 1 within Poisson errors."""
    n, box, amp, ns, gam, dz = 16, 300.0, 1.0e4, 0.96, 0.21, 0.5
    cut = oracle.cut_n2max_strict(n)
    nb = 4
    edges = oracle.linear_edges(nb, n, 3, cut)
    kF = 2 * np.pi / box
    acc = np.zeros(nb)
    nseed = 24
    for s in range(nseed):
        d1 = oracle.linear_field(n, box, amp, ns, gam, dz, cut, 1000 + s)
        fk = oracle.forward(d1)
        pk, km, nm = oracle.power([fk], box, [(0, 0)], edges)
        acc += pk[0]
    # compare with the shell average of D^2 P0 over the same modes
    n2 = signed_n2(n)
    ratio = []
    for b in range(nb):
        sel = (n2 >= edges[b]) & (n2 < edges[b + 1])
        p0m = np.mean([oracle.p0(kF * math.sqrt(x), amp, ns, gam) for x in n2[sel]]) * dz * dz
        # a mode and its mirror are one complex Gaussian: nm / 2 independent values
        sigma = p0m / math.sqrt(nseed * sel.sum() / 2.0)
        ratio.append((acc[b] / nseed - p0m) / sigma)
    chi2 = float(np.sum(np.square(ratio)))
    assert stats.chi2.sf(chi2, nb) > 1e-3, ratio


def _shell_index(n, edges):
    n2 = signed_n2(n)
    b = np.full(n2.shape, -1)
    for i in range(len(edges) - 1):
        b[(n2 >= edges[i]) & (n2 < edges[i + 1])] = i
    return b


def test_bispectrum_plane_wave_triangle():
    """Three plane waves closing a triangle: the only closed triangles are
    (q1, q2, q3) and its mirror, so T = 2 Re(a1 a2 a3)."""
    n, box = 12, 60.0
    q1, q2 = np.array([1, 0, 0]), np.array([0, 2, 0])
    q3 = -(q1 + q2)
    a = [0.3 + 0.1j, -0.2 + 0.4j, 0.25 - 0.05j]
    h = np.zeros((n, n, n // 2 + 1), complex)
    for amp, q in zip(a, (q1, q2, q3)):
        for v, val in ((q, amp), (-q, np.conj(amp))):
            x, y, z = v
            if z >= 0:          # the half layout keeps iz >= 0; the z = 0 plane keeps both mirrors
                h[x % n, y % n, z] += val
    edges = np.array([1, 2, 5, 6], dtype=np.int64)        # shells: n2=1 | 2..4 | 5
    bk, nt = oracle.bispectrum([h], box, [(0, 1, 2)], [(0, 0, 0, 0)], edges)
    # count ordered triangles by brute force over the grid
    sh = _shell_index(n, edges).reshape(-1)
    i = np.fft.fftfreq(n, 1.0 / n).astype(int)
    v = np.stack(np.meshgrid(i, i, i, indexing="ij"), -1).reshape(-1, 3)
    A = v[sh == 0]
    B = v[sh == 1]
    C = -(A[:, None, :] + B[None, :, :])
    c2 = (C * C).sum(-1)
    count = ((c2 >= 5) & (c2 < 6)).sum()
    assert nt[0] == count
    want = box ** 6 * 2 * np.real(a[0] * a[1] * a[2]) / count
    assert math.isclose(bk[0], want, rel_tol=1e-12)


def test_bispectrum_matches_fft_estimator():
    """Direct triangle enumeration against the FFT estimator
    T = N^-3 sum_x I_a I_b I_c with I = inverse transform of a shell-filtered
    spectrum (numpy FFT); exact when every shell lies below N/3."""
    n, box = 12, 80.0
    fs = [inputs.band_limited(n, 20 + s, 5, amp=1.0) for s in range(3)]
    fks = [oracle.forward(f) for f in fs]
    edges = np.array([1, 4, 8, 13, 17], dtype=np.int64)
    tris = [(0, 0, 0), (1, 1, 1), (2, 2, 2), (1, 1, 0), (3, 3, 0), (0, 1, 2), (2, 3, 1)]
    terms = [(0, 0, 0, 0), (0, 1, 2, 1), (2, 1, 0, 2), (1, 1, 2, 3), (0, 2, 1, 4), (0, 1, 2, 5), (2, 2, 0, 6)]
    bk, nt = oracle.bispectrum(fks, box, tris, terms, edges)
    sh = _shell_index(n, edges)
    full = [full_spectrum(f) for f in fs]

    def inv(spec, b):
        return np.fft.ifftn(np.where(sh == b, spec, 0)).real * n ** 3

    for t, (b1, b2, b3) in enumerate(tris):
        J = [inv(np.ones_like(full[0]), b) for b in (b1, b2, b3)]
        cnt = (J[0] * J[1] * J[2]).sum() / n ** 3
        assert abs(nt[t] - cnt) < 1e-6 * max(cnt, 1)
    for u, (fa, fb, fc, t) in enumerate(terms):
        b1, b2, b3 = tris[t]
        T = (inv(full[fa], b1) * inv(full[fb], b2) * inv(full[fc], b3)).sum() / n ** 3
        want = box ** 6 * T / nt[t]
        assert math.isclose(bk[u], want, rel_tol=1e-9, abs_tol=1e-12 * abs(want)), u


def test_sum_orders():
    d = np.random.default_rng(0).standard_normal((3, 4, 4, 4))
    c = [1.0, 0.5, 0.25]
    assert np.allclose(oracle.sum_orders(d, c), d[0] + 0.5 * d[1] + 0.25 * d[2], atol=1e-15)
