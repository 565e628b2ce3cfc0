"""Pins of the oracle's recursion (Eq. 10, 11) in both source forms.

- closed form: two plane waves give the textbook F2 / G2 kernels at order 2;
- brute force: the Fourier-space recursion as explicit mode-pair sums on 8^3,
  with per-pair coefficients derived from Eq. 10 (P-form) and from its
  divergence rewriting (D-form), including cuts wide enough to alias;
- the planar (1D) Zel'dovich series, which SPT reproduces order by order;
- invariants: P = D without aliasing, exact homogeneity, translations,
  axis permutations, zero k = 0 mode.
"""
import math

import numpy as np
import pytest

import oracle
from tests import inputs


def half_value(h, n, m):
    """value of a half-layout spectrum at signed integer mode m"""
    a, b, c = m
    if c < 0:
        return np.conj(h[(-a) % n, (-b) % n, -c])
    return h[a % n, b % n, c]


def f2(q1, q2):
    q1, q2 = np.asarray(q1, float), np.asarray(q2, float)
    a, b = np.linalg.norm(q1), np.linalg.norm(q2)
    mu = q1 @ q2 / (a * b)
    return 5.0 / 7.0 + 0.5 * mu * (a / b + b / a) + 2.0 / 7.0 * mu * mu


def g2(q1, q2):
    q1, q2 = np.asarray(q1, float), np.asarray(q2, float)
    a, b = np.linalg.norm(q1), np.linalg.norm(q2)
    mu = q1 @ q2 / (a * b)
    return 3.0 / 7.0 + 0.5 * mu * (a / b + b / a) + 4.0 / 7.0 * mu * mu


@pytest.mark.parametrize("form", ["D", "P"])
def test_two_plane_waves_give_F2_G2(form):
    n, box = 32, 100.0
    k1, k2 = np.array([2, 1, 0]), np.array([1, -3, 2])
    a1, a2 = 0.3, 0.2
    d1 = inputs.plane_waves(n, [(a1, k1), (a2, k2)])
    cut = oracle.cut_n2max_strict(n)
    _, _, dk, tk = oracle.orders(d1, box, 2, cut, cut, form=form)
    d2, t2 = dk[1], tk[1]
    tol = 1e-14
    for s in (+1, -1):
        q2 = s * k2
        assert abs(half_value(d2, n, k1 + q2) - 0.5 * a1 * a2 * f2(k1, q2)) < tol
        assert abs(half_value(t2, n, k1 + q2) - 0.5 * a1 * a2 * g2(k1, q2)) < tol
    for a, k in ((a1, k1), (a2, k2)):
        assert abs(half_value(d2, n, 2 * k) - 0.5 * a * a) < tol     # F2(k, k) = 2
        assert abs(half_value(t2, n, 2 * k) - 0.5 * a * a) < tol     # G2(k, k) = 2
    assert d2[0, 0, 0] == 0 and t2[0, 0, 0] == 0                     # F2(k, -k) = 0
    # nothing else is excited
    allowed = {tuple(v) for s in (1, -1) for v in (s * (k1 + k2), s * (k1 - k2), 2 * s * k1, 2 * s * k2)}
    mask = np.ones(d2.shape, bool)
    for v in allowed:
        a, b, c = v
        if c >= 0:
            mask[a % n, b % n, c] = False
        if c <= 0:
            mask[(-a) % n, (-b) % n, -c] = False
    assert np.abs(d2[mask]).max() < tol and np.abs(t2[mask]).max() < tol


def _modes(n):
    i = np.fft.fftfreq(n, 1.0 / n).astype(int)
    v = np.stack(np.meshgrid(i, i, i, indexing="ij"), -1).reshape(-1, 3)
    d = np.where(v == -n // 2, 0, v)      # derivative wavenumber: zero at Nyquist
    return v, d


def bruteforce_recursion(d1, nmax, n2max1, n2max2, form):
    """Fourier-space recursion by explicit sums over mode pairs q1 + q2 = k
    (mod N).  Uses numpy's FFT for the input spectrum only."""
    n = d1.shape[0]
    v, d = _modes(n)
    n2 = (v * v).sum(1)
    M = n ** 3
    F1 = (np.fft.fftn(d1) / M).reshape(-1)
    F1 = np.where((n2 > 0) & (n2 <= n2max1), F1, 0)
    # index of q2 = k - q1 for every (k, q1)
    idx = lambda w: ((w[..., 0] % n) * n + (w[..., 1] % n)) * n + (w[..., 2] % n)
    k_ = v[:, None, :]
    q1 = v[None, :, :]
    q2 = k_ - q1
    j2 = idx(q2)
    q2s = v[j2]                      # q2 as a signed grid mode
    q1d, q2d = np.broadcast_to(d[None, :, :], q2s.shape), d[j2]
    kd = np.broadcast_to(d[:, None, :], q2s.shape)
    n2q1 = np.broadcast_to(n2[None, :], j2.shape).astype(float)
    n2q2 = n2[j2].astype(float)
    n2k = np.broadcast_to(n2[:, None], j2.shape).astype(float)
    ok = (n2q1 > 0) & (n2q2 > 0)
    safe1, safe2 = np.where(ok, n2q1, 1), np.where(ok, n2q2, 1)
    dot12 = (q1d * q2d).sum(-1)
    if form == "D":
        c_alpha = (kd * q2d).sum(-1) / safe2
        c_beta = 0.5 * n2k * dot12 / (safe1 * safe2)
    else:
        ksum = q1d + q2d                 # unwrapped q1 + q2
        c_alpha = (ksum * q2d).sum(-1) / safe2
        c_beta = dot12 ** 2 / (safe1 * safe2) + dot12 / safe1
    c_alpha, c_beta = np.where(ok, c_alpha, 0), np.where(ok, c_beta, 0)
    dks, tks = [F1], [F1]
    for order in range(2, nmax + 1):
        sd = np.zeros(M, complex)
        st = np.zeros(M, complex)
        for m in range(1, order):
            dm, tm, tnm = dks[m - 1], tks[m - 1], tks[order - m - 1]
            sd += (c_alpha * dm[None, :] * tnm[j2]).sum(1)
            st += (c_beta * tm[None, :] * tnm[j2]).sum(1)
        c = 2.0 / ((2 * order + 3) * (order - 1))
        keep = (n2 > 0) & (n2 <= n2max2)
        dks.append(np.where(keep, c * ((order + 0.5) * sd + st), 0))
        tks.append(np.where(keep, c * (1.5 * sd + order * st), 0))
    shape = (n, n, n)
    return ([x.reshape(shape)[:, :, : n // 2 + 1] for x in dks],
            [x.reshape(shape)[:, :, : n // 2 + 1] for x in tks])


@pytest.mark.parametrize("form", ["D", "P"])
@pytest.mark.parametrize("n2max1,n2max2", [(7, 7), (9, 9), (5, 9), (11, 6)])
def test_bruteforce_fourier_recursion_8cubed(form, n2max1, n2max2):
    n, box, nmax = 8, 50.0, 5
    d1 = inputs.band_limited(n, 42 + n2max1, 3, amp=0.5)
    _, _, dk, tk = oracle.orders(d1, box, nmax, n2max1, n2max2, form=form)
    bd, bt = bruteforce_recursion(d1, nmax, n2max1, n2max2, form)
    for o in range(nmax):
        scale = max(np.abs(bd[o]).max(), 1e-300)
        assert np.abs(dk[o] - bd[o]).max() <= 1e-13 * scale, (form, o + 1)
        assert np.abs(tk[o] - bt[o]).max() <= 1e-13 * max(np.abs(bt[o]).max(), 1e-300), (form, o + 1)


def test_forms_differ_under_aliasing():
    """With a cut wider than the 2/3 rule the two source forms differ (the
    aliased mode pairs carry different coefficients)."""
    n, box = 8, 50.0
    d1 = inputs.band_limited(n, 7, 3, amp=0.5)
    _, _, dD, _ = oracle.orders(d1, box, 3, 9, 9, form="D")
    _, _, dP, _ = oracle.orders(d1, box, 3, 9, 9, form="P")
    assert np.abs(dD[1] - dP[1]).max() > 1e-6 * np.abs(dD[1]).max()


def test_zeldovich_planar_series():
    """A planar field evolves exactly as the Zel'dovich solution before shell
    crossing: delta_n(k) = theta_n(k) = (-i k)^n / n! FT[psi^n](k) with
    psi(k) = i delta_1(k) / k (checked with numpy's 1D FFT; the band of
    delta_1 is small enough that neither the 2/3 cut nor aliasing act)."""
    n, box, nmax, band = 64, 200.0, 5, 4
    d1 = inputs.planar(n, 5, band, amp=0.3)
    cut = oracle.cut_n2max_strict(n)
    _, _, dk, tk = oracle.orders(d1, box, nmax, cut, cut, form="D")
    kF = 2 * np.pi / box
    kx = kF * np.fft.fftfreq(n, 1.0 / n)
    f1 = np.fft.fft(d1[:, 0, 0]) / n
    psik = np.where(kx != 0, 1j * f1 / np.where(kx != 0, kx, 1), 0)
    psi = np.fft.ifft(psik * n).real
    for order in range(1, nmax + 1):
        want = (-1j * kx) ** order / math.factorial(order) * np.fft.fft(psi ** order) / n
        got_d = dk[order - 1][:, 0, 0]
        got_t = tk[order - 1][:, 0, 0]
        scale = np.abs(want).max()
        assert np.abs(got_d - want).max() <= 1e-12 * scale, order
        assert np.abs(got_t - want).max() <= 1e-12 * scale, order
        rest = dk[order - 1].copy()
        rest[:, 0, 0] = 0
        assert np.abs(rest).max() <= 1e-14 * scale


def test_forms_agree_without_aliasing():
    n, box = 16, 80.0
    d1 = inputs.band_limited(n, 3, 7, amp=0.6)
    cut = oracle.cut_n2max_strict(n)
    dD, tD, _, _ = oracle.orders(d1, box, 5, cut, cut, form="D", spectra=False)
    dP, tP, _, _ = oracle.orders(d1, box, 5, cut, cut, form="P", spectra=False)
    for o in range(5):
        assert np.linalg.norm(dD[o] - dP[o]) <= 1e-13 * np.linalg.norm(dD[o])
        assert np.linalg.norm(tD[o] - tP[o]) <= 1e-13 * np.linalg.norm(tD[o])


@pytest.mark.parametrize("form", ["D", "P"])
def test_homogeneity_is_exact(form):
    """delta_n[2 delta_1] = 2^n delta_n[delta_1] bit for bit (powers of two)."""
    n, box = 16, 80.0
    d1 = inputs.band_limited(n, 9, 6, amp=0.4)
    cut = oracle.cut_n2max_strict(n)
    a, b, _, _ = oracle.orders(d1, box, 5, cut, cut, form=form, spectra=False)
    a2, b2, _, _ = oracle.orders(2 * d1, box, 5, cut, cut, form=form, spectra=False)
    for o in range(5):
        assert np.array_equal(a2[o], a[o] * 2.0 ** (o + 1))
        assert np.array_equal(b2[o], b[o] * 2.0 ** (o + 1))


def test_translation_and_axis_permutation_commute():
    n, box = 16, 80.0
    d1 = inputs.band_limited(n, 13, 6, amp=0.4)
    cut = oracle.cut_n2max_strict(n)
    a, b, _, _ = oracle.orders(d1, box, 4, cut, cut, spectra=False)
    s, _, _, _ = oracle.orders(np.roll(d1, (3, -5, 7), axis=(0, 1, 2)), box, 4, cut, cut, spectra=False)
    p, _, _, _ = oracle.orders(np.transpose(d1, (2, 0, 1)), box, 4, cut, cut, spectra=False)
    for o in range(4):
        ref = np.linalg.norm(a[o])
        assert np.linalg.norm(np.roll(a[o], (3, -5, 7), axis=(0, 1, 2)) - s[o]) <= 1e-12 * ref
        assert np.linalg.norm(np.transpose(a[o], (2, 0, 1)) - p[o]) <= 1e-12 * ref


def test_zero_mode_and_mask():
    n, box = 16, 80.0
    d1 = inputs.white(n, 1)
    cut = oracle.cut_n2max_strict(n)
    _, _, dk, tk = oracle.orders(d1, box, 4, cut, cut)
    i = np.fft.fftfreq(n, 1.0 / n)
    nx, ny, nz = np.meshgrid(i, i, np.arange(n // 2 + 1), indexing="ij")
    outside = (nx * nx + ny * ny + nz * nz) > cut
    for o in range(4):
        assert dk[o][0, 0, 0] == 0 and tk[o][0, 0, 0] == 0
        assert np.all(dk[o][outside] == 0) and np.all(tk[o][outside] == 0)
