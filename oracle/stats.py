"""Field-level statistics of the GridSPT fields -- TEST INFRASTRUCTURE ONLY.

Plain FP64 numpy definitions (only tests/, the package smoke entry and the
benchmark's CPU-baseline leg use this module), for the smoothed density
fields and the one-point statistics of Sec. III A-B:
  * Gaussian smoothing W(kR) = exp(-k^2 R^2 / 2) of spectra, optionally of the
    cumulative sums delta_SPT^(n) = sum_{i <= n} c_i delta_i (the truncated
    series of Eq. 8 with c_i = D^i);
  * mean, variance, skewness and excess kurtosis of each field; the Pearson
    correlation coefficient between fields (the cross-correlation of Sec. III B
    between fields on the same grid);
  * histograms of one field and joint histograms of a reference field with
    each other field (the one-point and joint PDFs of Sec. III B), with bin
    b = floor((x - lo) * nbins / (hi - lo)), values outside [0, nbins) dropped.
"""
from __future__ import annotations

import numpy as np


def _full_k2(n: int):
    i = np.fft.fftfreq(n, 1.0 / n)
    iz = np.arange(n // 2 + 1)
    nx, ny, nz = np.meshgrid(i, i, iz, indexing="ij")
    return nx * nx + ny * ny + nz * nz


def smooth(fields_k, coef, radius: float, box: float, cumulative: bool = True):
    """Real fields F^-1[W(kR) S_j(k)] for S_j = sum_{i <= j} coef_i F_i (cumulative)
    or S_j = coef_j F_j; fields_k are half-layout spectra [N, N, N/2 + 1]."""
    n = fields_k[0].shape[0]
    kf = 2.0 * np.pi / box
    w = np.exp(-0.5 * (kf * kf) * _full_k2(n) * radius * radius)
    out = []
    acc = np.zeros_like(fields_k[0], dtype=np.complex128)
    for c, f in zip(coef, fields_k):
        s = c * np.asarray(f, dtype=np.complex128)
        if cumulative:
            acc = acc + s
            s = acc
        # f(x) = sum_k F(k) e^{ik.x}: numpy's inverse carries 1/N^3
        out.append(np.fft.irfftn(w * s, s=(n, n, n), axes=(0, 1, 2)) * n ** 3)
    return out


def moments(fields):
    """[nfields, 4]: mean, variance (1/N), skewness, excess kurtosis."""
    res = []
    for f in fields:
        x = np.asarray(f, dtype=np.float64).ravel()
        m = x.mean()
        d = x - m
        v = (d * d).mean()
        res.append([m, v, (d ** 3).mean() / v ** 1.5, (d ** 4).mean() / v ** 2 - 3.0])
    return np.array(res)


def correlation(fields):
    """[nfields, nfields] Pearson r."""
    x = np.stack([np.asarray(f, dtype=np.float64).ravel() for f in fields])
    return np.corrcoef(x)


def bins_of(x, lo: float, hi: float, nbins: int):
    """Bin index of every value (int64), -1 outside [lo, hi)."""
    scale = nbins / (hi - lo)
    b = np.floor((np.asarray(x, dtype=np.float64).ravel() - lo) * scale)
    b = np.where((b >= 0) & (b < nbins), b, -1)
    return b.astype(np.int64)


def histogram(x, lo: float, hi: float, nbins: int):
    b = bins_of(x, lo, hi, nbins)
    return np.bincount(b[b >= 0], minlength=nbins).astype(np.float64)


def joint_histogram(ref, x, lo: float, hi: float, nbins: int):
    """[nbins (ref), nbins (x)] counts of cells with both values in range."""
    a = bins_of(ref, lo, hi, nbins)
    b = bins_of(x, lo, hi, nbins)
    ok = (a >= 0) & (b >= 0)
    return np.bincount(a[ok] * nbins + b[ok], minlength=nbins * nbins).reshape(nbins, nbins).astype(np.float64)
