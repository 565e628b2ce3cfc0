"""Seeded synthetic inputs shared by the oracle tests and the GPU parity tests.

Holds no arithmetic of the method itself: white noise, band-limited random
fields and plane waves built with numpy's own generator and FFT.
"""
from __future__ import annotations

import numpy as np


def white(n: int, seed: int) -> np.ndarray:
    """Unit-variance white noise on an n^3 grid."""
    return np.random.default_rng(seed).standard_normal((n, n, n))


def band_limited(n: int, seed: int, nmax_abs: int, amp: float = 1.0, slope: float = -1.5) -> np.ndarray:
    """Real random field whose modes satisfy |n_i| <= nmax_abs (cube) with
    power ~ |n|^slope; zero mean."""
    rng = np.random.default_rng(seed)
    f = rng.standard_normal((n, n, n))
    fk = np.fft.rfftn(f)
    i = np.fft.fftfreq(n, 1.0 / n)
    iz = np.arange(n // 2 + 1)
    nx, ny, nz = np.meshgrid(i, i, iz, indexing="ij")
    keep = (np.abs(nx) <= nmax_abs) & (np.abs(ny) <= nmax_abs) & (nz <= nmax_abs)
    r2 = nx * nx + ny * ny + nz * nz
    with np.errstate(divide="ignore"):
        shape = np.where(r2 > 0, r2 ** (slope / 4.0), 0.0)
    fk = fk * keep * shape
    out = np.fft.irfftn(fk, s=(n, n, n), axes=(0, 1, 2))
    out *= amp / max(out.std(), 1e-300)
    return out


def plane_waves(n: int, waves) -> np.ndarray:
    """sum_i A_i cos(2 pi (m_i . j) / n) for integer mode vectors m_i."""
    j = np.arange(n)
    X, Y, Z = np.meshgrid(j, j, j, indexing="ij")
    out = np.zeros((n, n, n))
    for a, m in waves:
        out += a * np.cos(2.0 * np.pi * (m[0] * X + m[1] * Y + m[2] * Z) / n)
    return out


def planar(n: int, seed: int, band: int, amp: float = 0.1) -> np.ndarray:
    """Field varying along x only, modes |n_x| <= band, zero mean."""
    rng = np.random.default_rng(seed)
    c = np.zeros(n // 2 + 1, dtype=np.complex128)
    c[1: band + 1] = rng.standard_normal(band) + 1j * rng.standard_normal(band)
    f = np.fft.irfft(c, n)
    f *= amp / f.std()
    return np.broadcast_to(f[:, None, None], (n, n, n)).copy()
