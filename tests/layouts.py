"""Host-side layout conversions for comparing GPU cube spectra with the
oracle's half-layout spectra (numpy only)."""
from __future__ import annotations

import numpy as np


def cube_positions(n: int, kc: int) -> np.ndarray:
    """grid position of each fftfreq index of a (2kc+1)-long axis"""
    i = np.arange(2 * kc + 1)
    return np.where(i <= kc, i, n - (2 * kc + 1) + i)


def half_to_cube(h: np.ndarray, kc: int) -> np.ndarray:
    """[ix, iy, iz] half layout -> [kz, ky, kx] cube layout (complex)."""
    n = h.shape[0]
    p = cube_positions(n, kc)
    sub = h[np.ix_(p, p, np.arange(kc + 1))]          # [kx, ky, kz]
    return np.ascontiguousarray(np.transpose(sub, (2, 1, 0)))


def cube_from_tensor(t) -> np.ndarray:
    """cube tensor [..., 2] (real) -> complex numpy array"""
    a = t.detach().cpu().numpy()
    return a[..., 0] + 1j * a[..., 1]


def cube_to_tensor_array(c: np.ndarray, dtype) -> np.ndarray:
    return np.ascontiguousarray(np.stack([c.real, c.imag], -1).astype(dtype))


def rel_l2(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / (den if den > 0 else 1.0))
