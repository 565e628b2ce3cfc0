"""Helpers of the full-size GPU checks against the sparse Fourier-space
oracle: plane-wave inputs made on the GPU, their spectrum, and the relative
L2 error of a cube-layout spectrum against a sparse expectation (numpy and
torch only; no arithmetic of the method)."""
import math

import numpy as np
import torch


def plane_field(n, waves, dtype):
    """sum of A cos(2 pi m.x / N + phi) on the GPU (torch, FP64, slab by slab)"""
    out = torch.empty((n, n, n), dtype=dtype, device="cuda")
    j = torch.arange(n, device="cuda", dtype=torch.int64)
    slab = 32
    for x0 in range(0, n, slab):
        xs = j[x0:x0 + slab].view(-1, 1, 1)
        acc = torch.zeros((xs.shape[0], n, n), dtype=torch.float64, device="cuda")
        for amp, phase, m in waves:
            e = (m[0] * xs + m[1] * j.view(1, -1, 1) + m[2] * j.view(1, 1, -1)) % n
            acc += amp * torch.cos(e.to(torch.float64) * (2 * math.pi / n) + phase)
        out[x0:x0 + slab] = acc.to(dtype)
        del acc, e
    return out


def spectrum_of(waves):
    spec = {}
    for amp, phase, m in waves:
        v = 0.5 * amp * complex(math.cos(phase), math.sin(phase))
        spec[tuple(m)] = spec.get(tuple(m), 0) + v
        spec[tuple(-x for x in m)] = spec.get(tuple(-x for x in m), 0) + v.conjugate()
    return spec


def cube_index(kc, m):
    """(kz, ky', kx') of signed mode m in the cube, and whether m is stored or its mirror"""
    a, b, c = m
    conj = c < 0
    if conj:
        a, b, c = -a, -b, -c
    K = 2 * kc + 1
    return (c, b % K if b >= 0 else b + K, a if a >= 0 else a + K), conj


def compare_sparse(cube, kc, sparse):
    """relative L2 error of a GPU cube spectrum against a sparse expectation,
    counting energy at every mode the expectation leaves empty"""
    keys = [k for k in sparse if k[2] > 0 or (k[2] == 0)]
    idx = [cube_index(kc, k)[0] for k in keys]
    t = torch.tensor(idx, device="cuda", dtype=torch.int64)
    vals = cube[t[:, 0], t[:, 1], t[:, 2]].double().cpu().numpy()
    got = vals[:, 0] + 1j * vals[:, 1]
    want = np.array([sparse[k] for k in keys])
    w = np.array([1.0 if k[2] == 0 else 2.0 for k in keys])
    c = cube.double()
    e2 = (c[..., 0] ** 2 + c[..., 1] ** 2)
    # the energy off the expected modes, summed directly (the difference of the total
    # and the on-mode energy would cancel to about 1e-16 of the total, i.e. an error
    # floor near 1e-8 after the square root)
    e2[t[:, 0], t[:, 1], t[:, 2]] = 0.0
    leak = float(e2[0].sum() + 2.0 * e2[1:].sum())
    err2 = float((w * np.abs(got - want) ** 2).sum()) + leak
    ref2 = float((w * np.abs(want) ** 2).sum())
    return math.sqrt(err2 / ref2)
