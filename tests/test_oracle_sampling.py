"""Pins of the oracle's sampling routines used for full-size GPU checks:
the direct-DFT linear modes and the sparse Fourier-space recursion, both
against the dense oracle (itself pinned in the other oracle tests)."""
import numpy as np
import pytest

import oracle
from tests import inputs


def test_linear_modes_match_dense_oracle():
    n, box, seed, stream = 16, 150.0, 9, 2
    amp, ns, gam, dz = 3.0e4, 0.96, 0.21, 0.8
    cut = oracle.cut_n2max_strict(n)
    d1 = oracle.linear_field(n, box, amp, ns, gam, dz, cut, seed, stream)
    full = np.fft.fftn(d1) / n ** 3
    modes = [(1, 0, 0), (0, -2, 3), (3, 3, -2), (-4, 1, 1), (0, 0, 0), (5, 5, 5)]
    got = oracle.linear_modes(n, box, amp, ns, gam, dz, cut, seed, modes, stream)
    for (a, b, c), v in zip(modes, got):
        want = full[a % n, b % n, c % n]
        assert abs(v - want) <= 1e-12 * max(abs(want), np.abs(full).max() * 1e-3), (a, b, c)
    assert got[4] == 0 and got[5] == 0          # k = 0 and a masked mode


def _plane_wave_spectrum(waves):
    spec = {}
    for amp, phase, m in waves:
        m = tuple(int(x) for x in m)
        v = 0.5 * amp * np.exp(1j * phase)
        spec[m] = spec.get(m, 0) + v
        mm = tuple(-x for x in m)
        spec[mm] = spec.get(mm, 0) + np.conj(v)
    return spec


def _field_from_waves(n, waves):
    j = np.arange(n)
    X, Y, Z = np.meshgrid(j, j, j, indexing="ij")
    out = np.zeros((n, n, n))
    for amp, phase, m in waves:
        out += amp * np.cos(2 * np.pi * (m[0] * X + m[1] * Y + m[2] * Z) / n + phase)
    return out


# low modes: on 32^3 no sum of up to five of them leaves |n_i| < 16, so nothing wraps
WAVES32 = [(0.3, 0.2, (1, 2, 0)), (0.2, -1.1, (0, -1, 3)), (0.25, 2.0, (2, 0, -1)), (0.15, 0.7, (3, 1, 1))]
# modes near the cut (|n|^2 <= 100): sums of two or three wrap and land inside the wider output
# cuts, e.g. (10, 0, 0) + (10, 0, 0) = (20, 0, 0), which is (-12, 0, 0) on the grid
WAVES32_ALIAS = [(0.3, 0.2, (10, 0, 0)), (0.2, -1.1, (-7, 6, 1)), (0.25, 2.0, (2, -3, 8)), (0.15, 0.7, (8, 1, -5))]
CUTS32 = {"wide": (150, 200),
          # the paper's cuts on 512^3 (1 and 4/3 h/Mpc with L = 1000: |n| <= 159 and 212, where
          # 159 + 159 wraps to -194) scaled to 32^3: |n| <= 10 and 13.2
          "paper": (100, 175)}


@pytest.mark.parametrize("form", ["D", "P"])
@pytest.mark.parametrize("cut_kind", ["strict", "wide", "paper"])
def test_sparse_recursion_matches_dense_oracle(cut_kind, form):
    """Every mode of delta_n and theta_n, n <= 5, on 32^3, in both forms of the
    sources; under the wide cuts mode sums wrap around the grid (aliasing),
    which both must treat alike."""
    n, box, nmax = 32, 100.0, 5
    if cut_kind == "strict":
        c1 = c2 = oracle.cut_n2max_strict(n)
        waves = WAVES32
    else:
        c1, c2 = CUTS32[cut_kind]
        waves = WAVES32_ALIAS
    d1 = _field_from_waves(n, waves)
    _, _, dk, tk = oracle.orders(d1, box, nmax, c1, c2, form=form)
    sd, st = oracle.sparse_orders(_plane_wave_spectrum(waves), n, nmax, c1, c2, form=form)
    for o in range(nmax):
        for dense, sparse in ((dk[o], sd[o]), (tk[o], st[o])):
            # the half layout keeps c >= 0; its c = 0 plane holds both mirrors
            want = np.zeros_like(dense)
            for (a, b, c), v in sparse.items():
                if c >= 0:
                    want[a % n, b % n, c] += v
            scale = np.abs(want).max()
            assert scale > 0
            assert np.abs(dense - want).max() <= 1e-12 * scale, o + 1


def test_sparse_forms_agree_only_without_aliasing():
    """P = D mode by mode when every kept mode lies below N/3 (a wrapped sum
    then lands outside the mask), and they differ once the cut admits wraps."""
    n, nmax = 32, 4
    c = oracle.cut_n2max_strict(n)
    for waves, cuts, equal in ((WAVES32, (c, c), True), (WAVES32_ALIAS, CUTS32["wide"], False),
                               (WAVES32_ALIAS, CUTS32["paper"], False)):
        spec = _plane_wave_spectrum(waves)
        dd, td = oracle.sparse_orders(spec, n, nmax, *cuts, form="D")
        dp, tp = oracle.sparse_orders(spec, n, nmax, *cuts, form="P")
        diff = scale = 0.0
        for o in range(1, nmax):
            for a, b in ((dd[o], dp[o]), (td[o], tp[o])):
                for k in set(a) | set(b):
                    diff = max(diff, abs(a.get(k, 0) - b.get(k, 0)))
                    scale = max(scale, abs(a.get(k, 0)))
        assert (diff <= 1e-14 * scale) == equal, (cuts, diff / scale)
