"""Field statistics on the GPU (gridspt_smooth, gridspt_field_stats) against the
oracle's plain definitions (oracle/stats.py, pinned in test_oracle_stats.py).

Smoothed fields: relative L2 1e-12 (FP64), 1e-5 (FP32).  Statistics are taken
of fields the oracle made (rounded to the grid's precision and uploaded), on
both sides, so moments and correlations agree to FP64 summation order and
histogram counts exactly.  At 512^3 (the statistics workload's size) plane
waves are smoothed and measured against the sparse Fourier-space recursion.
"""
import math
import numpy as np
import pytest
import torch

import oracle
from oracle import stats
import paper_1807_04215_amd as g
from tests.layouts import rel_l2

pytestmark = pytest.mark.gpu

NS, GAMMA = 0.96, 0.21
TOL = {g.F64: 1e-12, g.F32: 1e-5}


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available()
    return g.Context()


def _orders(ctx, n, box, nmax, dtype, seed):
    cut = g.cut_n2max(n, box)
    grid = g.Grid(n, box, g.cube_kc(cut), dtype)
    d1 = oracle.linear_field(n, box, oracle.sigma8_amp(0.8, NS, GAMMA), NS, GAMMA, 1.0, cut, seed)
    if dtype == g.F32:
        d1 = d1.astype(np.float32).astype(np.float64)
    out = g.orders(ctx, grid, nmax, cut, cut, torch.from_numpy(d1).to("cuda", grid.real_dtype))
    ref = oracle.orders(d1, box, nmax, cut, cut)
    return grid, out, ref


@pytest.mark.parametrize("dtype", [g.F64, g.F32])
@pytest.mark.parametrize("n,box,radius", [(32, 200.0, 12.0), (48, 300.0, 9.0), (32, 200.0, 0.0)])
def test_smooth_matches_oracle(ctx, dtype, n, box, radius):
    nmax = 5
    grid, out, (rd, rt, rdk, rtk) = _orders(ctx, n, box, nmax, dtype, 3)
    coef = [0.8 ** (i + 1) for i in range(nmax)]
    for cumulative in (True, False):
        sm = g.smooth(ctx, grid, out.delta_k, coef, radius, cumulative=cumulative)
        ctx.sync()
        ref = stats.smooth(list(rdk), coef, radius, box, cumulative=cumulative)
        for j in range(nmax):
            e = rel_l2(sm[j].cpu().numpy(), ref[j])
            assert e < TOL[dtype], (cumulative, j, e)


@pytest.mark.parametrize("dtype", [g.F64, g.F32])
def test_field_stats_match_oracle(ctx, dtype):
    """The oracle's smoothed truncated series (reference first: the highest-order
    sum), rounded to the grid's precision, uploaded, and measured on both sides."""
    n, box, nmax = 48, 300.0, 4
    cut = g.cut_n2max(n, box)
    grid = g.Grid(n, box, g.cube_kc(cut), dtype)
    d1 = oracle.linear_field(n, box, oracle.sigma8_amp(0.8, NS, GAMMA), NS, GAMMA, 1.0, cut, 5)
    _, _, rdk, _ = oracle.orders(d1, box, nmax, cut, cut)
    sm = stats.smooth(list(rdk), [1.0] * nmax, 8.0, box, cumulative=True)
    host = [sm[-1]] + list(sm[:-1])
    if dtype == g.F32:
        host = [h.astype(np.float32).astype(np.float64) for h in host]
    fields = [torch.from_numpy(np.ascontiguousarray(h)).to("cuda", grid.real_dtype) for h in host]
    mom, cor, cnt, jnt = g.field_stats(ctx, grid, fields, nbins=40, lo=-0.6, hi=0.9, nbins2=16)
    ctx.sync()
    assert np.allclose(mom.cpu().numpy(), stats.moments(host), rtol=1e-10, atol=1e-14)
    assert np.allclose(cor.cpu().numpy(), stats.correlation(host), rtol=1e-10, atol=1e-14)
    for i, h in enumerate(host):
        assert np.array_equal(cnt[i].cpu().numpy(), stats.histogram(h, -0.6, 0.9, 40)), i
    for j in range(1, len(host)):
        assert np.array_equal(jnt[j - 1].cpu().numpy(), stats.joint_histogram(host[0], host[j], -0.6, 0.9, 16)), j


def test_smooth_and_stats_512_plane_waves(ctx):
    """The statistics workload's size: 512^3, L = 1000 Mpc/h, R = 10 Mpc/h, the
    truncated series of orders 1..5 of five plane waves (FP32), against the
    sparse recursion: the smoothed series at sampled cells (a finite sum of
    smoothed modes), and the mean (zero), the variance of each truncation and
    the correlation coefficients between them (Parseval over the sparse
    spectra: var = sum_k |S(k)|^2 with the forward DFT carrying N^-3)."""
    from tests.sparse_check import plane_field, spectrum_of
    n, box, nmax, radius = 512, 1000.0, 5, 10.0
    cut = g.cut_n2max(n, box)
    grid = g.Grid(n, box, g.cube_kc(cut), g.F32)
    waves = [(0.08, 0.3, (13, -7, 2)), (0.06, -1.2, (-5, 21, 9)), (0.07, 2.1, (30, 4, -17)),
             (0.05, 0.9, (2, -3, 44)), (0.04, -2.5, (-45, 30, 11))]
    out = g.orders(ctx, grid, nmax, cut, cut, plane_field(n, waves, grid.real_dtype))
    sm = g.smooth(ctx, grid, out.delta_k, [1.0] * nmax, radius, cumulative=True)
    mom, cor, _, _ = g.field_stats(ctx, grid, sm)
    ctx.sync()
    sd, _ = oracle.sparse_orders(spectrum_of(waves), n, nmax, cut, cut)
    kf2r2 = (2.0 * math.pi / box * radius) ** 2
    acc, series = {}, []
    for j in range(nmax):
        for k, v in sd[j].items():
            acc[k] = acc.get(k, 0) + v
        series.append({k: v * math.exp(-0.5 * kf2r2 * (k[0] ** 2 + k[1] ** 2 + k[2] ** 2)) for k, v in acc.items()})
    keys = sorted(series[-1])
    spec = np.array([[s.get(k, 0) for k in keys] for s in series])   # [truncation, mode]
    var = (np.abs(spec) ** 2).sum(axis=1)
    cov = (spec @ spec.conj().T).real
    got_mom, got_cor = mom.cpu().numpy(), cor.cpu().numpy()
    assert np.allclose(got_mom[:, 1], var, rtol=2e-5, atol=0), (got_mom[:, 1], var)
    assert np.all(np.abs(got_mom[:, 0]) <= 1e-5 * np.sqrt(var))
    assert np.allclose(got_cor, cov / np.sqrt(np.outer(var, var)), rtol=0, atol=2e-5)
    # sampled cells
    rng = np.random.default_rng(12)
    cells = rng.integers(0, n, size=(64, 3))
    kv = np.array(keys, dtype=np.float64)
    phase = np.exp(2j * np.pi * (cells @ kv.T) / n)                    # [cell, mode]
    for j in range(nmax):
        want = (phase @ spec[j]).real
        t = torch.tensor(cells, device="cuda")
        have = sm[j][t[:, 0], t[:, 1], t[:, 2]].double().cpu().numpy()
        assert np.abs(have - want).max() <= 1e-5 * np.sqrt(var[j]) * 10, (j, np.abs(have - want).max())


@pytest.mark.parametrize("dtype", [g.F64, g.F32])
def test_histogram_bin_edges_exact(ctx, dtype):
    """Values on bin edges, on lo and hi, just inside and outside: the bin
    decision is the same FP64 expression on both sides."""
    n = 16
    grid = g.Grid(n, 100.0, 5, dtype)
    rng = np.random.default_rng(7)
    vals = np.concatenate([np.arange(-8, 9) / 8.0, [-1.0 - 1e-7, 1.0 - 1e-7, 0.5 + 1e-9, -0.25 - 1e-9]])
    x = rng.choice(vals, size=(n, n, n))
    if dtype == g.F32:
        x = x.astype(np.float32)
    xt = torch.from_numpy(np.ascontiguousarray(x)).to("cuda")
    y = torch.roll(xt, 3, dims=0)
    _, _, cnt, jnt = g.field_stats(ctx, grid, [xt, y], nbins=16, lo=-1.0, hi=1.0, nbins2=8)
    ctx.sync()
    xh, yh = x.astype(np.float64), y.cpu().numpy().astype(np.float64)
    assert np.array_equal(cnt[0].cpu().numpy(), stats.histogram(xh, -1.0, 1.0, 16))
    assert np.array_equal(cnt[1].cpu().numpy(), stats.histogram(yh, -1.0, 1.0, 16))
    assert np.array_equal(jnt[0].cpu().numpy(), stats.joint_histogram(xh, yh, -1.0, 1.0, 8))


def test_stats_properties_at_512(ctx):
    """At 512^3 (ragged against the block grid-stride): counts plus the values
    outside the range add up to N^3, r(a, a) = 1, r(a, -a) = -1."""
    n = 512
    grid = g.Grid(n, 1000.0, 170, g.F32)
    gen = torch.Generator(device="cuda").manual_seed(3)
    a = torch.randn((n,) * 3, generator=gen, device="cuda")
    mom, cor, cnt, _ = g.field_stats(ctx, grid, [a, -a, a], nbins=64, lo=-2.0, hi=2.0)
    ctx.sync()
    inside = int(((a >= -2.0) & (a < 2.0)).sum().item())
    assert cnt[0].sum().item() == inside
    c = cor.cpu().numpy()
    assert abs(c[0, 2] - 1.0) < 1e-12 and abs(c[0, 1] + 1.0) < 1e-12
    assert abs(mom[0, 1].item() - 1.0) < 1e-3


@pytest.mark.parametrize("dtype", [g.F64, g.F32])
def test_histograms_many_bins_and_moments_alone(ctx, dtype):
    """Eight fields and 1024 bins (the one-point counts then share one LDS copy
    per block instead of one per wavefront) against the oracle's histogram; the
    moments without histograms equal, bit for bit, those of the pass that also
    counts (the same cells in the same order)."""
    n = 32
    grid = g.Grid(n, 200.0, 10, dtype)
    gen = torch.Generator(device="cuda").manual_seed(11)
    fields = [torch.randn((n,) * 3, generator=gen, device="cuda", dtype=grid.real_dtype) * (0.5 + 0.1 * i)
              for i in range(8)]
    mom, cor, cnt, _ = g.field_stats(ctx, grid, fields, nbins=1024, lo=-3.0, hi=3.0)
    mom0, cor0, cnt0, _ = g.field_stats(ctx, grid, fields, nbins=0)
    ctx.sync()
    assert cnt0 is None
    assert torch.equal(mom, mom0) and torch.equal(cor, cor0)
    for i, f in enumerate(fields):
        ref = stats.histogram(f.cpu().numpy().astype(np.float64), -3.0, 3.0, 1024)
        assert np.array_equal(cnt[i].cpu().numpy(), ref), i
