"""GPU checks at the full sizes of the benchmark workloads.

384^3, 512^3 (FP32 and FP64) and 768^3: a plane-wave input through all five
orders against the sparse Fourier-space oracle.
1024^3 (the benchmark configuration: L = 2000 Mpc/h, strict 2/3 cut, FP32):
  - a plane-wave input through all five orders against the sparse Fourier-
    space oracle, at every excited mode, plus the energy anywhere else and
    sampled real-space values, in FP32 and in FP64 (the reference of the
    benchmark step's test, tests/test_gpu_headline.py);
  - the seeded linear field against the direct-DFT oracle at sampled modes;
  - bitwise determinism and exact homogeneity of the whole recursion.
256^3 (L = 1000 Mpc/h, z = 1): every field against the full oracle in FP64 and
FP32, the 15 delta-delta cross spectra in 64 bins, and the bispectrum of the
lowest shells against direct triangle enumeration.
"""
import gc
import math

import numpy as np
import pytest
import torch

import oracle
import paper_1807_04215_amd as g
from tests.layouts import cube_from_tensor, half_to_cube, rel_l2
from tests.sparse_check import compare_sparse as _compare_sparse, cube_index as _cube_index
from tests.sparse_check import plane_field as _plane_field, spectrum_of as _spectrum_of

pytestmark = pytest.mark.gpu

NS, GAMMA, SIGMA8 = 0.96, 0.21, 0.8


def _free():
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("dtype", [g.F32, g.F64])
def test_c3_plane_waves_all_orders(dtype):
    """The benchmark grid in both precisions; the FP64 run pins the path that
    serves as the 1024^3 reference of the FP32 benchmark step."""
    n, box, nmax = 1024, 2000.0, 5
    cut = g.cut_n2max(n, box)
    grid = g.Grid(n, box, g.cube_kc(cut), dtype)
    tol = 1e-5 if dtype == g.F32 else 1e-12
    waves = [(0.08, 0.3, (13, -7, 2)), (0.06, -1.2, (-5, 21, 9)), (0.07, 2.1, (30, 4, -17)),
             (0.05, 0.9, (2, -3, 44)), (0.04, -2.5, (-95, 60, 31))]       # the last one makes high orders hit the cut
    d1 = _plane_field(n, waves, grid.real_dtype)
    ctx = g.Context()
    out = g.orders(ctx, grid, nmax, cut, cut, d1)
    ctx.sync()
    sd, st = oracle.sparse_orders(_spectrum_of(waves), n, nmax, cut, cut)
    rng = np.random.default_rng(0)
    pts = rng.integers(0, n, size=(24, 3))
    for o in range(nmax):
        ed = _compare_sparse(out.delta_k[o], grid.kc, sd[o])
        et = _compare_sparse(out.theta_k[o], grid.kc, st[o])
        print("1024^3 plane waves, %s, order %d: spectral rel L2 delta %.2e theta %.2e"
              % ("f32" if dtype == g.F32 else "f64", o + 1, ed, et), flush=True)
        assert ed < tol and et < tol, (o + 1, ed, et)
        # sampled real-space values: delta_n(x) = sum_k delta_n(k) e^{ik.x}
        modes = np.array(list(sd[o].keys()), dtype=np.float64)
        amps = np.array(list(sd[o].values()))
        rms = math.sqrt(float((np.abs(amps) ** 2).sum()))
        want = np.real(np.exp(2j * np.pi * (pts @ modes.T) / n) @ amps)
        t = torch.tensor(pts, device="cuda")
        got = out.delta[o][t[:, 0], t[:, 1], t[:, 2]].double().cpu().numpy()
        # the maximum over 24 points of an error field whose relative L2 is below
        # the tolerance can reach a few times the tolerance of the rms
        assert np.abs(got - want).max() < 5 * tol * rms, (o + 1, np.abs(got - want).max() / rms)
    del out, d1, ctx
    _free()


@pytest.mark.parametrize("n,dtype", [(384, g.F32), (512, g.F32), (768, g.F32), (512, g.F64)])
def test_large_grids_plane_waves(n, dtype):
    """The other large compiled sizes (3 x 2^7, 2^9, 3 x 2^8), five orders of a
    plane-wave input against the sparse oracle at every excited mode (and the
    energy anywhere else)."""
    box, nmax = 1000.0, 5
    cut = g.cut_n2max(n, box)
    grid = g.Grid(n, box, g.cube_kc(cut), dtype)
    waves = [(0.08, 0.3, (13, -7, 2)), (0.06, -1.2, (-5, 21, 9)), (0.07, 2.1, (30, 4, -17)),
             (0.05, 0.9, (2, -3, 44)), (0.04, -2.5, (-95, 60, 31))]
    d1 = _plane_field(n, waves, torch.float32 if dtype == g.F32 else torch.float64)
    ctx = g.Context()
    out = g.orders(ctx, grid, nmax, cut, cut, d1)
    ctx.sync()
    sd, st = oracle.sparse_orders(_spectrum_of(waves), n, nmax, cut, cut)
    tol = 1e-5 if dtype == g.F32 else 1e-12
    for o in range(nmax):
        ed = _compare_sparse(out.delta_k[o], grid.kc, sd[o])
        et = _compare_sparse(out.theta_k[o], grid.kc, st[o])
        print("%d^3 plane waves, order %d: spectral rel L2 delta %.2e theta %.2e" % (n, o + 1, ed, et), flush=True)
        assert ed < tol and et < tol, (o + 1, ed, et)
    del out, d1, ctx
    _free()


def test_c3_linear_field_sampled_modes():
    """The benchmark's linear field (seed 3, z = 0) at sampled modes against
    the oracle's direct DFT over all 1024^3 noise cells."""
    n, box = 1024, 2000.0
    cut = g.cut_n2max(n, box)
    grid = g.Grid(n, box, g.cube_kc(cut), g.F32)
    amp = g.sigma8_amp(SIGMA8, NS, GAMMA)
    dz = g.growth(0.279, 0.721, 0.0)
    ctx = g.Context()
    d1, d1k = g.linear_field(ctx, grid, g.LinearSpectrum(amp=amp, ns=NS, gamma=GAMMA, growth=dz, n2max=cut,
                                                         seed=3), spectrum=True)
    ctx.sync()
    modes = [(1, 0, 0), (0, 7, -3), (-40, 12, 5), (150, -200, 33), (0, 0, 341), (-197, 197, 196)]
    want = oracle.linear_modes(n, box, amp, NS, GAMMA, dz, cut, 3, modes)
    for m, wv in zip(modes, want):
        (kz, ky, kx), conj = _cube_index(grid.kc, m)
        v = d1k[kz, ky, kx].double().cpu().numpy()
        got = complex(v[0], -v[1] if conj else v[1])
        assert abs(got - wv) <= 1e-4 * abs(wv), (m, got, wv)
    del d1, d1k, ctx
    _free()


def test_c3_determinism_and_homogeneity_bitwise():
    n, box, nmax = 1024, 2000.0, 5
    cut = g.cut_n2max(n, box)
    grid = g.Grid(n, box, g.cube_kc(cut), g.F32)
    amp = g.sigma8_amp(SIGMA8, NS, GAMMA)
    ctx = g.Context()
    d1 = g.linear_field(ctx, grid, g.LinearSpectrum(amp=amp, n2max=cut, seed=5))
    a = g.orders(ctx, grid, nmax, cut, cut, d1, spectra=False)
    b = g.orders(ctx, grid, nmax, cut, cut, d1, spectra=False)
    ctx.sync()
    for i in range(nmax):
        assert torch.equal(a.delta[i], b.delta[i]) and torch.equal(a.theta[i], b.theta[i]), i + 1
    d1.mul_(2.0)
    g.orders(ctx, grid, nmax, cut, cut, d1, out=b, spectra=False)
    ctx.sync()
    for i in range(nmax):
        s = 2.0 ** (i + 1)
        assert torch.equal(b.delta[i], a.delta[i] * s) and torch.equal(b.theta[i], a.theta[i] * s), i + 1
    del a, b, d1, ctx
    _free()


@pytest.fixture(scope="module")
def c2_reference():
    n, box, z, nmax = 256, 1000.0, 1.0, 5
    cut = oracle.cut_n2max_strict(n)
    amp = oracle.sigma8_amp(SIGMA8, NS, GAMMA)
    dz = oracle.growth(0.279, 0.721, z)
    d1 = oracle.linear_field(n, box, amp, NS, GAMMA, dz, cut, 2)
    rd, rt, rdk, rtk = oracle.orders(d1, box, nmax, cut, cut, form="D")
    return dict(n=n, box=box, nmax=nmax, cut=cut, amp=amp, dz=dz, d1=d1, rd=rd, rt=rt, rdk=rdk, rtk=rtk)


@pytest.mark.parametrize("dtype", [g.F64, g.F32])
def test_c2_full_oracle_parity(c2_reference, dtype):
    R = c2_reference
    n, box, nmax, cut = R["n"], R["box"], R["nmax"], R["cut"]
    grid = g.Grid(n, box, g.cube_kc(cut), dtype)
    tol = 1e-12 if dtype == g.F64 else 1e-5
    ctx = g.Context()
    # the seeded linear field itself
    d1 = g.linear_field(ctx, grid, g.LinearSpectrum(amp=R["amp"], ns=NS, gamma=GAMMA, growth=R["dz"],
                                                    n2max=cut, seed=2))
    ctx.sync()
    assert rel_l2(d1.cpu().numpy(), R["d1"]) < tol
    # the recursion from the oracle's delta_1 (FP32 runs take it rounded to FP32; the
    # reference stays the unrounded one: rounding moves delta_n by < n * 6e-8, far
    # below the FP32 tolerance)
    rd, rt, rdk, rtk = R["rd"], R["rt"], R["rdk"], R["rtk"]
    out = g.orders(ctx, grid, nmax, cut, cut, torch.from_numpy(R["d1"]).to("cuda", grid.real_dtype))
    ctx.sync()
    errs = []
    for i in range(nmax):
        ed = rel_l2(out.delta[i].cpu().numpy(), rd[i])
        et = rel_l2(out.theta[i].cpu().numpy(), rt[i])
        errs.append((ed, et))
        assert ed < tol and et < tol, (i + 1, ed, et)
    print("C2 %s per-order rel L2 (delta, theta): %s" % ("f64" if dtype == g.F64 else "f32",
                                                        ["%.2e/%.2e" % e for e in errs]))
    # 15 delta-delta cross spectra in 64 bins
    edges = g.linear_edges(64, n, 3, cut)
    pairs = [(a, b) for a in range(nmax) for b in range(a, nmax)]
    pk, km, nm = g.power(ctx, grid, out.delta_k, pairs, edges)
    rpk, rkm, rnm = oracle.power(list(rdk), box, pairs, edges)
    assert np.array_equal(nm.cpu().numpy(), rnm)
    diag = {f: oracle.power([rdk[f]], box, [(0, 0)], edges)[0][0] for f in range(nmax)}
    got = pk.cpu().numpy()
    for p, (a, b) in enumerate(pairs):
        e = np.abs(got[p] - rpk[p]) / (np.sqrt(diag[a] * diag[b]) + 1e-300)
        assert np.all(e[rnm > 0] < 10 * tol), (a, b, e.max())
    # bispectrum: equilateral (b, b, b) and squeezed (b, b, 0) in 20 bins, tree
    # and one-loop terms; the two lowest shells against direct enumeration
    e20 = g.linear_edges(20, n, 3, cut)
    tris = [(b, b, b) for b in range(20)] + [(b, b, 0) for b in range(1, 20)]
    combos = [(0, 0, 1), (0, 1, 0), (1, 0, 0), (0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0),
              (1, 1, 1), (0, 0, 3), (0, 3, 0), (3, 0, 0)]
    terms = [c + (t,) for t in range(len(tris)) for c in combos]
    bk, nt = g.bispectrum(ctx, grid, out.delta_k[:4], tris, terms, e20)
    ctx.sync()
    low = [t for t, tr in enumerate(tris) if max(tr) <= 1]
    lt = [tris[t] for t in low]
    lterms = [c + (i,) for i in range(len(low)) for c in combos]
    rbk, rnt = oracle.bispectrum(list(rdk[:4]), box, lt, lterms, e20)
    sbk, _ = oracle.bispectrum([np.abs(x) for x in rdk[:4]], box, lt, lterms, e20)
    gnt = nt.cpu().numpy()
    gbk = bk.cpu().numpy()
    for i, t in enumerate(low):
        assert gnt[t] == rnt[i], (tris[t], gnt[t], rnt[i])       # exact triangle counts
        got_t = gbk[t * len(combos):(t + 1) * len(combos)]
        want_t = rbk[i * len(combos):(i + 1) * len(combos)]
        scale_t = sbk[i * len(combos):(i + 1) * len(combos)]
        assert np.all(np.abs(got_t - want_t) <= (1e-12 if dtype == g.F64 else 1e-5) * scale_t), tris[t]
    # every triangle count is an integer, and the counts of the same shells in the
    # two precisions agree exactly
    assert np.array_equal(gnt, np.rint(gnt))
    del out, d1, ctx
    _free()
