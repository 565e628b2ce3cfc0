"""GPU parity: libgridspt (through the C ABI) against the FP64 CPU oracle on
the same seeded inputs.

Tolerances (relative L2 over the whole field, per order): 1e-12 for FP64 runs
and 1e-5 for FP32 runs, against the FP64 oracle.  FP32 runs take the oracle's
input rounded to FP32 so that input rounding is not counted.  The orders are
also held cell by cell: the largest error of any cell or mode against the
largest value of the field, 1e-11 (FP64) and 1e-4 (FP32), so that a bad tile
edge touching a few cells cannot hide in the L2 norm.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1807_04215_amd as g
from tests import inputs
from tests.layouts import cube_from_tensor, half_to_cube, rel_l2

pytestmark = pytest.mark.gpu

TOL = {g.F64: 1e-12, g.F32: 1e-5}
CELL = {g.F64: 1e-11, g.F32: 1e-4}  # largest cell (or mode) error against the largest value
NS, GAMMA = 0.96, 0.21


def max_rel(a, b) -> float:
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available()
    return g.Context()


def _amp():
    return oracle.sigma8_amp(0.8, NS, GAMMA)


def _to_dev(a, grid):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=grid.real_dtype)


def _rounded(a, grid):
    return a.astype(np.float32).astype(np.float64) if grid.dtype == g.F32 else a


@pytest.mark.parametrize("dtype", [g.F64, g.F32])
@pytest.mark.parametrize("n,box", [(16, 100.0), (32, 200.0), (64, 500.0), (128, 300.0),
                                   (48, 150.0), (96, 300.0), (192, 600.0)])
def test_forward_transform(ctx, dtype, n, box):
    cut = g.cut_n2max(n, box)
    grid = g.Grid(n, box, g.cube_kc(cut), dtype)
    f = _rounded(inputs.white(n, 100 + n), grid)
    fk = g.forward(ctx, grid, cut, _to_dev(f, grid))
    ctx.sync()
    ref = oracle.forward(f)
    i = np.fft.fftfreq(n, 1.0 / n)
    nx, ny, nz = np.meshgrid(i, i, np.arange(n // 2 + 1), indexing="ij")
    n2 = nx * nx + ny * ny + nz * nz
    ref = np.where((n2 > 0) & (n2 <= cut), ref, 0)
    got = cube_from_tensor(fk)
    want = half_to_cube(ref, grid.kc)
    assert rel_l2(got, want) < TOL[dtype] * (10 if dtype == g.F32 else 1)


@pytest.mark.parametrize("dtype", [g.F64, g.F32])
@pytest.mark.parametrize("n,box,seed", [(32, 200.0, 3), (64, 500.0, 1), (48, 150.0, 2), (192, 600.0, 4)])
def test_linear_field(ctx, dtype, n, box, seed):
    cut = g.cut_n2max(n, box)
    grid = g.Grid(n, box, g.cube_kc(cut), dtype)
    amp, dz = _amp(), 0.61
    lp = g.LinearSpectrum(amp=amp, ns=NS, gamma=GAMMA, growth=dz, n2max=cut, seed=seed, stream=2)
    d1, d1k = g.linear_field(ctx, grid, lp, spectrum=True)
    ctx.sync()
    ref = oracle.linear_field(n, box, amp, NS, GAMMA, dz, cut, seed, 2)
    assert rel_l2(d1.cpu().numpy(), ref) < TOL[dtype]
    assert rel_l2(cube_from_tensor(d1k), half_to_cube(oracle.forward(ref), grid.kc)) < TOL[dtype]


def _orders_case(ctx, dtype, n, box, nmax, seed, cut1=None, cut2=None, kc=None):
    c = g.cut_n2max(n, box)
    cut1 = c if cut1 is None else cut1
    cut2 = c if cut2 is None else cut2
    kc = g.cube_kc(max(cut1, cut2)) if kc is None else kc
    grid = g.Grid(n, box, kc, dtype)
    d1 = oracle.linear_field(n, box, _amp(), NS, GAMMA, 1.0, cut1, seed)
    d1 = _rounded(d1, grid)
    out = g.orders(ctx, grid, nmax, cut1, cut2, _to_dev(d1, grid))
    ctx.sync()
    rd, rt, rdk, rtk = oracle.orders(d1, box, nmax, cut1, cut2, form="D")
    return grid, out, (rd, rt, rdk, rtk)


@pytest.mark.parametrize("dtype", [g.F64, g.F32])
@pytest.mark.parametrize("n,box,nmax,seed", [(16, 100.0, 5, 4), (32, 200.0, 5, 5), (64, 500.0, 3, 1),
                                             (64, 500.0, 5, 6), (128, 500.0, 5, 7), (48, 150.0, 5, 8),
                                             (96, 300.0, 4, 9), (192, 600.0, 3, 10)])
def test_orders_match_oracle(ctx, dtype, n, box, nmax, seed):
    grid, out, (rd, rt, rdk, rtk) = _orders_case(ctx, dtype, n, box, nmax, seed)
    for i in range(nmax):
        gd, gt = out.delta[i].cpu().numpy(), out.theta[i].cpu().numpy()
        ed, et = rel_l2(gd, rd[i]), rel_l2(gt, rt[i])
        assert ed < TOL[dtype] and et < TOL[dtype], (i + 1, ed, et)
        gdk, gtk = cube_from_tensor(out.delta_k[i]), cube_from_tensor(out.theta_k[i])
        rdc, rtc = half_to_cube(rdk[i], grid.kc), half_to_cube(rtk[i], grid.kc)
        edk, etk = rel_l2(gdk, rdc), rel_l2(gtk, rtc)
        assert edk < TOL[dtype] and etk < TOL[dtype], (i + 1, edk, etk)
        cells = [max_rel(gd, rd[i]), max_rel(gt, rt[i]), max_rel(gdk, rdc), max_rel(gtk, rtc)]
        assert max(cells) < CELL[dtype], (i + 1, cells)


@pytest.mark.parametrize("dtype", [g.F64, g.F32])
def test_orders_two_cuts_and_wider_cube(ctx, dtype):
    """W1 != W2 (the paper's two-cut setup, here inside the 2/3 rule) and a
    cube wider than both masks."""
    n, box = 64, 400.0
    grid, out, (rd, rt, rdk, rtk) = _orders_case(ctx, dtype, n, box, 4, 11, cut1=200, cut2=300, kc=19)
    for i in range(4):
        assert rel_l2(out.delta[i].cpu().numpy(), rd[i]) < TOL[dtype]
        assert rel_l2(out.theta[i].cpu().numpy(), rt[i]) < TOL[dtype]
        assert rel_l2(cube_from_tensor(out.delta_k[i]), half_to_cube(rdk[i], grid.kc)) < TOL[dtype]


def test_orders_aliasing_cut(ctx):
    """A cut beyond the 2/3 rule (aliasing on): the GPU follows the oracle's
    divergence form exactly."""
    n, box = 32, 100.0
    cut = 140                     # |n| <= 11 > 32/3
    grid, out, (rd, rt, _, _) = _orders_case(ctx, g.F64, n, box, 3, 12, cut1=cut, cut2=cut)
    for i in range(3):
        assert rel_l2(out.delta[i].cpu().numpy(), rd[i]) < 1e-12


@pytest.mark.parametrize("dtype", [g.F64, g.F32])
def test_homogeneity_and_determinism_bitwise(ctx, dtype):
    """delta_n[2 delta_1] = 2^n delta_n[delta_1] bit for bit, and two runs are
    bitwise identical (no unordered reductions, no races)."""
    n, box = 64, 500.0
    cut = g.cut_n2max(n, box)
    grid = g.Grid(n, box, g.cube_kc(cut), dtype)
    d1 = _to_dev(_rounded(oracle.linear_field(n, box, _amp(), NS, GAMMA, 1.0, cut, 9), grid), grid)
    a = g.orders(ctx, grid, 5, cut, cut, d1)
    b = g.orders(ctx, grid, 5, cut, cut, d1)
    c = g.orders(ctx, grid, 5, cut, cut, 2 * d1)
    ctx.sync()
    for i in range(5):
        assert torch.equal(a.delta[i], b.delta[i]) and torch.equal(a.theta[i], b.theta[i])
        assert torch.equal(c.delta[i], a.delta[i] * 2.0 ** (i + 1))
        assert torch.equal(c.theta[i], a.theta[i] * 2.0 ** (i + 1))


@pytest.mark.parametrize("dtype", [g.F64, g.F32])
@pytest.mark.parametrize("n,box", [(64, 500.0), (48, 300.0)])
def test_power_matches_oracle(ctx, dtype, n, box):
    nmax = 3
    grid, out, (rd, rt, rdk, rtk) = _orders_case(ctx, dtype, n, box, nmax, 1)
    cut = g.cut_n2max(n, box)
    edges = g.linear_edges(32, n, 3, cut)
    pairs = [(0, 0), (0, 1), (1, 1), (0, 2), (1, 2), (2, 2), (3, 4), (5, 0)]
    fields = out.delta_k + out.theta_k
    pk, km, nm = g.power(ctx, grid, fields, pairs, edges)
    ctx.sync()
    ref_fields = list(rdk) + list(rtk)
    rpk, rkm, rnm = oracle.power(ref_fields, box, pairs, edges)
    assert np.array_equal(nm.cpu().numpy(), rnm)
    assert np.allclose(km.cpu().numpy(), rkm, rtol=1e-13, atol=0)
    got = pk.cpu().numpy()
    # per bin, relative to sqrt(P_aa P_bb)
    diag = {}
    for f in range(len(ref_fields)):
        diag[f] = oracle.power([ref_fields[f]], box, [(0, 0)], edges)[0][0]
    for p, (a, b) in enumerate(pairs):
        scale = np.sqrt(np.abs(diag[a] * diag[b])) + 1e-300
        err = np.abs(got[p] - rpk[p]) / scale
        assert np.all(err[rnm > 0] < TOL[dtype] * 10), (p, err.max())


def test_power_many_pairs_chunked(ctx):
    """More pairs than one launch holds (pairs are processed in chunks)."""
    n, box = 32, 200.0
    grid, out, (rd, rt, rdk, rtk) = _orders_case(ctx, g.F64, n, box, 4, 2)
    cut = g.cut_n2max(n, box)
    edges = g.linear_edges(200, n * 10, 30, cut)
    fields = out.delta_k + out.theta_k[1:]
    ref_fields = list(rdk) + list(rtk[1:])
    pairs = [(a, b) for a in range(len(fields)) for b in range(len(fields))][:40]
    pk, _, nm = g.power(ctx, grid, fields, pairs, edges)
    rpk, _, rnm = oracle.power(ref_fields, box, pairs, edges)
    assert np.array_equal(nm.cpu().numpy(), rnm)
    assert np.allclose(pk.cpu().numpy(), rpk, rtol=1e-10, atol=1e-12 * np.abs(rpk).max())


def _random_cubes(grid, nf, seed):
    gen = torch.Generator(device="cuda").manual_seed(seed)
    return [torch.randn(grid.cube_shape, generator=gen, device="cuda", dtype=grid.real_dtype) for _ in range(nf)]


def _cube_to_half(c, n, kc):
    """cube [kz, ky', kx'] (complex numpy) -> half layout [ix, iy, iz], zero outside the cube"""
    from tests.layouts import cube_positions
    h = np.zeros((n, n, n // 2 + 1), dtype=np.complex128)
    p = cube_positions(n, kc)
    h[np.ix_(p, p, np.arange(kc + 1))] = np.transpose(c, (2, 1, 0))
    return h


@pytest.mark.parametrize("dtype", [g.F64, g.F32])
@pytest.mark.parametrize("nf,npairs", [(5, 15), (6, 9)])
def test_power_narrow_and_empty_bins(ctx, dtype, nf, npairs):
    """256 bins a third of a mode step wide in |n| on a 256^3 grid (Kc = 85),
    so that a half-row near the axis meets more than 64 bins and its pieces
    take two groups of bins, and several rounds of 64 pieces where bins hold
    many modes; two empty bins (equal edges).  All pairs of five fields (each
    field loaded once per mode) and pairs over six fields.  Random spectra, so
    every product counts.  Products of FP32 values are exact in FP64, so
    both precisions are held to 1e-12 against the oracle's direct sum."""
    n, box = 256, 1000.0
    cut = g.cut_n2max(n, box)
    kc = g.cube_kc(cut)
    grid = g.Grid(n, box, kc, dtype)
    r = np.sqrt(cut) * np.arange(1, 255) / 254.0
    edges = np.concatenate([[1, 1, 2, 2], np.ceil(r * r).astype(np.int64)[1:]]).astype(np.int64)
    edges = np.maximum.accumulate(edges)
    edges[-1] = cut + 1
    assert len(edges) == 257 and np.all(np.diff(edges) >= 0)
    cubes = _random_cubes(grid, nf, 70 + nf)
    if nf == 5:
        pairs = [(a, b) for a in range(5) for b in range(a, 5)]
    else:
        pairs = [(0, 5), (1, 4), (2, 3), (5, 5), (3, 1), (4, 4), (0, 0), (2, 5), (1, 1)]
    assert len(pairs) == npairs
    pk, km, nm = g.power(ctx, grid, cubes, pairs, edges)
    ctx.sync()
    halves = [_cube_to_half(cube_from_tensor(c), n, kc) for c in cubes]
    rpk, rkm, rnm = oracle.power(halves, box, pairs, edges)
    assert np.array_equal(nm.cpu().numpy(), rnm)
    assert rnm[0] == 0 and rnm[2] == 0 and rnm[1] == 6     # [1, 1) and [2, 2) are empty, [1, 2) holds |n| = 1
    assert np.allclose(km.cpu().numpy(), rkm, rtol=1e-13, atol=0)
    got = pk.cpu().numpy()
    auto = {f: oracle.power([halves[f]], box, [(0, 0)], edges)[0][0] for f in range(nf)}
    ok = rnm > 0
    for p, (a, b) in enumerate(pairs):
        err = np.abs(got[p] - rpk[p])[ok] / np.sqrt(auto[a] * auto[b])[ok]
        assert err.max() < 1e-12, (pairs[p], err.max())


@pytest.mark.parametrize("dtype", [g.F64, g.F32])
@pytest.mark.parametrize("nf", [1, 2, 3, 4, 5])
def test_power_every_field_count(ctx, dtype, nf):
    """One to five fields, each count its own kernel (every pair i <= j formed from
    one load of each field per mode), with the requested pairs a subset of those
    in reversed order and orientation (P_ba for P_ab): random spectra against the
    oracle's direct sum, N_k exactly and P within 1e-12 of sqrt(P_aa P_bb) per bin."""
    n, box = 64, 400.0
    cut = g.cut_n2max(n, box)
    kc = g.cube_kc(cut)
    grid = g.Grid(n, box, kc, dtype)
    edges = g.linear_edges(24, n, 3, cut)
    cubes = _random_cubes(grid, nf, 300 + nf)
    every = [(a, b) for a in range(nf) for b in range(a, nf)]
    pairs = [(b, a) for (a, b) in every[::-1]][: max(1, len(every) - 1)]
    pk, km, nm = g.power(ctx, grid, cubes, pairs, edges)
    ctx.sync()
    halves = [_cube_to_half(cube_from_tensor(c), n, kc) for c in cubes]
    rpk, rkm, rnm = oracle.power(halves, box, pairs, edges)
    assert np.array_equal(nm.cpu().numpy(), rnm)
    assert np.allclose(km.cpu().numpy(), rkm, rtol=1e-13, atol=0)
    got = pk.cpu().numpy()
    auto = {f: oracle.power([halves[f]], box, [(0, 0)], edges)[0][0] for f in range(nf)}
    ok = rnm > 0
    for p, (a, b) in enumerate(pairs):
        err = np.abs(got[p] - rpk[p])[ok] / np.sqrt(auto[a] * auto[b])[ok]
        assert err.max() < 1e-12, (pairs[p], err.max())


@pytest.mark.parametrize("dtype", [g.F64, g.F32])
def test_power_bins_past_the_cube_corners(ctx, dtype):
    """A last edge past the cube's corners (3 (Kc + 1)^2): every stored mode but
    k = 0 is binned, so sum_b N_b = (2 Kc + 1)^3 - 1 and sum_b N_b P_aa / L^3
    is the weighted power of the whole cube; the first bin ends at the cut."""
    n, box = 96, 300.0
    cut = g.cut_n2max(n, box)
    kc = g.cube_kc(cut)
    grid = g.Grid(n, box, kc, dtype)
    edges = [1, cut + 1, 3 * (kc + 1) ** 2 + 7]
    cubes = _random_cubes(grid, 2, 81)
    pk, km, nm = g.power(ctx, grid, cubes, [(0, 0), (0, 1)], edges)
    ctx.sync()
    nmv = nm.cpu().numpy()
    assert nmv.sum() == (2 * kc + 1) ** 3 - 1
    c = [cube_from_tensor(t).astype(np.complex128) for t in cubes]  # products in FP64, as on the GPU
    kz = np.arange(kc + 1)[:, None, None]
    w = np.where(kz == 0, 1.0, 2.0) * np.ones((1, 2 * kc + 1, 2 * kc + 1))
    w[0, 0, 0] = 0.0                                   # k = 0 (cube index [0, 0, 0])
    want = [(w * np.abs(c[0]) ** 2).sum(), (w * (c[0] * np.conj(c[1])).real).sum()]
    got = (pk.cpu().numpy() * nmv).sum(axis=1) / box ** 3
    assert np.allclose(got, want, rtol=1e-12, atol=0)


@pytest.mark.parametrize("dtype", [g.F64, g.F32])
@pytest.mark.parametrize("n,box", [(32, 300.0), (48, 450.0)])
def test_bispectrum_matches_oracle(ctx, dtype, n, box):
    grid, out, (rd, rt, rdk, rtk) = _orders_case(ctx, dtype, n, box, 3, 3)
    cut = g.cut_n2max(n, box)
    edges = g.linear_edges(8, 32, 3, cut)
    tris = [(b, b, b) for b in range(2, 8)] + [(b, b, 1) for b in range(2, 8)]
    terms = []
    for t in range(len(tris)):
        terms += [(0, 0, 1, t), (0, 1, 0, t), (1, 0, 0, t), (0, 1, 2, t), (1, 1, 1, t)]
    bk, nt = g.bispectrum(ctx, grid, out.delta_k, tris, terms, edges)
    ctx.sync()
    rbk, rnt = oracle.bispectrum(list(rdk), box, tris, terms, edges)
    # N_123 is a count of closed triangles: exact, in either precision
    assert np.array_equal(nt.cpu().numpy(), rnt)
    # each term against the same triangle sum taken with |delta(k)| factors
    sbk, _ = oracle.bispectrum([np.abs(x) for x in rdk], box, tris, terms, edges)
    has = rnt[np.asarray(terms)[:, 3]] > 0
    err = np.abs(bk.cpu().numpy() - rbk)[has] / sbk[has]
    assert np.all(err <= (1e-12 if dtype == g.F64 else 1e-5)), err.max()


@pytest.mark.parametrize("dtype", [g.F64, g.F32])
def test_sum_orders(ctx, dtype):
    """The FP64 sum of orders in both instantiations (FP32 fields are what the
    benchmark sums): the oracle's fields, rounded to the grid's precision and
    uploaded, against the oracle's sum of the same values; and, through the
    whole path, the sum of the GPU's orders against the oracle's FP64 fields."""
    n, box = 64, 500.0
    grid, out, (rd, _, _, _) = _orders_case(ctx, dtype, n, box, 5, 8)
    coef = [0.9 ** (i + 1) for i in range(5)]
    host = [_rounded(np.ascontiguousarray(r), grid) for r in rd]
    given = g.sum_orders(ctx, grid, [_to_dev(h, grid) for h in host], coef)
    whole = g.sum_orders(ctx, grid, out.delta, coef)
    ctx.sync()
    got = given.cpu().numpy()
    own = oracle.sum_orders(np.stack(host), coef)
    assert rel_l2(got, own) < 1e-15
    assert np.abs(got - own).max() <= 4e-16 * np.abs(own).max() * 5
    assert rel_l2(whole.cpu().numpy(), oracle.sum_orders(rd, coef)) < TOL[dtype]


@pytest.mark.parametrize("dtype", [g.F64, g.F32])
@pytest.mark.parametrize("nf", [1, 2, 3, 4, 5, 6, 7, 8])
def test_sum_orders_every_count(ctx, dtype, nf):
    """The FP64 sum for every number of fields the call accepts (1 .. 8, each its
    own kernel instantiation): white-noise fields rounded to the grid's precision
    against the oracle's sum of the same values, cell by cell within twice the
    recursive-summation bound (nf + 1) u sum_i |c_i v_i| of one FP64 evaluation.
    N = 48: the cell count is a multiple of 4 but not of the launch's threads."""
    n, box = 48, 150.0
    grid = g.Grid(n, box, g.cube_kc(g.cut_n2max(n, box)), dtype)
    host = [_rounded(inputs.white(n, 900 + 10 * nf + i), grid) for i in range(nf)]
    coef = [(-0.7) ** i + 0.1 * i for i in range(nf)]
    got = g.sum_orders(ctx, grid, [_to_dev(h, grid) for h in host], coef)
    ctx.sync()
    got = got.cpu().numpy()
    want = oracle.sum_orders(np.stack(host), coef)
    scale = sum(abs(c) * np.abs(h) for c, h in zip(coef, host))
    u = np.finfo(np.float64).eps / 2
    assert np.all(np.abs(got - want) <= 2 * (nf + 1) * u * scale)


def test_zeldovich_planar_on_gpu(ctx):
    """The planar pin of the oracle, directly on the GPU path (FP64)."""
    n, box, nmax = 64, 200.0, 5
    cut = g.cut_n2max(n, box)
    grid = g.Grid(n, box, g.cube_kc(cut), g.F64)
    d1 = inputs.planar(n, 5, 4, amp=0.3)
    out = g.orders(ctx, grid, nmax, cut, cut, _to_dev(d1, grid))
    ctx.sync()
    rd, _, _, _ = oracle.orders(d1, box, nmax, cut, cut)
    for i in range(nmax):
        assert rel_l2(out.delta[i].cpu().numpy(), rd[i]) < 1e-12


@pytest.mark.parametrize("dtype", [g.F64, g.F32])
@pytest.mark.parametrize("n,box,nmax,seed", [(32, 200.0, 5, 21), (48, 300.0, 4, 22), (64, 500.0, 3, 23)])
def test_orders_linear_matches_oracle(ctx, dtype, n, box, nmax, seed):
    """The seeded linear field and the orders in one pass sequence (no round trip
    of delta_1 through real space) against the oracle's linear field + orders,
    and against the two-call GPU path."""
    cut = g.cut_n2max(n, box)
    grid = g.Grid(n, box, g.cube_kc(cut), dtype)
    amp, dz = _amp(), 0.7
    lp = g.LinearSpectrum(amp=amp, ns=NS, gamma=GAMMA, growth=dz, n2max=cut, seed=seed, stream=4)
    out = g.orders_linear(ctx, grid, lp, nmax, cut)
    two = g.orders(ctx, grid, nmax, cut, cut, g.linear_field(ctx, grid, lp))
    ctx.sync()
    ref1 = oracle.linear_field(n, box, amp, NS, GAMMA, dz, cut, seed, 4)
    rd, rt, rdk, rtk = oracle.orders(ref1, box, nmax, cut, cut)
    for i in range(nmax):
        assert rel_l2(out.delta[i].cpu().numpy(), rd[i]) < TOL[dtype], i + 1
        assert rel_l2(out.theta[i].cpu().numpy(), rt[i]) < TOL[dtype], i + 1
        assert rel_l2(cube_from_tensor(out.delta_k[i]), half_to_cube(rdk[i], grid.kc)) < TOL[dtype], i + 1
        e = (torch.linalg.vector_norm((out.delta[i] - two.delta[i]).double()) /
             torch.linalg.vector_norm(two.delta[i].double())).item()
        assert e < TOL[dtype], (i + 1, e)


def test_tuned_context_matches_untuned():
    """After gridspt_tune_orders the context runs each pass in the fastest
    compiled variant; the fields equal the untuned ones to FP32 tolerance."""
    n, box, nmax = 128, 500.0, 4
    cut = g.cut_n2max(n, box)
    grid = g.Grid(n, box, g.cube_kc(cut), g.F32)
    lp = g.LinearSpectrum(amp=_amp(), ns=NS, gamma=GAMMA, n2max=cut, seed=31)
    plain = g.Context()
    tuned = g.Context()
    tu = g.tune_orders(tuned, grid, lp, nmax, cut)
    print("tuning 128^3:", tu, flush=True)
    assert tu and all(v in (0, 1, 4, 5) for v, _ in tu.values())
    a = g.orders_linear(plain, grid, lp, nmax, cut)
    b = g.orders_linear(tuned, grid, lp, nmax, cut)
    torch.cuda.synchronize()
    for i in range(nmax):
        e = (torch.linalg.vector_norm((a.delta[i] - b.delta[i]).double()) /
             torch.linalg.vector_norm(a.delta[i].double())).item()
        assert e < 2e-6, (i + 1, e)


def _own_theta1(grid, nmax):
    """Orders outputs where theta_1 and its spectrum have buffers of their own,
    filled with NaN so that a missed store shows."""
    out = g.alloc_orders(grid, nmax, True)
    out.theta[0] = torch.full_like(out.delta[0], float("nan"))
    out.theta_k[0] = torch.full_like(out.delta_k[0], float("nan"))
    return out


@pytest.mark.parametrize("dtype", [g.F64, g.F32])
@pytest.mark.parametrize("nmax", [1, 2, 3, 5])
def test_separate_theta1_buffers(ctx, dtype, nmax):
    """theta_1 = delta_1 (growing mode): with theta_1 in its own buffer the library
    writes it as a second copy of delta_1, bit for bit, on the two-call path
    (delta_1 given), the seeded path and the P-form; every order still matches
    the oracle."""
    n, box, seed = 32, 200.0, 41
    cut = g.cut_n2max(n, box)
    grid = g.Grid(n, box, g.cube_kc(cut), dtype)
    lp = g.LinearSpectrum(amp=_amp(), ns=NS, gamma=GAMMA, growth=1.0, n2max=cut, seed=seed, stream=2)
    ref1 = _rounded(oracle.linear_field(n, box, lp.amp, NS, GAMMA, 1.0, cut, seed, 2), grid)
    refs = {form: oracle.orders(ref1, box, nmax, cut, cut, form=form, spectra=False)[:2] for form in "DP"}
    runs = {
        "given": lambda o: g.orders(ctx, grid, nmax, cut, cut, _to_dev(ref1, grid), out=o),
        "seeded": lambda o: g.orders_linear(ctx, grid, lp, nmax, cut, out=o),
        "pform": lambda o: g.orders_pform(ctx, grid, nmax, cut, cut, _to_dev(ref1, grid), out=o),
    }
    for name, run in runs.items():
        out = _own_theta1(grid, nmax)
        run(out)
        ctx.sync()
        assert torch.equal(out.theta[0], out.delta[0]), name
        assert torch.equal(out.theta_k[0], out.delta_k[0]), name
        rd, rt = refs["P" if name == "pform" else "D"]
        for i in range(nmax):
            assert rel_l2(out.delta[i].cpu().numpy(), rd[i]) < TOL[dtype], (name, i + 1)
            assert rel_l2(out.theta[i].cpu().numpy(), rt[i]) < TOL[dtype], (name, i + 1)
