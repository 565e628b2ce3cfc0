"""Every call that takes a caller workspace, run on exactly the size its query
returns, inside an allocation that continues with guard bytes.  The whole
allocation starts as 0xFF bytes, a NaN in FP32 and FP64: no call may write past
its workspace (the guard bytes must come back as they were), and no call may
read a workspace word it has not written first (its outputs must equal, bit for
bit, those of the same call on a plain context, whose workspace holds whatever
earlier calls left in it)."""
import numpy as np
import pytest
import torch

import oracle
import paper_1807_04215_amd as g
from tests import inputs

pytestmark = pytest.mark.gpu

GUARD = 1 << 20
PATTERN = 0xFF
NS, GAMMA = 0.96, 0.21


class GuardedContext(g.Context):
    """A context whose byte buffers (the workspace of each call, the batch's work
    buffer) are fresh views of exactly the requested size, each followed by
    GUARD bytes in the same allocation, all of it filled with PATTERN."""

    def __init__(self):
        super().__init__()
        self.guarded = []

    def empty(self, shape, dtype):
        if dtype != torch.uint8 or not isinstance(shape, int):
            return super().empty(shape, dtype)
        buf = super().empty(shape + GUARD, dtype)
        with torch.cuda.stream(self.stream):
            buf.fill_(PATTERN)
        self.guarded.append((buf, shape))
        return buf[:shape]

    def workspace(self, nbytes):
        self._ws = None  # a new exact buffer for every call
        return super().workspace(nbytes)

    def guards_intact(self):
        self.sync()
        torch.cuda.synchronize()
        bad = [i for i, (b, n) in enumerate(self.guarded) if not bool(torch.all(b[n:] == PATTERN))]
        self.guarded.clear()
        return bad


@pytest.fixture(scope="module")
def gctx():
    assert torch.cuda.is_available()
    return GuardedContext()


@pytest.fixture(scope="module")
def pctx():
    return g.Context()


def _grid(n, box, dtype):
    cut = g.cut_n2max(n, box)
    return g.Grid(n, box, g.cube_kc(cut), dtype), cut


def _lin(cut, seed):
    return g.LinearSpectrum(amp=oracle.sigma8_amp(0.8, NS, GAMMA), ns=NS, gamma=GAMMA, growth=0.8, n2max=cut,
                            seed=seed)


def _dev(a, grid):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=grid.real_dtype)


def _flat(x):
    if isinstance(x, torch.Tensor):
        return [x]
    if isinstance(x, g.Orders):
        return _flat([x.delta, x.theta, x.delta_k, x.theta_k])
    if isinstance(x, dict):
        return _flat([x[k] for k in sorted(x)])
    if isinstance(x, (list, tuple)):
        return [t for y in x for t in _flat(y)]
    return []  # None


def _same(gctx, pctx, a, b):
    """The guards hold, and the guarded call's outputs a equal the plain call's b."""
    assert gctx.guards_intact() == []
    pctx.sync()
    ta, tb = _flat(a), _flat(b)
    assert len(ta) == len(tb) and len(ta) > 0
    for i, (x, y) in enumerate(zip(ta, tb)):
        assert torch.equal(x, y), i


@pytest.mark.parametrize("dtype", [g.F64, g.F32])
def test_transform_pipeline_calls(gctx, pctx, dtype):
    """Linear field, noise field, forward transform, orders (two nmax), seeded
    orders, P-form, the reverse mode and autotuning: each on an exact workspace."""
    grid, cut = _grid(32, 200.0, dtype)
    for c in (gctx, pctx):
        g.set_tuning(c, grid, 0)
    lp = _lin(cut, 5)
    _same(gctx, pctx, *[g.linear_field(c, grid, lp, spectrum=True) for c in (gctx, pctx)])
    noise = _dev(inputs.white(32, 41), grid)
    d1 = [g.noise_field(c, grid, lp, noise) for c in (gctx, pctx)]
    _same(gctx, pctx, *d1)
    d1 = d1[1]
    _same(gctx, pctx, *[g.forward(c, grid, cut, d1) for c in (gctx, pctx)])
    for nmax in (2, 5):
        _same(gctx, pctx, *[g.orders(c, grid, nmax, cut, cut, d1) for c in (gctx, pctx)])
    _same(gctx, pctx, *[g.orders_linear(c, grid, lp, 5, cut) for c in (gctx, pctx)])
    _same(gctx, pctx, *[g.orders_pform(c, grid, 3, cut, cut, d1) for c in (gctx, pctx)])
    out = g.orders(pctx, grid, 3, cut, cut, d1)
    pctx.sync()
    gd = [_dev(inputs.white(32, 50 + i), grid) for i in range(3)]
    _same(gctx, pctx, *[g.adjoint(c, grid, lp, 3, cut, out.delta_k, out.theta_k, gd) for c in (gctx, pctx)])
    g.tune_orders(gctx, grid, lp, 3, cut)  # timings decide the variants: guards only
    assert gctx.guards_intact() == []
    g.set_tuning(gctx, grid, 0)


@pytest.mark.parametrize("dtype", [g.F64, g.F32])
def test_estimator_calls(gctx, pctx, dtype):
    """Smoothing, one-point and joint statistics, cross spectra (one chunk, a
    subset of the pairs of two fields, and several chunks) and bispectra."""
    grid, cut = _grid(48, 300.0, dtype)
    for c in (gctx, pctx):
        g.set_tuning(c, grid, 0)
    out = g.orders_linear(pctx, grid, _lin(cut, 7), 3, cut)
    pctx.sync()
    _same(gctx, pctx, *[g.smooth(c, grid, out.delta_k, [1.0, 0.8, 0.6], 10.0) for c in (gctx, pctx)])
    _same(gctx, pctx, *[g.field_stats(c, grid, out.delta, 40, -1.0, 1.0, 16) for c in (gctx, pctx)])
    edges = g.linear_edges(20, 48, 3, cut)
    for pairs in ([(0, 0), (0, 1), (1, 1)], [(1, 0)], [(a, b) for a in range(3) for b in range(3)] * 3):
        _same(gctx, pctx, *[g.power(c, grid, out.delta_k, pairs, edges) for c in (gctx, pctx)])
    bedges = g.linear_edges(8, 32, 3, cut)
    tris = [(b, b, b) for b in range(2, 8)] + [(b, b, 1) for b in range(2, 8)]
    terms = [c + (t,) for t in range(len(tris)) for c in ((0, 0, 1), (0, 1, 0), (1, 0, 0), (0, 1, 2))]
    _same(gctx, pctx, *[g.bispectrum(c, grid, out.delta_k, tris, terms, bedges) for c in (gctx, pctx)])


def test_batch(gctx, pctx):
    """A two-group batch (spectra and bispectra) on an exact work buffer,
    captured and replayed twice."""
    groups = []
    for n, box, nreal, seed in ((32, 200.0, 3, 11), (48, 300.0, 2, 12)):
        grid, cut = _grid(n, box, g.F32)
        lp = _lin(cut, seed)
        tris = [(b, b, b) for b in range(2, 6)]
        terms = [c + (t,) for t in range(len(tris)) for c in ((0, 0, 1), (0, 1, 0), (1, 0, 0))]
        groups.append(g.BatchGroup(grid, nreal, 3, cut, lp, [(0, 0), (0, 1), (1, 2)], g.linear_edges(10, n, 3, cut),
                                   tris, terms))
    bg, bp = g.Batch(gctx, groups), g.Batch(pctx, groups)
    for _ in range(2):
        bg.run()
        bp.run()
    _same(gctx, pctx, bg.out, bp.out)


def test_batch_bispectrum_in_chunks(gctx, pctx):
    """A batch group whose bispectrum needs more shell slots than one chunk holds
    (three fields over 20 bins: 60 field slots against 32 per chunk, 20 indicator
    slots against 16), on an exact work buffer: guards and bitwise outputs."""
    n, box = 64, 400.0
    cut = g.cut_n2max(n, box)
    grid = g.Grid(n, box, g.cube_kc(cut), g.F32)
    edges = g.linear_edges(20, n, 4, cut)  # shells up to N/4: every triangle closes without wrapping
    tris = [(b, b, b) for b in range(20)] + [(b, b, 0) for b in range(1, 20)]
    terms = [c + (t,) for t in range(len(tris)) for c in ((0, 0, 1), (0, 1, 2), (1, 1, 1))]
    groups = [g.BatchGroup(grid, 2, 3, cut, _lin(cut, 13), [(0, 0), (1, 2)], edges, tris, terms)]
    bg, bp = g.Batch(gctx, groups), g.Batch(pctx, groups)
    bg.run()
    bp.run()
    _same(gctx, pctx, bg.out, bp.out)


@pytest.mark.parametrize("dtype", [g.F64, g.F32])
def test_field_stats_at_the_limits(gctx, pctx, dtype):
    """One-point and joint statistics at the largest sizes the call accepts (8
    fields, 1024 bins, 64 x 64 joint bins), on an exact workspace."""
    grid, _ = _grid(32, 200.0, dtype)
    fields = [_dev(0.4 * inputs.white(32, 200 + i), grid) for i in range(8)]
    _same(gctx, pctx, *[g.field_stats(c, grid, fields, 1024, -1.5, 1.5, 64) for c in (gctx, pctx)])


@pytest.mark.parametrize("dtype", [g.F64, g.F32])
def test_power_at_the_limits(gctx, pctx, dtype):
    """Cross spectra at the largest sizes the call accepts (16 fields, 64 pairs,
    256 bins: 13 launches of 5 pairs), on an exact workspace."""
    grid, cut = _grid(32, 200.0, dtype)
    gen = torch.Generator(device="cuda").manual_seed(17)
    cubes = [torch.randn(grid.cube_shape, generator=gen, device="cuda", dtype=grid.real_dtype) for _ in range(16)]
    pairs = [(i % 16, (5 * i + 3) % 16) for i in range(64)]
    r = np.sqrt(cut) * np.arange(1, 257) / 256.0
    edges = np.maximum.accumulate(np.concatenate([[1], np.ceil(r * r).astype(np.int64)]))
    edges[-1] = cut + 1
    _same(gctx, pctx, *[g.power(c, grid, cubes, pairs, edges) for c in (gctx, pctx)])


@pytest.mark.parametrize("dtype", [g.F64, g.F32])
def test_bispectrum_many_triangles(gctx, pctx, dtype):
    """Every closable shell triple b1 <= b2 <= b3 of 12 shells up to N/4 (the
    shells of a triangle overlap when b3 <= b1 + b2 + 1), three terms each, on an
    exact workspace."""
    grid, cut = _grid(48, 300.0, dtype)
    out = g.orders_linear(pctx, grid, _lin(cut, 19), 3, cut)
    pctx.sync()
    edges = g.linear_edges(12, 48, 4, cut)
    tris = [(a, b, c) for a in range(12) for b in range(a, 12) for c in range(b, 12) if c <= a + b + 1]
    terms = [f + (t,) for t in range(len(tris)) for f in ((0, 0, 1), (0, 1, 2), (1, 1, 1))]
    assert len(tris) > 150
    _same(gctx, pctx, *[g.bispectrum(c, grid, out.delta_k, tris, terms, edges) for c in (gctx, pctx)])
