"""Every call that takes a caller workspace, run on exactly the size its query
returns, inside an allocation that continues with guard bytes: no call may
write past its workspace (the guard bytes must come back as they were)."""
import numpy as np
import pytest
import torch

import oracle
import paper_1807_04215_amd as g
from tests import inputs

pytestmark = pytest.mark.gpu

GUARD = 1 << 20
PATTERN = 0xA5
NS, GAMMA = 0.96, 0.21


class GuardedContext(g.Context):
    """A context whose byte buffers (the workspace of each call, the batch's work
    buffer) are fresh views of exactly the requested size, each followed by
    GUARD bytes of PATTERN in the same allocation."""

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


def _grid(n, box, dtype):
    cut = g.cut_n2max(n, box)
    return g.Grid(n, box, g.cube_kc(cut), dtype), cut


def _lin(cut, seed):
    return g.LinearSpectrum(amp=oracle.sigma8_amp(0.8, NS, GAMMA), ns=NS, gamma=GAMMA, growth=0.8, n2max=cut,
                            seed=seed)


def _dev(a, grid):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=grid.real_dtype)


@pytest.mark.parametrize("dtype", [g.F64, g.F32])
def test_transform_pipeline_calls(gctx, dtype):
    """Linear field, noise field, forward transform, orders (two nmax), seeded
    orders, P-form, autotuning and the reverse mode: each on an exact workspace."""
    grid, cut = _grid(32, 200.0, dtype)
    lp = _lin(cut, 5)
    g.linear_field(gctx, grid, lp, spectrum=True)
    assert gctx.guards_intact() == []
    noise = _dev(inputs.white(32, 41), grid)
    d1 = g.noise_field(gctx, grid, lp, noise)
    assert gctx.guards_intact() == []
    g.forward(gctx, grid, cut, d1)
    assert gctx.guards_intact() == []
    for nmax in (2, 5):
        g.orders(gctx, grid, nmax, cut, cut, d1)
        assert gctx.guards_intact() == [], nmax
    g.orders_linear(gctx, grid, lp, 5, cut)
    assert gctx.guards_intact() == []
    g.orders_pform(gctx, grid, 3, cut, cut, d1)
    assert gctx.guards_intact() == []
    g.tune_orders(gctx, grid, lp, 3, cut)
    assert gctx.guards_intact() == []
    g.set_tuning(gctx, grid, 0)
    out = g.orders(gctx, grid, 3, cut, cut, d1)
    assert gctx.guards_intact() == []
    gd = [_dev(inputs.white(32, 50 + i), grid) for i in range(3)]
    g.adjoint(gctx, grid, lp, 3, cut, out.delta_k, out.theta_k, gd)
    assert gctx.guards_intact() == []


@pytest.mark.parametrize("dtype", [g.F64, g.F32])
def test_estimator_calls(gctx, dtype):
    """Smoothing, one-point and joint statistics, cross spectra (one chunk, a
    subset of the pairs of two fields, and several chunks) and bispectra."""
    grid, cut = _grid(48, 300.0, dtype)
    out = g.orders_linear(gctx, grid, _lin(cut, 7), 3, cut)
    assert gctx.guards_intact() == []
    g.smooth(gctx, grid, out.delta_k, [1.0, 0.8, 0.6], 10.0)
    assert gctx.guards_intact() == []
    g.field_stats(gctx, grid, out.delta, 40, -1.0, 1.0, 16)
    assert gctx.guards_intact() == []
    edges = g.linear_edges(20, 48, 3, cut)
    for pairs in ([(0, 0), (0, 1), (1, 1)], [(1, 0)], [(a, b) for a in range(3) for b in range(3)] * 3):
        g.power(gctx, grid, out.delta_k, pairs, edges)
        assert gctx.guards_intact() == [], pairs
    bedges = g.linear_edges(8, 32, 3, cut)
    tris = [(b, b, b) for b in range(2, 8)] + [(b, b, 1) for b in range(2, 8)]
    terms = [c + (t,) for t in range(len(tris)) for c in ((0, 0, 1), (0, 1, 0), (1, 0, 0), (0, 1, 2))]
    g.bispectrum(gctx, grid, out.delta_k, tris, terms, bedges)
    assert gctx.guards_intact() == []


def test_batch(gctx):
    """A two-group batch (spectra and bispectra) on an exact work buffer,
    captured and replayed."""
    groups = []
    for n, box, nreal, seed in ((32, 200.0, 3, 11), (48, 300.0, 2, 12)):
        grid, cut = _grid(n, box, g.F32)
        lp = _lin(cut, seed)
        tris = [(b, b, b) for b in range(2, 6)]
        terms = [c + (t,) for t in range(len(tris)) for c in ((0, 0, 1), (0, 1, 0), (1, 0, 0))]
        groups.append(g.BatchGroup(grid, nreal, 3, cut, lp, [(0, 0), (0, 1), (1, 2)], g.linear_edges(10, n, 3, cut),
                                   tris, terms))
    b = g.Batch(gctx, groups)
    for _ in range(2):
        b.run()
    assert gctx.guards_intact() == []
