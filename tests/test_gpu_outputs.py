"""Every output a call writes, handed over as a view of exactly its shape that
continues with guard elements in the same allocation (all bytes 0xFF): no call
may write past any of its outputs."""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_1807_04215_amd as g
from tests import inputs

pytestmark = pytest.mark.gpu

GUARD = 4096  # elements after each output
NS, GAMMA = 0.96, 0.21


class Guarded:
    """Outputs allocated with guard elements behind them."""

    def __init__(self):
        self.items = []

    def new(self, shape, dtype):
        numel = math.prod(shape)
        buf = torch.empty(numel + GUARD, dtype=dtype, device="cuda")
        buf.view(torch.uint8).fill_(0xFF)
        self.items.append((buf, numel))
        return buf[:numel].view(shape)

    def intact(self):
        torch.cuda.synchronize()
        return [i for i, (b, n) in enumerate(self.items) if not bool(torch.all(b[n:].view(torch.uint8) == 0xFF))]


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available()
    return g.Context()


def _dev(a, grid):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=grid.real_dtype)


@pytest.mark.parametrize("dtype", [g.F64, g.F32])
@pytest.mark.parametrize("n,box", [(32, 200.0), (48, 300.0)])
def test_outputs_stay_in_bounds(ctx, dtype, n, box):
    cut = g.cut_n2max(n, box)
    grid = g.Grid(n, box, g.cube_kc(cut), dtype)
    lp = g.LinearSpectrum(amp=oracle.sigma8_amp(0.8, NS, GAMMA), ns=NS, gamma=GAMMA, growth=0.8, n2max=cut, seed=3)
    G = Guarded()
    R = lambda: G.new(grid.real_shape, grid.real_dtype)  # noqa: E731
    C = lambda: G.new(grid.cube_shape, grid.real_dtype)  # noqa: E731

    def orders_out(nmax):
        d = [R() for _ in range(nmax)]
        dk = [C() for _ in range(nmax)]
        return g.Orders(d, [d[0]] + [R() for _ in range(nmax - 1)], dk, [dk[0]] + [C() for _ in range(nmax - 1)])

    def check(what):
        ctx.sync()
        assert G.intact() == [], what

    d1, d1k = R(), C()
    g.linear_field(ctx, grid, lp, out=d1, out_k=d1k)
    check("linear_field")
    noise = _dev(inputs.white(n, 61), grid)
    g.noise_field(ctx, grid, lp, noise, out=R(), out_k=C())
    check("noise_field")
    g.forward(ctx, grid, cut, d1, out_k=C())
    check("forward")
    g.spectrum_half(ctx, grid, d1k, out=G.new((n, n, n // 2 + 1, 2), grid.real_dtype))
    check("spectrum_half")
    out = g.orders(ctx, grid, 5, cut, cut, d1, out=orders_out(5))
    check("orders")
    g.orders_linear(ctx, grid, lp, 4, cut, out=orders_out(4))
    check("orders_linear")
    g.orders_pform(ctx, grid, 3, cut, cut, d1, out=orders_out(3))
    check("orders_pform")
    gd = [_dev(inputs.white(n, 70 + i), grid) for i in range(3)]
    low = g.orders(ctx, grid, 3, cut, cut, d1)
    g.adjoint(ctx, grid, lp, 3, cut, low.delta_k, low.theta_k, gd, out=R())
    check("adjoint")
    g.smooth(ctx, grid, out.delta_k[:3], [1.0, 0.8, 0.6], 10.0, out=[R(), R(), R()])
    check("smooth")
    g.sum_orders(ctx, grid, out.delta, [1.0] * 5, out=G.new(grid.real_shape, torch.float64))
    check("sum_orders")
    edges = g.linear_edges(12, n, 3, cut)
    pairs = [(a, b) for a in range(5) for b in range(a, 5)] + [(4, 0), (2, 2)]
    pk = G.new((len(pairs), len(edges) - 1), torch.float64)
    km, nm = G.new((len(edges) - 1,), torch.float64), G.new((len(edges) - 1,), torch.float64)
    g.power_static(ctx, grid, out.delta_k, pairs, edges, out=(pk, km, nm))
    check("power_static")
