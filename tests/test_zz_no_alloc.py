"""gridspt_power_static, the cross spectra for callers that cannot allocate:
two calls in a row through the C ABI (the second on a smaller grid with fewer
bins and pairs, in the other precision), each equal bit for bit to
gridspt_power on the same spectra (the same kernels and launch shapes, with
the scratch in the library's own array instead of `work`) and within the
tolerance of the oracle's direct mode sum."""
import numpy as np
import pytest
import torch

import oracle
import paper_1807_04215_amd as g
from tests.layouts import half_to_cube

pytestmark = pytest.mark.gpu

NS, GAMMA = 0.96, 0.21


def _case(ctx, n, box, dtype, nmax, seed):
    cut = g.cut_n2max(n, box)
    grid = g.Grid(n, box, g.cube_kc(cut), dtype)
    d1 = oracle.linear_field(n, box, oracle.sigma8_amp(0.8, NS, GAMMA), NS, GAMMA, 1.0, cut, seed)
    if dtype == g.F32:
        d1 = d1.astype(np.float32).astype(np.float64)
    out = g.orders(ctx, grid, nmax, cut, cut, torch.from_numpy(d1).to("cuda", grid.real_dtype))
    _, _, rdk, _ = oracle.orders(d1, box, nmax, cut, cut)
    return grid, cut, out.delta_k, list(rdk)


@pytest.mark.parametrize("first,second", [((128, 500.0, g.F32, 4, 64), (32, 200.0, g.F64, 2, 8)),
                                          ((64, 300.0, g.F64, 3, 32), (48, 150.0, g.F32, 2, 5))])
def test_power_static_matches_power(first, second):
    assert torch.cuda.is_available()
    ctx = g.Context()
    for n, box, dtype, nmax, nbins in (first, second):
        grid, cut, cubes, rcubes = _case(ctx, n, box, dtype, nmax, 60 + n)
        edges = g.linear_edges(nbins, n, 3, cut)
        pairs = [(a, b) for a in range(nmax) for b in range(a, nmax)]
        want = g.power(ctx, grid, cubes, pairs, edges)
        dev = dict(device="cuda", dtype=torch.float64)
        got = (torch.full((len(pairs), nbins), float("nan"), **dev), torch.full((nbins,), float("nan"), **dev),
               torch.full((nbins,), float("nan"), **dev))
        g.power_static(ctx, grid, cubes, pairs, edges, out=got)
        ctx.sync()
        for a, b in zip(got, want):
            assert torch.equal(a, b), (n, dtype)
        rpk, rkm, rnm = oracle.power(rcubes, box, pairs, edges)
        assert np.array_equal(got[2].cpu().numpy(), rnm)
        tol = 1e-12 if dtype == g.F64 else 1e-5
        pk = got[0].cpu().numpy()
        for p, (a, b) in enumerate(pairs):
            scale = np.sqrt(rpk[pairs.index((a, a))] * rpk[pairs.index((b, b))]) + 1e-300
            err = np.abs(pk[p] - rpk[p])[rnm > 0] / scale[rnm > 0]
            assert np.all(err <= 10 * tol), (n, a, b, err.max())


def test_power_static_rejects_bad_arguments():
    """Validation happens on the host, before the scratch is touched."""
    ctx = g.Context()
    grid = g.Grid(32, 200.0, 10, g.F32)
    c = [torch.zeros(grid.cube_shape, device="cuda")]
    with pytest.raises(g.GridSPTError) as ei:
        g.power_static(ctx, grid, c, [(0, 1)], [1, 5, 9])      # pair index beyond the fields
    assert ei.value.status == -1
    with pytest.raises(g.GridSPTError) as ei:
        g.power_static(ctx, grid, c, [(0, 0)], [1, 9, 5])      # decreasing edges
    assert ei.value.status == -1
