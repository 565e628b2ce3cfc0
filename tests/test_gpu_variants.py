"""Every compiled launch variant of the pass kernels, pinned with
gridspt_set_tuning, against variant 0 and (at 64^3) against the FP64 oracle.

Variants change only block shapes (rows per block) and radix splits, so the
fields must agree with variant 0 to FP32 rounding.  The autotuner may pick any
of them at run time, so each one is checked on every path that launches pass
kernels: the seeded linear field and D-form orders, the reverse mode, the
P-form with its derived fields, the smoothing pass and the bispectrum's shell
transforms.  FP32 grids of 64 .. 1024 (powers of two) compile variants
{0, 1, 4, 5}; 96, 192 and 384 compile {0, 1, 2}.

Tolerances (relative L2 per field): 2e-6 between variants (a few FP32
roundings apart), 1e-5 against the oracle, as for every FP32 parity test.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1807_04215_amd as g
from tests.layouts import cube_from_tensor, half_to_cube, rel_l2

pytestmark = pytest.mark.gpu

NS, GAMMA = 0.96, 0.21
POW2, THREE = (0, 1, 4, 5), (0, 1, 2)


def _variants(n):
    return POW2 if (n & (n - 1)) == 0 else THREE


def _dev_rel(a, b):
    return (torch.linalg.vector_norm((a - b).double()) / torch.linalg.vector_norm(b.double())).item()


def _lp(n, box, seed):
    cut = g.cut_n2max(n, box)
    amp = oracle.sigma8_amp(0.8, NS, GAMMA)
    return cut, g.LinearSpectrum(amp=amp, ns=NS, gamma=GAMMA, growth=0.8, n2max=cut, seed=seed, stream=2)


@pytest.mark.parametrize("n,box,nmax", [(64, 500.0, 5), (96, 300.0, 4), (256, 1000.0, 4), (384, 1000.0, 3),
                                        (512, 1000.0, 3), (1024, 2000.0, 2)])
def test_orders_every_variant(n, box, nmax):
    cut, lp = _lp(n, box, 40 + n)
    grid = g.Grid(n, box, g.cube_kc(cut), g.F32)
    ctx = g.Context()
    g.set_tuning(ctx, grid, 0)
    ref = g.orders_linear(ctx, grid, lp, nmax, cut)
    out = g.alloc_orders(grid, nmax, True)
    if n == 64:
        r1 = oracle.linear_field(n, box, lp.amp, NS, GAMMA, lp.growth, cut, lp.seed, lp.stream)
        rd, rt, _, _ = oracle.orders(r1, box, nmax, cut, cut)
    for v in _variants(n):
        g.set_tuning(ctx, grid, v)
        g.orders_linear(ctx, grid, lp, nmax, cut, out=out)
        torch.cuda.synchronize()
        for i in range(nmax):
            for got, want, what in ((out.delta[i], ref.delta[i], "delta"), (out.theta[i], ref.theta[i], "theta"),
                                    (out.delta_k[i], ref.delta_k[i], "delta_k")):
                e = _dev_rel(got, want)
                assert e < 2e-6, (n, v, what, i + 1, e)
            if n == 64:
                assert rel_l2(out.delta[i].cpu().numpy(), rd[i]) < 1e-5, (v, i + 1)
                assert rel_l2(out.theta[i].cpu().numpy(), rt[i]) < 1e-5, (v, i + 1)
        print("orders N=%d variant %d ok" % (n, v), flush=True)


@pytest.mark.parametrize("n,box", [(64, 500.0), (96, 300.0)])
def test_reverse_mode_every_variant(n, box):
    nmax = 3
    cut, lp = _lp(n, box, 7)
    grid = g.Grid(n, box, g.cube_kc(cut), g.F32)
    rng = np.random.default_rng(8)
    w = rng.standard_normal((n, n, n)).astype(np.float32)
    gd = rng.standard_normal((nmax, n, n, n)).astype(np.float32)
    wd = torch.from_numpy(w).cuda()
    gdd = [torch.from_numpy(x).cuda() for x in gd]
    ref_oracle = oracle.adjoint(w.astype(np.float64), box, lp.amp, NS, GAMMA, lp.growth, nmax, cut, cut,
                                gd.astype(np.float64))
    ctx = g.Context()
    ref = None
    for v in _variants(n):
        g.set_tuning(ctx, grid, v)
        d1 = g.noise_field(ctx, grid, lp, wd)
        fwd = g.orders(ctx, grid, nmax, cut, cut, d1)
        gw = g.adjoint(ctx, grid, lp, nmax, cut, fwd.delta_k, fwd.theta_k, gdd)
        torch.cuda.synchronize()
        ref = gw.clone() if ref is None else ref
        assert _dev_rel(gw, ref) < 2e-6, (n, v)
        assert rel_l2(gw.cpu().numpy(), ref_oracle) < 1e-5, (n, v)


@pytest.mark.parametrize("n,box", [(64, 250.0), (96, 300.0)])
def test_pform_smooth_bispectrum_every_variant(n, box):
    nmax = 3
    cut, lp = _lp(n, box, 9)
    grid = g.Grid(n, box, g.cube_kc(cut), g.F32)
    d1 = g.linear_field(g.Context(), grid, lp)
    torch.cuda.synchronize()
    edges = g.linear_edges(6, n // 2, 3, cut)
    tris = [(b, b, b) for b in range(2, 6)] + [(b, b, 1) for b in range(2, 6)]
    terms = []
    for t in range(len(tris)):
        terms += [(0, 0, 1, t), (0, 1, 2, t), (1, 1, 1, t)]
    ctx = g.Context()
    ref = None
    for v in _variants(n):
        g.set_tuning(ctx, grid, v)
        pf = g.orders_pform(ctx, grid, nmax, cut, cut, d1)
        sm = g.smooth(ctx, grid, pf.delta_k, [1.0] * nmax, 6.0)
        bk, _ = g.bispectrum(ctx, grid, pf.delta_k, tris, terms, edges)
        torch.cuda.synchronize()
        got = [t.clone() for t in pf.delta + pf.theta + sm] + [bk.clone()]
        if ref is None:
            ref = got
            continue
        for i, (a, b) in enumerate(zip(got[:-1], ref[:-1])):
            assert _dev_rel(a, b) < 2e-6, (n, v, i)
        scale = ref[-1].abs().max().item()
        assert (got[-1] - ref[-1]).abs().max().item() <= 1e-5 * scale, (n, v)
