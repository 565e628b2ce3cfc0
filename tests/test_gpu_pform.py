"""The paper-literal P-form of the recursion on the GPU (gridspt_orders_pform)
against the oracle's P-form, and its relation to the divergence form:
identical on de-aliased inputs, different by the aliased terms under the
paper's wider cuts (and by the same amount as in the oracle).

Tolerances: relative L2 per order 1e-12 (FP64), 1e-5 (FP32).
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1807_04215_amd as g
from tests.layouts import cube_from_tensor, half_to_cube, rel_l2

pytestmark = pytest.mark.gpu

NS, GAMMA = 0.96, 0.21
TOL = {g.F64: 1e-12, g.F32: 1e-5}


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available()
    return g.Context()


def _input(n, box, cut1, seed, dtype):
    d1 = oracle.linear_field(n, box, oracle.sigma8_amp(0.8, NS, GAMMA), NS, GAMMA, 1.0, cut1, seed)
    if dtype == g.F32:
        d1 = d1.astype(np.float32).astype(np.float64)
    return d1


def _dev(a, grid):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=grid.real_dtype)


@pytest.mark.parametrize("dtype", [g.F64, g.F32])
@pytest.mark.parametrize("n,box,nmax,cut1,cut2", [(16, 100.0, 5, None, None), (32, 200.0, 3, None, None),
                                                  (32, 100.0, 4, 100, 140), (48, 300.0, 5, None, None),
                                                  (64, 300.0, 3, 300, 500)])
def test_pform_matches_oracle(ctx, dtype, n, box, nmax, cut1, cut2):
    """Strict 2/3 cuts and cuts beyond it (the paper's two-cut setup: W1 inside W2)."""
    c = g.cut_n2max(n, box)
    cut1 = c if cut1 is None else cut1
    cut2 = c if cut2 is None else cut2
    grid = g.Grid(n, box, g.cube_kc(max(cut1, cut2)), dtype)
    d1 = _input(n, box, cut1, 3 + n, dtype)
    out = g.orders_pform(ctx, grid, nmax, cut1, cut2, _dev(d1, grid))
    ctx.sync()
    rd, rt, rdk, rtk = oracle.orders(d1, box, nmax, cut1, cut2, form="P")
    for i in range(nmax):
        ed = rel_l2(out.delta[i].cpu().numpy(), rd[i])
        et = rel_l2(out.theta[i].cpu().numpy(), rt[i])
        ek = rel_l2(cube_from_tensor(out.delta_k[i]), half_to_cube(rdk[i], grid.kc))
        tk = rel_l2(cube_from_tensor(out.theta_k[i]), half_to_cube(rtk[i], grid.kc))
        print("P-form N=%d n=%d dtype=%d: %.2e %.2e %.2e %.2e" % (n, i + 1, dtype, ed, et, ek, tk), flush=True)
        assert max(ed, et, ek, tk) < TOL[dtype], (i + 1, ed, et, ek, tk)


@pytest.mark.parametrize("dtype", [g.F64, g.F32])
def test_pform_equals_dform_dealiased(ctx, dtype):
    """Under the strict 2/3 rule no product aliases, so the two forms agree
    mode by mode (an identity at any size; here 128^3, n <= 5)."""
    n, box, nmax = 128, 500.0, 5
    cut = g.cut_n2max(n, box)
    grid = g.Grid(n, box, g.cube_kc(cut), dtype)
    lp = g.LinearSpectrum(amp=oracle.sigma8_amp(0.8, NS, GAMMA), n2max=cut, seed=4)
    d1 = g.linear_field(ctx, grid, lp)
    p = g.orders_pform(ctx, grid, nmax, cut, cut, d1)
    d = g.orders(ctx, grid, nmax, cut, cut, d1)
    ctx.sync()
    for i in range(nmax):
        for a, b in ((p.delta[i], d.delta[i]), (p.theta[i], d.theta[i])):
            e = (torch.linalg.vector_norm((a - b).double()) / torch.linalg.vector_norm(b.double())).item()
            assert e < TOL[dtype] * 5, (i + 1, e)


def test_pform_minus_dform_under_aliasing_cuts(ctx):
    """Cuts beyond the 2/3 rule in the ratio of the paper's (1 and 4/3 h/Mpc on
    512^3, L = 1000): the forms differ from order 2 on, and the GPU's P - D
    difference equals the oracle's."""
    n, box, nmax = 64, 1000.0 * 64 / 512, 4
    cut1 = g.cut_n2max(n, box, 1.0)
    cut2 = g.cut_n2max(n, box, 4.0 / 3.0)
    grid = g.Grid(n, box, g.cube_kc(cut2), g.F64)
    d1 = _input(n, box, cut1, 9, g.F64)
    p = g.orders_pform(ctx, grid, nmax, cut1, cut2, _dev(d1, grid))
    d = g.orders(ctx, grid, nmax, cut1, cut2, _dev(d1, grid))
    ctx.sync()
    rp = oracle.orders(d1, box, nmax, cut1, cut2, form="P", spectra=False)[0]
    rd = oracle.orders(d1, box, nmax, cut1, cut2, form="D", spectra=False)[0]
    for i in range(1, nmax):
        gdiff = p.delta[i].cpu().numpy() - d.delta[i].cpu().numpy()
        odiff = rp[i] - rd[i]
        frac = np.linalg.norm(odiff) / np.linalg.norm(rd[i])
        print("order %d: |P - D| / |D| = %.3e" % (i + 1, frac), flush=True)
        assert frac > 1e-6                      # aliasing is visible
        assert rel_l2(gdiff, odiff) < 1e-9      # and the GPU reproduces it


@pytest.mark.parametrize("dtype", [g.F32, g.F64])
def test_pform_512_paper_cuts_plane_waves(dtype):
    """The P-form workload itself: 512^3, L = 1000 Mpc/h, the paper's cuts of 1
    and 4/3 h/Mpc (n2max 25330 and 45031), orders 1..5, for plane waves one of
    which (|n_x| = 155) folds onto kept modes when doubled (310 wraps to -202,
    inside the 212 of the second cut).  Both forms against the sparse
    Fourier-space recursion in the same form, at every excited mode (and the
    energy anywhere else), and the aliased difference P - D it predicts."""
    import gc
    from tests.sparse_check import compare_sparse, plane_field, spectrum_of
    n, box, nmax = 512, 1000.0, 5
    cut1 = g.cut_n2max(n, box, 1.0)
    cut2 = g.cut_n2max(n, box, 4.0 / 3.0)
    assert (cut1, cut2) == (25330, 45031)
    grid = g.Grid(n, box, g.cube_kc(cut2), dtype)
    waves = [(0.08, 0.3, (13, -7, 2)), (0.06, -1.2, (-5, 21, 9)), (0.07, 2.1, (30, 4, -17)),
             (0.05, 0.9, (155, 3, -2)), (0.04, -2.5, (-95, 60, 31))]
    spec = spectrum_of(waves)
    ctx = g.Context()
    d1 = plane_field(n, waves, grid.real_dtype)
    tol = TOL[dtype]
    kc = grid.kc
    for form, run in (("P", g.orders_pform), ("D", g.orders)):
        out = run(ctx, grid, nmax, cut1, cut2, d1)
        ctx.sync()
        sd, st = oracle.sparse_orders(spec, n, nmax, cut1, cut2, form=form)
        for o in range(nmax):
            ed = compare_sparse(out.delta_k[o], kc, sd[o])
            et = compare_sparse(out.theta_k[o], kc, st[o])
            print("512^3 paper cuts, %s-form, %s, order %d: rel L2 delta %.2e theta %.2e"
                  % (form, "f32" if dtype == g.F32 else "f64", o + 1, ed, et), flush=True)
            assert ed < tol and et < tol, (form, o + 1, ed, et)
        del out
        gc.collect()
        torch.cuda.empty_cache()
    # the aliased terms are real: the sparse forms differ from order 2 on
    dd, _ = oracle.sparse_orders(spec, n, 3, cut1, cut2, form="D")
    dp, _ = oracle.sparse_orders(spec, n, 3, cut1, cut2, form="P")
    diff = max(abs(dp[1].get(k, 0) - dd[1].get(k, 0)) for k in set(dd[1]) | set(dp[1]))
    assert diff > 1e-6 * max(abs(v) for v in dd[1].values())
