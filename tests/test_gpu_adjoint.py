"""Reverse mode on the GPU (gridspt_noise_field, gridspt_adjoint and the
torch.autograd.Function over them) against the FP64 oracle's own adjoint,
whose pins are in test_oracle_adjoint.py, and against directional
derivatives of the GPU forward map itself.

Tolerances: relative L2 of the gradient field 1e-12 (FP64) and 1e-5 (FP32)
against the oracle on the same inputs (FP32 runs take inputs rounded to FP32).
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1807_04215_amd as g
from tests.layouts import rel_l2

pytestmark = pytest.mark.gpu

NS, GAMMA = 0.96, 0.21
TOL = {g.F64: 1e-12, g.F32: 1e-5}


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available()
    return g.Context()


def _case(n, box, nmax, dtype, seed, c1=None, c2=None, dz=0.9):
    c = g.cut_n2max(n, box)
    c1 = c if c1 is None else c1
    c2 = c if c2 is None else c2
    grid = g.Grid(n, box, g.cube_kc(max(c1, c2)), dtype)
    amp = oracle.sigma8_amp(0.8, NS, GAMMA)
    lp = g.LinearSpectrum(amp=amp, ns=NS, gamma=GAMMA, growth=dz, n2max=c1)
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((n, n, n))
    gd = rng.standard_normal((nmax, n, n, n))
    if dtype == g.F32:
        w = w.astype(np.float32).astype(np.float64)
        gd = gd.astype(np.float32).astype(np.float64)
    return grid, lp, c2, w, gd


def _dev(a, grid):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=grid.real_dtype)


@pytest.mark.parametrize("dtype", [g.F64, g.F32])
@pytest.mark.parametrize("n,box", [(32, 200.0), (48, 300.0)])
def test_noise_field_matches_oracle(ctx, dtype, n, box):
    grid, lp, _, w, _ = _case(n, box, 1, dtype, 1)
    d1 = g.noise_field(ctx, grid, lp, _dev(w, grid))
    ctx.sync()
    ref = oracle.noise_field(w, box, lp.amp, NS, GAMMA, lp.growth, lp.n2max)
    assert rel_l2(d1.cpu().numpy(), ref) < TOL[dtype]


@pytest.mark.parametrize("dtype", [g.F64, g.F32])
@pytest.mark.parametrize("n,box,nmax,c1,c2", [(16, 100.0, 1, None, None), (16, 100.0, 2, None, None),
                                              (32, 200.0, 3, None, None), (32, 200.0, 5, None, None),
                                              (48, 300.0, 4, None, None), (32, 250.0, 4, 80, 60)])
def test_adjoint_matches_oracle(ctx, dtype, n, box, nmax, c1, c2):
    grid, lp, c2, w, gd = _case(n, box, nmax, dtype, 2 + nmax, c1, c2)
    wd = _dev(w, grid)
    d1 = g.noise_field(ctx, grid, lp, wd)
    fwd = g.orders(ctx, grid, nmax, lp.n2max, c2, d1)
    gw = g.adjoint(ctx, grid, lp, nmax, c2, fwd.delta_k, fwd.theta_k, [_dev(x, grid) for x in gd])
    ctx.sync()
    ref = oracle.adjoint(w, box, lp.amp, NS, GAMMA, lp.growth, nmax, lp.n2max, c2, gd)
    err = rel_l2(gw.cpu().numpy(), ref)
    print("adjoint N=%d nmax=%d dtype=%d rel L2 %.2e" % (n, nmax, dtype, err), flush=True)
    assert err < TOL[dtype], err


def _loss(deltas, obs, box, pnoise, n):
    """sum_k L^3 |obs(k) - sum_n delta_n(k)|^2 / P_noise over all N^3 modes, by
    Parseval N^-3 sum_x |r(x)|^2 of the residual (k = 0 included; both sides
    have zero mean, so it contributes nothing)."""
    r = obs - sum(deltas)
    return (box ** 3 / pnoise) * (r * r).sum() / n ** 3


def test_autograd_gradient_is_exact_directional_derivative(ctx):
    """Field-level loss of the reconstruction setup, FP64, 16^3, nmax = 3: the
    backward's gradient against the seven-point central difference of the
    GPU forward (the loss is a polynomial of degree 6 in the step, for which
    that stencil is exact), and against the oracle adjoint of the same loss."""
    n, box, nmax, pnoise = 16, 100.0, 3, 100.0
    grid, lp, c2, w, _ = _case(n, box, nmax, g.F64, 11)
    rng = np.random.default_rng(12)
    # observed field: a fifth-order field of another seed plus white noise of power P_noise
    w_obs = rng.standard_normal((n, n, n))
    d_obs = oracle.orders(oracle.noise_field(w_obs, box, lp.amp, NS, GAMMA, lp.growth, lp.n2max), box, 5,
                          lp.n2max, c2, spectra=False)[0].sum(axis=0)
    obs = d_obs + rng.standard_normal((n, n, n)) * np.sqrt(pnoise * n ** 3 / box ** 3)
    obs_t = _dev(obs, grid)
    wt = _dev(w, grid).requires_grad_(True)
    deltas = g.orders_from_noise(wt, ctx, grid, lp, nmax, c2)
    loss = _loss(deltas, obs_t, box, pnoise, n)
    loss.backward()
    grad = wt.grad.detach().clone()
    v = _dev(rng.standard_normal((n, n, n)), grid)

    def L(t):
        with torch.no_grad():
            return _loss(g.orders_from_noise(wt.detach() + t * v, ctx, grid, lp, nmax, c2), obs_t, box, pnoise,
                         n).item()

    h = 0.2
    fd = (-L(-3 * h) + 9 * L(-2 * h) - 45 * L(-h) + 45 * L(h) - 9 * L(2 * h) + L(3 * h)) / (60 * h)
    got = (grad * v).sum().item()
    assert abs(got - fd) <= 1e-9 * abs(fd), (got, fd)
    # the oracle's adjoint of the same loss: dL/d delta_n = -2 (L^3 / P_noise) N^-3 r(x) for every n
    rd = oracle.orders(oracle.noise_field(w, box, lp.amp, NS, GAMMA, lp.growth, lp.n2max), box, nmax, lp.n2max, c2,
                       spectra=False)[0]
    r = obs - rd.sum(axis=0)
    gdl = np.stack([-2.0 * (box ** 3 / pnoise) * r / n ** 3] * nmax)
    ref = oracle.adjoint(w, box, lp.amp, NS, GAMMA, lp.growth, nmax, lp.n2max, c2, gdl)
    assert rel_l2(grad.cpu().numpy(), ref) < 1e-12


@pytest.mark.parametrize("dtype", [g.F64, g.F32])
def test_adjoint_euler_identity_256(ctx, dtype):
    """At the adjoint workload's size (256^3, L = 1000 Mpc/h, n <= 3): the
    degree-n homogeneity of delta_n gives <w, dJ/dw> = sum_n n <g_n, delta_n>
    for J = sum_n <g_n, delta_n>, an identity at any size."""
    n, box, nmax = 256, 1000.0, 3
    c = g.cut_n2max(n, box)
    grid = g.Grid(n, box, g.cube_kc(c), dtype)
    lp = g.LinearSpectrum(amp=oracle.sigma8_amp(0.8, NS, GAMMA), ns=NS, gamma=GAMMA,
                          growth=g.growth(0.279, 0.721, 1.0), n2max=c)
    gen = torch.Generator(device="cuda").manual_seed(5)
    w = torch.randn((n,) * 3, generator=gen, device="cuda", dtype=torch.float64).to(grid.real_dtype)
    gd = [torch.randn((n,) * 3, generator=gen, device="cuda", dtype=torch.float64).to(grid.real_dtype)
          for _ in range(nmax)]
    d1 = g.noise_field(ctx, grid, lp, w)
    fwd = g.orders(ctx, grid, nmax, c, c, d1)
    gw = g.adjoint(ctx, grid, lp, nmax, c, fwd.delta_k, fwd.theta_k, gd)
    ctx.sync()
    lhs = (w.double() * gw.double()).sum().item()
    terms = [(i + 1) * (gd[i].double() * fwd.delta[i].double()).sum().item() for i in range(nmax)]
    tol = 1e-11 if dtype == g.F64 else 2e-5
    assert abs(lhs - sum(terms)) <= tol * sum(abs(t) for t in terms), (lhs, terms)


def test_adjoint_256_matches_oracle(ctx):
    """The reverse mode at the adjoint workload's size and setup (256^3,
    L = 1000 Mpc/h, z = 1, n <= 3, FP32) against the oracle's own adjoint on
    the same noise and objective gradients (rounded to FP32)."""
    n, box, nmax = 256, 1000.0, 3
    c = g.cut_n2max(n, box)
    grid = g.Grid(n, box, g.cube_kc(c), g.F32)
    dz = oracle.growth(0.279, 0.721, 1.0)
    lp = g.LinearSpectrum(amp=oracle.sigma8_amp(0.8, NS, GAMMA), ns=NS, gamma=GAMMA, growth=dz, n2max=c)
    rng = np.random.default_rng(256)
    w = rng.standard_normal((n, n, n)).astype(np.float32).astype(np.float64)
    gd = rng.standard_normal((nmax, n, n, n)).astype(np.float32).astype(np.float64)
    d1 = g.noise_field(ctx, grid, lp, _dev(w, grid))
    fwd = g.orders(ctx, grid, nmax, c, c, d1)
    gw = g.adjoint(ctx, grid, lp, nmax, c, fwd.delta_k, fwd.theta_k, [_dev(x, grid) for x in gd])
    ctx.sync()
    ref = oracle.adjoint(w, box, lp.amp, NS, GAMMA, dz, nmax, c, c, gd)
    err = rel_l2(gw.cpu().numpy(), ref)
    print("adjoint 256^3 FP32, nmax 3: rel L2 %.2e" % err, flush=True)
    assert err < TOL[g.F32], err
