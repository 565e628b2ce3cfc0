"""The benchmark's own step at its full size, checked.

The 1024^3 FP32 step (L = 2000 Mpc/h, z = 0, seed 3, strict 2/3 cut, n <= 5,
launch variants from the autotuner, FP64 sum of the orders, 15 delta-delta
cross spectra in 64 bins) against the same step on the FP64 GPU path from the
same seed.  The FP64 path is the reference at this size: the oracle cannot
hold a 1024^3 grid (about 230 GB in FP64), and the FP64 path is pinned to the
oracle field by field at 256^3, and on plane waves at 512^3 and 1024^3
(tests/test_gpu_fullsize.py).

Checked per order n: the relative L2 error of delta_n and theta_n (tolerance
1e-5), the largest cell error against the largest value of the field
(1e-4), the FP64 sum of orders, and every spectrum bin; the mode counts agree
exactly.  The FP32 results wait in host memory while the FP64 path runs;
comparisons go slab by slab in FP64.

The bound per spectrum bin follows from the field tolerance.  With
d_a = delta_a + e_a, P_ab(bin) changes by <delta_a e_b*> + <e_a delta_b*> +
<e_a e_b*> over the bin's modes, which Cauchy-Schwarz bounds by
sqrt(P_aa E_bb) + sqrt(E_aa P_bb) + sqrt(E_aa E_bb), with E the power of the
error field in that bin.  FP32 rounding noise is white over the kept modes,
so E_aa = t^2 Pbar_aa, where Pbar_aa is the mean power of delta_a over every
kept mode and t = 1e-5 the tolerance of the field's relative L2 error.  This
matters at the lowest k: delta_n (n >= 2) falls off like k^2 there, far below
its mean power, so a bin relative to sqrt(P_aa P_bb) alone would hold the
white floor to the tiny low-k power of the field.
"""
import gc

import numpy as np
import pytest
import torch

import paper_1807_04215_amd as g

pytestmark = pytest.mark.gpu

N, BOX, Z, NMAX, SEED, NBINS = 1024, 2000.0, 0.0, 5, 3, 64
NS, GAMMA, SIGMA8 = 0.96, 0.21, 0.8
SLAB = 64


def _free():
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def _step(dtype, tune):
    """One benchmark step on a fresh context; everything moved to host memory."""
    cut = g.cut_n2max(N, BOX)
    grid = g.Grid(N, BOX, g.cube_kc(cut), dtype)
    lp = g.LinearSpectrum(amp=g.sigma8_amp(SIGMA8, NS, GAMMA), ns=NS, gamma=GAMMA,
                          growth=g.growth(0.279, 0.721, Z), n2max=cut, seed=SEED)
    edges = g.linear_edges(NBINS, N, 3, cut)
    pairs = [(a, b) for a in range(NMAX) for b in range(a, NMAX)]
    ctx = g.Context()
    # theta spectra are not needed: theta_k entries stay None (the library skips them)
    out = g.alloc_orders(grid, NMAX, spectra=False)
    out.delta_k = [torch.empty(grid.cube_shape, dtype=grid.real_dtype, device="cuda") for _ in range(NMAX)]
    tuning = g.tune_orders(ctx, grid, lp, NMAX, cut, out=out) if tune else None
    g.orders_linear(ctx, grid, lp, NMAX, cut, out=out)
    total = g.sum_orders(ctx, grid, out.delta, [1.0] * NMAX)
    pk, km, nm = g.power(ctx, grid, out.delta_k, pairs, edges)
    # the mean power of each delta_n over every kept mode (one bin holding them all)
    pbar, _, _ = g.power(ctx, grid, out.delta_k, [(a, a) for a in range(NMAX)], [1, cut + 1])
    ctx.sync()
    res = {"tuning": tuning, "pk": pk.cpu().numpy(), "nmodes": nm.cpu().numpy(), "kmean": km.cpu().numpy(),
           "pairs": pairs, "pbar": pbar.cpu().numpy()[:, 0]}
    if dtype == g.F32:
        res["delta"] = [t.cpu() for t in out.delta]
        res["theta"] = [t.cpu() for t in out.theta]
        res["sum"] = total.cpu()
        del out, total
        _free()
    else:
        res["out"], res["total"] = out, total   # stays on the GPU for the comparison
    return res


def _compare(host32, dev64):
    """(relative L2, max |diff| / max |ref|) of a host FP32 (or FP64) field against a GPU FP64 field."""
    num = den = 0.0
    dmax = rmax = 0.0
    for x0 in range(0, N, SLAB):
        a = host32[x0:x0 + SLAB].to("cuda", torch.float64)
        b = dev64[x0:x0 + SLAB].double()
        d = a - b
        num += float((d * d).sum())
        den += float((b * b).sum())
        dmax = max(dmax, float(d.abs().max()))
        rmax = max(rmax, float(b.abs().max()))
        del a, b, d
    return (num / den) ** 0.5, dmax / rmax


@pytest.fixture(scope="module")
def headline():
    assert torch.cuda.is_available()
    r32 = _step(g.F32, tune=True)
    r64 = _step(g.F64, tune=False)
    out, total = r64["out"], r64["total"]
    errs = []
    for i in range(NMAX):
        ed = _compare(r32["delta"][i], out.delta[i])
        et = _compare(r32["theta"][i], out.theta[i])
        errs.append((ed, et))
        print("1024^3 FP32 vs FP64, order %d: delta rel L2 %.3e max %.3e | theta rel L2 %.3e max %.3e"
              % (i + 1, ed[0], ed[1], et[0], et[1]), flush=True)
    esum = _compare(r32["sum"], total)
    print("FP64 sum of orders: rel L2 %.3e, max %.3e" % esum, flush=True)
    print("autotuned variants: %s" % r32["tuning"], flush=True)
    del r64["out"], r64["total"], out, total
    _free()
    return {"errs": errs, "sum": esum, "r32": r32, "r64": r64}


def test_c3_fields_per_order(headline):
    for i, ((ed, md), (et, mt)) in enumerate(headline["errs"]):
        assert ed <= 1e-5 and et <= 1e-5, (i + 1, ed, et)
        assert md <= 1e-4 and mt <= 1e-4, (i + 1, md, mt)


def test_c3_sum_of_orders(headline):
    e, m = headline["sum"]
    assert e <= 1e-5 and m <= 1e-4, (e, m)


def test_c3_cross_spectra_per_bin(headline):
    r32, r64 = headline["r32"], headline["r64"]
    assert np.array_equal(r32["nmodes"], r64["nmodes"])
    assert np.allclose(r32["kmean"], r64["kmean"], rtol=1e-14, atol=0)
    pairs = r64["pairs"]
    diag = {a: r64["pk"][pairs.index((a, a))] for a in range(NMAX)}
    pbar = r64["pbar"]
    t = 1e-5
    ok = r64["nmodes"] > 0
    worst_rel, worst_bound = 0.0, 0.0
    for p, (a, b) in enumerate(pairs):
        dp = np.abs(r32["pk"][p] - r64["pk"][p])[ok]
        rel = dp / np.sqrt(diag[a] * diag[b])[ok]
        bound = (t * (np.sqrt(diag[a] * pbar[b]) + np.sqrt(pbar[a] * diag[b])) + t * t * np.sqrt(pbar[a] * pbar[b]))[ok]
        worst_rel = max(worst_rel, float(rel.max()))
        worst_bound = max(worst_bound, float((dp / bound).max()))
        print("P_%d%d: max |dP|/sqrt(P_aa P_bb) %.2e (bin %d), max |dP|/bound %.3f"
              % (a + 1, b + 1, rel.max(), int(np.argmax(rel)), (dp / bound).max()))
        assert np.all(dp <= bound), ((a + 1, b + 1), float((dp / bound).max()))
    print("over the 15 pairs: max |dP| / sqrt(P_aa P_bb) %.3e, max |dP| / bound %.3f" % (worst_rel, worst_bound))
