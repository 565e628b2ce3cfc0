"""Benchmark of the GridSPT hot path on one MI355X.

One step = the whole path on one synthetic realisation:
  linear field (seeded Gaussian, BBKS spectrum, sharp cut at 2/3 k_Nyq)
  -> delta_n, theta_n for n = 1..5 (all real fields resident, spectra stored)
  -> FP64 sum of orders -> 15 delta-delta cross spectra P_mn(k) in 64 bins.
Default workload: 1024^3 cells, L = 2000 Mpc/h, z = 0, FP32.

Prints one JSON line.  `value` is cells per
second to 5th order with inputs resident in HBM; `roofline` is measured for
the kernel that takes the most time, with HIP events on the library's stream
over the timed steps; `cpu_baseline` times the FP64 CPU oracle on a bounded
sample of the same workload on this host.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Mcells/s to 5th order (delta_n,theta_n), FP32 vs FP64 at stated error; FFT HBM GB/s"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # name: (N, L [Mpc/h], z, nmax, bins, description)
    "c3": (1024, 2000.0, 0.0, 5, 64, "1024^3 grid, L=2000 Mpc/h, z=0, n=1..5, all 10 real fields resident"),
    "c2": (256, 1000.0, 1.0, 5, 64, "256^3 grid, L=1000 Mpc/h, z=1, n=1..5"),
    "c1": (64, 500.0, 0.0, 3, 32, "64^3 grid, L=500 Mpc/h, z=0, n=1..3"),
}
# batched uneven grids in one captured graph: (N, realisations); L = 1000 Mpc/h, z = 1, n <= 4, FP32
BATCH_C4 = ((128, 32), (192, 16), (256, 8))
BATCH_BOX, BATCH_Z, BATCH_NMAX, BATCH_BINS = 1000.0, 1.0, 4, 20
FFT_KINDS = ("zfwd_field", "zfwd_noise", "zfwd_products", "yfwd", "xfused_linear", "xfused_order1",
             "xfused_order", "yinv", "zinv")


def cpu_baseline(n_sample: int = 256, box: float = 1000.0, nmax: int = 5, threads: int = 0):
    """The FP64 oracle (as it stands) on a bounded sample: linear field and
    D-form orders 1..nmax on an n_sample^3 grid, on `threads` host threads
    (0: all)."""
    import oracle
    prev = oracle.set_threads(0)  # the current count (0 changes nothing)
    cores = oracle.set_threads(threads) if threads > 0 else prev
    amp = oracle.sigma8_amp(0.8, 0.96, 0.21)
    cut = oracle.cut_n2max_strict(n_sample)
    t0 = time.perf_counter()
    d1 = oracle.linear_field(n_sample, box, amp, 0.96, 0.21, 1.0, cut, 3)
    oracle.orders(d1, box, nmax, cut, cut, form="D", spectra=False)
    dt = time.perf_counter() - t0
    oracle.set_threads(prev)
    return {"value": n_sample ** 3 / dt / 1e6, "unit": "Mcells/s", "cores": int(cores), "kind": "oracle",
            "sample": "%d^3 grid, L=%g, linear field + D-form orders 1..%d, FP64, %.1f s" % (n_sample, box, nmax, dt)}


def kernel_source_digest() -> str:
    import glob
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1807_04215_amd", "csrc")
    files = sorted(p for p in glob.glob(os.path.join(csrc, "**", "*"), recursive=True) if os.path.isfile(p))
    for p in files:
        h.update(os.path.relpath(p, csrc).encode())
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kind: str, args):
    """HBM bytes per launch (GB) of `kind` from the committed rocprofv3 counter
    summary, if it was taken on this workload and on the current kernel
    sources; otherwise None."""
    if args.workload != "c3" or args.dtype != "f32":
        return None
    path = os.path.join(ROOT, "profiles", "c3_fp32_hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    digest = kernel_source_digest()
    with open(path) as f:
        for line in f:
            if line.startswith("machine-readable: traffic "):
                _, _, k, nbytes, dg = line.split()
                if k == kind and dg == digest:
                    return round(float(nbytes) / 1e9, 3)
    return None


def _field_error(host, dev64, slab=64):
    """(relative L2, max |diff| / max |ref|) of a host field against a GPU FP64 field, slab by slab."""
    import torch
    num = den = dmax = rmax = 0.0
    for x0 in range(0, dev64.shape[0], slab):
        a = host[x0:x0 + slab].to(dev64.device, torch.float64)
        b = dev64[x0:x0 + slab]
        d = a - b
        num += float((d * d).sum())
        den += float((b * b).sum())
        dmax = max(dmax, float(d.abs().max()))
        rmax = max(rmax, float(b.abs().max()))
        del a, d
    return (num / den) ** 0.5, dmax / rmax


def fp64_leg(args, host32, steps: int = 2):
    """The same step on the FP64 path from the same seed, after the timed FP32
    steps: its rate, and the error of the FP32 results against it per order
    (relative L2 and largest cell error of delta_n and theta_n), of the FP64
    sum of orders, and per spectrum bin (|dP| against sqrt(P_aa P_bb), and
    against the bound the 1e-5 field tolerance implies for white rounding
    noise: t (sqrt(P_aa Pbar_bb) + sqrt(Pbar_aa P_bb)) + t^2 sqrt(Pbar_aa Pbar_bb),
    Pbar the mean power over every kept mode).  host32: the FP32 step's
    delta, theta, sum of orders and P in host memory."""
    import gc

    import numpy as np
    import torch

    import paper_1807_04215_amd as g

    n, box, z, nmax, nbins, _ = WORKLOADS[args.workload]
    cut = g.cut_n2max(n, box)
    grid = g.Grid(n, box, g.cube_kc(cut), g.F64)
    lp = g.LinearSpectrum(amp=g.sigma8_amp(0.8, 0.96, 0.21), ns=0.96, gamma=0.21, growth=g.growth(0.279, 0.721, z),
                          n2max=cut, seed=3)
    edges = g.linear_edges(nbins, n, 3, cut)
    pairs = [(a, b) for a in range(nmax) for b in range(a, nmax)]
    ctx = g.Context()
    out = g.alloc_orders(grid, nmax, spectra=False, ctx=ctx)
    out.delta_k = [ctx.empty(grid.cube_shape, grid.real_dtype) for _ in range(nmax)]
    total = ctx.empty(grid.real_shape, torch.float64)

    def step():
        g.orders_linear(ctx, grid, lp, nmax, cut, out=out)
        g.sum_orders(ctx, grid, out.delta, [1.0] * nmax, out=total)
        return g.power(ctx, grid, out.delta_k, pairs, edges)

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        pk = step()[0]
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1000.0 / steps
    pbar = g.power(ctx, grid, out.delta_k, [(a, a) for a in range(nmax)], [1, cut + 1])[0].cpu().numpy()[:, 0]
    pk = pk.cpu().numpy()
    del out.delta_k
    gc.collect()
    ed, et = [], []
    for i in range(nmax):
        ed.append(_field_error(host32["delta"][i], out.delta[i]))
        et.append(_field_error(host32["theta"][i], out.theta[i]))
    es = _field_error(host32["sum"], total)
    diag = [pk[pairs.index((a, a))] for a in range(nmax)]
    t = 1e-5
    worst_rel = worst_bound = 0.0
    for p, (a, b) in enumerate(pairs):
        dp = np.abs(host32["pk"][p] - pk[p])
        ok = diag[a] * diag[b] > 0
        worst_rel = max(worst_rel, float((dp[ok] / np.sqrt(diag[a] * diag[b])[ok]).max()))
        bound = t * (np.sqrt(diag[a] * pbar[b]) + np.sqrt(pbar[a] * diag[b])) + t * t * np.sqrt(pbar[a] * pbar[b])
        worst_bound = max(worst_bound, float((dp[ok] / bound[ok]).max()))
    del out, total, ctx
    gc.collect()
    torch.cuda.empty_cache()
    return {"value": round(n ** 3 / (ms / 1000.0) / 1e6, 3), "unit": "Mcells/s", "ms_per_step": round(ms, 3),
            "steps": steps, "error_of_fp32": {
                "delta_rel_l2": ["%.3e" % e[0] for e in ed], "theta_rel_l2": ["%.3e" % e[0] for e in et],
                "delta_max_cell": ["%.3e" % e[1] for e in ed], "theta_max_cell": ["%.3e" % e[1] for e in et],
                "sum_of_orders_rel_l2": "%.3e" % es[0],
                "pk_max_bin_over_sqrt_paa_pbb": "%.3e" % worst_rel,
                "pk_max_bin_over_tolerance_bound": "%.3f" % worst_bound,
                "tolerance_rel_l2": 1e-5}}


def batch_groups(g, amp, dz, seed0=40):
    """The C4 batch: per size class, all delta-delta spectra in 20 linear bins
    and the tree-level bispectrum (delta_1 delta_1 delta_2, three placements)
    on 20 equilateral (b, b, b) and 19 squeezed (b, b, 0) triangles."""
    groups = []
    for i, (n, nreal) in enumerate(BATCH_C4):
        cut = g.cut_n2max(n, BATCH_BOX)
        grid = g.Grid(n, BATCH_BOX, g.cube_kc(cut), g.F32)
        lp = g.LinearSpectrum(amp=amp, ns=0.96, gamma=0.21, growth=dz, n2max=cut, seed=seed0 + i, stream=0)
        edges = g.linear_edges(BATCH_BINS, n, 3, cut)
        pairs = [(a, b) for a in range(BATCH_NMAX) for b in range(a, BATCH_NMAX)]
        tris = [(b, b, b) for b in range(BATCH_BINS)] + [(b, b, 0) for b in range(1, BATCH_BINS)]
        terms = []
        for t in range(len(tris)):
            terms += [(0, 0, 1, t), (0, 1, 0, t), (1, 0, 0, t)]
        groups.append(g.BatchGroup(grid, nreal, BATCH_NMAX, cut, lp, pairs, edges, tris, terms))
    return groups


def batch_bench(args) -> int:
    """C4: 32 x 128^3 + 16 x 192^3 + 8 x 256^3 independent realisations, one
    graph launch per step (the batch's every pass, spectra, bispectra and
    realisation statistics); the roofline comes from one profiled eager run of
    the same batch after the timed steps."""
    import torch

    import paper_1807_04215_amd as g

    dz = g.growth(0.279, 0.721, BATCH_Z)
    amp = g.sigma8_amp(0.8, 0.96, 0.21)
    groups = batch_groups(g, amp, dz)
    ctx = g.Context()
    t0 = time.perf_counter()
    b = g.Batch(ctx, groups, tune=not args.no_tune)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    for _ in range(args.warmup):
        b.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.run()
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1000.0 / args.steps
    cells = sum(n ** 3 * nreal for n, nreal in BATCH_C4)
    tuning = [b.tuning(i) for i in range(len(groups))]
    pk_mean = b.out[0]["pk_mean"][0].cpu().tolist()
    del b
    torch.cuda.empty_cache()
    # one eager, profiled run of the same batch for the per-kernel figures
    eager = g.Batch(ctx, groups, tune=not args.no_tune, eager=True)
    eager.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    eager.run()
    torch.cuda.synchronize()
    eager_ms = (time.perf_counter() - t0) * 1000.0
    ctx.set_profiling(True)
    eager.run()
    ctx.set_profiling(False)
    prof = ctx.profile_read()
    dom = max(prof, key=lambda k: prof[k]["ms"])
    d = prof[dom]
    achieved = d["bytes"] / (d["ms"] / 1000.0) / 1e9
    kern_ms = sum(v["ms"] for v in prof.values())
    if args.kernels:
        for k, v in sorted(prof.items(), key=lambda kv: -kv[1]["ms"]):
            print("%-16s launches %4d  %9.3f ms  %8.1f GB/s" % (
                k, v["launches"], v["ms"], v["bytes"] / max(v["ms"], 1e-9) / 1e6), file=sys.stderr)
        for i, bg in enumerate(groups):
            print("tuning N=%d: %s" % (bg.grid.n, tuning[i]), file=sys.stderr)
        print("P_11 mean, N=128 group: %s" % ["%.4g" % v for v in pk_mean], file=sys.stderr)
    res = {
        "metric": "Mcells/s to 4th order, batched realisations (cells of all realisations per second)",
        "value": round(cells / (ms_step / 1000.0) / 1e6, 3),
        "unit": "Mcells/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded Gaussian linear fields, BBKS P0, sigma8=0.8, independent Philox streams)",
        "config": {"workload": "c4: 32 x 128^3 + 16 x 192^3 + 8 x 256^3 realisations, L=1000 Mpc/h, z=1, "
                               "n=1..4, FP32, cut 2/3 k_Nyq, 10 P_mn pairs and 117 tree-level bispectrum terms "
                               "in 20 bins, realisation means and scatter, one captured graph per step",
                   "autotuned": not args.no_tune, "plan_setup_s": round(setup_s, 2)},
        "eager_ms_per_step": round(eager_ms, 3),
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "launch_ms": round(d["ms"] / d["launches"], 3),
                     "algorithmic_gb_per_launch": round(d["bytes"] / d["launches"] / 1e9, 3),
                     "note": "per-kernel times from one profiled eager run of the same batch"},
        "kernel_ms_eager": round(kern_ms, 3),
        "path_gbs": round(sum(v["bytes"] for v in prof.values()) / (kern_ms / 1000.0) / 1e9, 1),
    }
    print(json.dumps(res), flush=True)
    return 0


def adjoint_cpu_baseline(n_sample: int = 256, box: float = 1000.0, nmax: int = 3):
    """The FP64 oracle's reverse mode (as it stands) on a bounded sample: the
    forward recursion plus the adjoint, n_sample^3 grid, all host threads."""
    import numpy as np

    import oracle
    cores = oracle.set_threads(0)
    amp = oracle.sigma8_amp(0.8, 0.96, 0.21)
    cut = oracle.cut_n2max_strict(n_sample)
    rng = np.random.default_rng(0)
    w = rng.standard_normal((n_sample,) * 3)
    gd = rng.standard_normal((nmax,) + (n_sample,) * 3)
    t0 = time.perf_counter()
    d1 = oracle.noise_field(w, box, amp, 0.96, 0.21, 1.0, cut)
    oracle.orders(d1, box, nmax, cut, cut, spectra=True)
    oracle.adjoint(w, box, amp, 0.96, 0.21, 1.0, nmax, cut, cut, gd)
    dt = time.perf_counter() - t0
    return {"value": n_sample ** 3 / dt / 1e6, "unit": "Mcells/s", "cores": int(cores), "kind": "oracle",
            "sample": "%d^3 grid, L=%g, forward orders 1..%d + reverse mode, FP64, %.1f s" % (n_sample, box, nmax, dt)}


def adjoint_bench(args) -> int:
    """C5: gradient of the field-level loss sum_k L^3 |delta_obs - sum_n delta_n|^2 / P_noise
    with respect to the white noise, 256^3, L = 1000 Mpc/h, z = 1, n <= 3, FP32.
    One step = noise -> linear field -> orders 1..3 (spectra of orders 1, 2 kept
    as checkpoints) -> objective gradient -> reverse mode to dJ/dw."""
    import torch

    import paper_1807_04215_amd as g

    n, box, nmax, pnoise = 256, 1000.0, 3, 100.0
    cut = g.cut_n2max(n, box)
    grid = g.Grid(n, box, g.cube_kc(cut), g.F32)
    lp = g.LinearSpectrum(amp=g.sigma8_amp(0.8, 0.96, 0.21), ns=0.96, gamma=0.21,
                          growth=g.growth(0.279, 0.721, 1.0), n2max=cut, seed=5)
    ctx = g.Context()
    # observed field: a seeded fifth-order field plus white noise of power P_noise
    obs_lp = g.LinearSpectrum(**{**lp.__dict__, "seed": 77})
    d1 = g.linear_field(ctx, grid, obs_lp)
    o5 = g.orders(ctx, grid, 5, cut, cut, d1, spectra=False)
    gen = torch.Generator(device="cuda").manual_seed(78)
    obs = sum(o5.delta) + torch.randn((n,) * 3, generator=gen, device="cuda") * (pnoise * n ** 3 / box ** 3) ** 0.5
    del o5, d1
    w = torch.randn((n,) * 3, generator=gen, device="cuda")
    scale = -2.0 * box ** 3 / pnoise / n ** 3

    def step():
        d1 = g.noise_field(ctx, grid, lp, w)
        out = g.orders(ctx, grid, nmax, cut, cut, d1)
        r = (obs - sum(out.delta)) * scale  # dJ/d delta_n, the same for every n
        return g.adjoint(ctx, grid, lp, nmax, cut, out.delta_k, out.theta_k, [r] * nmax)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.set_profiling(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        gw = step()
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1000.0 / args.steps
    ctx.set_profiling(False)
    prof = ctx.profile_read()
    dom = max(prof, key=lambda k: prof[k]["ms"])
    d = prof[dom]
    achieved = d["bytes"] / (d["ms"] / 1000.0) / 1e9
    kern_ms = sum(v["ms"] for v in prof.values())
    if args.kernels:
        for k, v in sorted(prof.items(), key=lambda kv: -kv[1]["ms"]):
            print("%-16s launches %4d  %9.3f ms/step  %8.1f GB/s" % (
                k, v["launches"], v["ms"] / args.steps, v["bytes"] / max(v["ms"], 1e-9) / 1e6), file=sys.stderr)
    res = {
        "metric": "Mcells/s of forward + reverse mode (gradient w.r.t. the white noise), 3rd order",
        "value": round(n ** 3 / (ms_step / 1000.0) / 1e6, 3), "unit": "Mcells/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded white noise; observed field = seeded 5th-order field + white noise, P_noise=100)",
        "config": {"workload": "c5: 256^3 grid, L=1000 Mpc/h, z=1, n=1..3, FP32, cut 2/3 k_Nyq, gradient of "
                               "sum_k L^3 |delta_obs - sum_n delta_n|^2 / P_noise w.r.t. the white noise, "
                               "spectra of orders < 3 as checkpoints",
                   "grad_rms": float(gw.double().pow(2).mean().sqrt().item())},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "launch_ms": round(d["ms"] / d["launches"], 3),
                     "algorithmic_gb_per_launch": round(d["bytes"] / d["launches"] / 1e9, 3)},
        "kernel_ms_per_step": round(kern_ms / args.steps, 3),
        "path_gbs": round(sum(v["bytes"] for v in prof.values()) / (kern_ms / 1000.0) / 1e9, 1),
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = adjoint_cpu_baseline()
    print(json.dumps(res), flush=True)
    return 0


def cut_sweep(args) -> int:
    """App. A: sensitivity to the high-k cutoff on the paper's grid (512^3,
    L = 1000 Mpc/h, z = 1).  For one sharp-k cut on every order, k_cut in
    {0.8, 1.0, 1.2, 4/3, 1.5, 1.6} h/Mpc, and for the default pair (1 and 4/3),
    the P-form (printed sources) and the D-form run on the same seeded linear
    field (FP32).  Reported per setup: the relative L2 of P - D of delta_n
    (the aliased terms), and the two-loop delta spectrum
    P11 + P22 + 2 P13 + P33 + 2 P24 + 2 P15 of the P-form in the lowest bins,
    relative to the default setup.  Not a timed benchmark."""
    import torch

    import paper_1807_04215_amd as g

    n, box, nmax = 512, 1000.0, 5
    dz = g.growth(0.279, 0.721, 1.0)
    setups = [("default 1, 4/3", 1.0, 4.0 / 3.0)] + [("%.3g" % k, k, k) for k in (0.8, 1.0, 1.2, 4.0 / 3.0, 1.5, 1.6)]
    kmax_bins = 0.5                                   # h/Mpc
    nb = 20
    n_kmax = int(kmax_bins * box / (2.0 * math.pi))  # bins on [0, about 0.5 h/Mpc]
    ctx = g.Context()
    pairs = [(0, 0), (1, 1), (0, 2), (2, 2), (1, 3), (0, 4)]
    coef = [1.0, 1.0, 2.0, 1.0, 2.0, 2.0]
    res = {}
    ref = None
    for name, k1, k2 in setups:
        cut1, cut2 = g.cut_n2max(n, box, k1), g.cut_n2max(n, box, k2)
        grid = g.Grid(n, box, g.cube_kc(max(cut1, cut2)), g.F32)
        lp = g.LinearSpectrum(amp=g.sigma8_amp(0.8, 0.96, 0.21), ns=0.96, gamma=0.21, growth=dz, n2max=cut1, seed=6)
        d1 = g.linear_field(ctx, grid, lp)
        pf = g.orders_pform(ctx, grid, nmax, cut1, cut2, d1)
        df = g.orders(ctx, grid, nmax, cut1, cut2, d1, spectra=False)
        edges = g.linear_edges(nb, n_kmax, 1, cut2)
        pk, km, nm = g.power(ctx, grid, pf.delta_k, pairs, edges)
        torch.cuda.synchronize()
        pd = []
        for i in range(nmax):
            a, b = pf.delta[i].double(), df.delta[i].double()
            pd.append(float((torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b)).item()))
            del a, b
        p2 = sum(c * pk[i] for i, c in enumerate(coef)).cpu().numpy()
        if ref is None:
            ref = p2
        res[name] = {"n2max": [int(cut1), int(cut2)], "p_minus_d_rel_l2_delta": ["%.3e" % e for e in pd],
                     "p2loop_over_default_bins_0_to_7": ["%.4f" % (p2[b] / ref[b]) for b in range(8)]}
        print("cut %-16s P-D %s  P2loop/default %s" % (name, res[name]["p_minus_d_rel_l2_delta"],
                                                     res[name]["p2loop_over_default_bins_0_to_7"]), file=sys.stderr,
              flush=True)
        del pf, df, d1
        torch.cuda.empty_cache()
    kmean = km.cpu().numpy()[:8]
    print(json.dumps({"cut_sweep": res, "grid": "512^3, L = 1000 Mpc/h, z = 1, seed 6, FP32",
                      "bins_kmean_h_per_mpc": ["%.4f" % k for k in kmean]}), flush=True)
    return 0


def pform_bench(args) -> int:
    """C6: the paper-literal P-form on the paper's own grid and cuts: 512^3,
    L = 1000 Mpc/h, z = 0, k_cut = 1 h/Mpc for the linear field and 4/3 h/Mpc for
    the higher orders (Sec. II C), n <= 5, FP32.  One step = linear field ->
    P-form orders 1..5 (17 derived fields per order).  After the timed steps
    the D-form runs on the same linear field and the per-order P - D
    difference (the aliased terms the paper's cut admits) is reported."""
    import torch

    import paper_1807_04215_amd as g

    n, box, nmax = 512, 1000.0, 5
    cut1 = g.cut_n2max(n, box, 1.0)
    cut2 = g.cut_n2max(n, box, 4.0 / 3.0)
    grid = g.Grid(n, box, g.cube_kc(cut2), g.F32)
    lp = g.LinearSpectrum(amp=g.sigma8_amp(0.8, 0.96, 0.21), ns=0.96, gamma=0.21, growth=1.0, n2max=cut1, seed=6)
    ctx = g.Context()
    d1 = g.linear_field(ctx, grid, lp)
    out = g.alloc_orders(grid, nmax, spectra=True)

    def step():
        g.linear_field(ctx, grid, lp, out=d1)
        g.orders_pform(ctx, grid, nmax, cut1, cut2, d1, out=out)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.set_profiling(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1000.0 / args.steps
    ctx.set_profiling(False)
    prof = ctx.profile_read()
    dom = max(prof, key=lambda k: prof[k]["ms"])
    dd = prof[dom]
    achieved = dd["bytes"] / (dd["ms"] / 1000.0) / 1e9
    kern_ms = sum(v["ms"] for v in prof.values())
    if args.kernels:
        for k, v in sorted(prof.items(), key=lambda kv: -kv[1]["ms"]):
            print("%-16s launches %4d  %9.3f ms/step  %8.1f GB/s" % (
                k, v["launches"], v["ms"] / args.steps, v["bytes"] / max(v["ms"], 1e-9) / 1e6), file=sys.stderr)
    # P - D per order on the same linear field, and the de-aliased control (strict 2/3 cut)
    dform = g.orders(ctx, grid, nmax, cut1, cut2, d1, spectra=False)
    torch.cuda.synchronize()
    pd = []
    for i in range(nmax):
        a, b = out.delta[i].double(), dform.delta[i].double()
        pd.append(float((torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b)).item()))
        del a, b
    del dform
    torch.cuda.empty_cache()
    res = {
        "metric": "Mcells/s to 5th order, P-form (printed sources of Eq. 10)",
        "value": round(n ** 3 / (ms_step / 1000.0) / 1e6, 3), "unit": "Mcells/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded Gaussian linear field, BBKS P0, sigma8=0.8)",
        "config": {"workload": "c6: 512^3 grid, L=1000 Mpc/h, z=0, n=1..5, FP32, P-form, cuts 1 and 4/3 h/Mpc "
                               "(n2max %d and %d), 17 derived fields per order" % (cut1, cut2),
                   "p_minus_d_rel_l2_delta": ["%.3e" % e for e in pd]},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "launch_ms": round(dd["ms"] / dd["launches"], 3),
                     "algorithmic_gb_per_launch": round(dd["bytes"] / dd["launches"] / 1e9, 3)},
        "kernel_ms_per_step": round(kern_ms / args.steps, 3),
        "path_gbs": round(sum(v["bytes"] for v in prof.values()) / (kern_ms / 1000.0) / 1e9, 1),
    }
    if not args.no_cpu_baseline:
        import oracle
        cores = oracle.set_threads(0)
        ns_ = 256
        c1 = oracle.cut_n2max_abs(ns_, box * ns_ / n, 1.0)
        c2 = oracle.cut_n2max_abs(ns_, box * ns_ / n, 4.0 / 3.0)
        t0 = time.perf_counter()
        x = oracle.linear_field(ns_, box * ns_ / n, lp.amp, 0.96, 0.21, 1.0, c1, 6)
        oracle.orders(x, box * ns_ / n, nmax, c1, c2, form="P", spectra=False)
        dt = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": ns_ ** 3 / dt / 1e6, "unit": "Mcells/s", "cores": int(cores), "kind": "oracle",
                               "sample": "%d^3 grid at the same cell size and cuts, linear field + P-form orders "
                                         "1..%d, FP64, %.1f s" % (ns_, nmax, dt)}
    print(json.dumps(res), flush=True)
    return 0


def stats_bench(args) -> int:
    """C7: field statistics of the P-form fields of the paper's grid and cuts
    (512^3, L = 1000 Mpc/h, z = 0, n <= 5): one step = Gaussian smoothing
    (R = 10 Mpc/h) of the cumulative sums delta_SPT^(n), n = 1..5, from the stored
    spectra, then mean, variance, skewness, kurtosis and the correlation
    matrix of the five fields, their PDFs (100 bins on [-1.5, 3.5]) and the
    joint PDFs of delta_SPT^(5) with each lower truncation (64 x 64)."""
    import numpy as np
    import torch

    import paper_1807_04215_amd as g

    n, box, nmax, radius = 512, 1000.0, 5, 10.0
    cut1 = g.cut_n2max(n, box, 1.0)
    cut2 = g.cut_n2max(n, box, 4.0 / 3.0)
    grid = g.Grid(n, box, g.cube_kc(cut2), g.F32)
    lp = g.LinearSpectrum(amp=g.sigma8_amp(0.8, 0.96, 0.21), ns=0.96, gamma=0.21, growth=1.0, n2max=cut1, seed=6)
    ctx = g.Context()
    d1 = g.linear_field(ctx, grid, lp)
    out = g.orders_pform(ctx, grid, nmax, cut1, cut2, d1)
    del d1
    sm = [torch.empty((n,) * 3, device="cuda") for _ in range(nmax)]
    coef = [1.0] * nmax

    def step():
        g.smooth(ctx, grid, out.delta_k, coef, radius, out=sm)
        return g.field_stats(ctx, grid, [sm[-1]] + sm[:-1], nbins=100, lo=-1.5, hi=3.5, nbins2=64)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.set_profiling(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        mom, cor, cnt, jnt = step()
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1000.0 / args.steps
    ctx.set_profiling(False)
    prof = ctx.profile_read()
    dom = max(prof, key=lambda k: prof[k]["ms"])
    dd = prof[dom]
    achieved = dd["bytes"] / (dd["ms"] / 1000.0) / 1e9
    kern_ms = sum(v["ms"] for v in prof.values())
    if args.kernels:
        for k, v in sorted(prof.items(), key=lambda kv: -kv[1]["ms"]):
            print("%-16s launches %4d  %9.3f ms/step  %8.1f GB/s" % (
                k, v["launches"], v["ms"] / args.steps, v["bytes"] / max(v["ms"], 1e-9) / 1e6), file=sys.stderr)
    m = mom.cpu().numpy()
    r = cor.cpu().numpy()
    below = [float((sm[i] < -1.0).double().mean().item()) for i in range(nmax)]
    res = {
        "metric": "Mcells/s of smoothing + one-point statistics of five truncated SPT fields",
        "value": round(n ** 3 / (ms_step / 1000.0) / 1e6, 3), "unit": "Mcells/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded Gaussian linear field, BBKS P0, sigma8=0.8)",
        "config": {"workload": "c7: 512^3 grid, L=1000 Mpc/h, z=0, P-form orders 1..5 with cuts 1 and 4/3 h/Mpc, "
                               "Gaussian R=10 Mpc/h, cumulative delta_SPT^(n), PDF 100 bins on [-1.5, 3.5), "
                               "joint PDF 64 x 64 with delta_SPT^(5)",
                   "sigma_n": ["%.4f" % np.sqrt(v) for v in np.roll(m[:, 1], -1)],
                   "skewness_n": ["%.4f" % v for v in np.roll(m[:, 2], -1)],
                   "r_n_5": ["%.5f" % v for v in np.roll(r[0], -1)],
                   "fraction_below_minus_1": ["%.2e" % v for v in below]},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "launch_ms": round(dd["ms"] / dd["launches"], 3),
                     "algorithmic_gb_per_launch": round(dd["bytes"] / dd["launches"] / 1e9, 3)},
        "kernel_ms_per_step": round(kern_ms / args.steps, 3),
        "path_gbs": round(sum(v["bytes"] for v in prof.values()) / (kern_ms / 1000.0) / 1e9, 1),
    }
    print(json.dumps(res), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOADS) + ["c4", "c5", "c6", "c7"])
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner of the pass variants")
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-spectra", action="store_true", help="skip the spectrum stores and P(k)")
    ap.add_argument("--kernels", action="store_true", help="also print the per-kernel table to stderr")
    ap.add_argument("--cut-sweep", action="store_true",
                    help="App. A: P - D and the two-loop P(k) for several sharp-k cuts on 512^3 (not timed)")
    ap.add_argument("--no-fp64", action="store_true",
                    help="skip the FP64 leg (its rate and the FP32 errors against it) after the timed FP32 steps")
    ap.add_argument("--copy-probe", action="store_true",
                    help="a 4 GiB fill, copy and sum (calibrate the HBM byte counters), then exit")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py: the library runs on exactly one GPU (got --gpus %d); sharding a grid over "
              "several GPUs is not implemented" % args.gpus, file=sys.stderr)
        return 2

    import torch

    import paper_1807_04215_amd as g

    torch.cuda.set_device(0)
    if args.copy_probe:
        # kernels of known HBM traffic, in this order: a fill (writes 4 GiB), a copy
        # (reads and writes 4 GiB), a sum (reads 4 GiB, writes one value)
        a = torch.empty(1 << 30, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        total = float(b.sum().item())
        print(json.dumps({"copy_probe_bytes_read": 4 << 30, "copy_probe_bytes_written": 4 << 30,
                          "fill_bytes_written": 4 << 30, "sum_bytes_read": 4 << 30, "sum": total}))
        return 0
    if args.workload == "c4":
        return batch_bench(args)
    if args.workload == "c5":
        return adjoint_bench(args)
    if args.cut_sweep:
        return cut_sweep(args)
    if args.workload == "c6":
        return pform_bench(args)
    if args.workload == "c7":
        return stats_bench(args)
    n, box, z, nmax, nbins, desc = WORKLOADS[args.workload]
    dtype = g.F64 if args.dtype == "f64" else g.F32
    cut = g.cut_n2max(n, box)
    grid = g.Grid(n, box, g.cube_kc(cut), dtype)
    dz = g.growth(0.279, 0.721, z)
    amp = g.sigma8_amp(0.8, 0.96, 0.21)
    lp = g.LinearSpectrum(amp=amp, ns=0.96, gamma=0.21, growth=dz, n2max=cut, seed=3)
    spectra = not args.no_spectra
    edges = g.linear_edges(nbins, n, 3, cut)
    pairs = [(a, b) for a in range(nmax) for b in range(a, nmax)]

    ctx = g.Context()
    out = g.alloc_orders(grid, nmax, spectra=spectra, ctx=ctx)
    ctx.workspace(g.workspace_bytes(grid, nmax))
    total = ctx.empty(grid.real_shape, torch.float64)
    coef = [1.0] * nmax

    tuning = g.tune_orders(ctx, grid, lp, nmax, cut, out=out) if not args.no_tune else None

    def step():
        g.orders_linear(ctx, grid, lp, nmax, cut, out=out)  # linear field + orders 1..nmax
        g.sum_orders(ctx, grid, out.delta, coef, out=total)
        return g.power(ctx, grid, out.delta_k, pairs, edges)[0] if spectra else None

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        pk = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.set_profiling(False)
    prof = ctx.profile_read()
    per_order = ctx.profile_orders()

    ms_step = (t1 - t0) * 1000.0 / args.steps
    value = n ** 3 / (ms_step / 1000.0) / 1e6
    kern_ms = sum(v["ms"] for v in prof.values())
    dom = max(prof, key=lambda k: prof[k]["ms"])
    d = prof[dom]
    achieved = d["bytes"] / (d["ms"] / 1000.0) / 1e9
    fft_ms = sum(prof[k]["ms"] for k in FFT_KINDS if k in prof)
    fft_b = sum(prof[k]["bytes"] for k in FFT_KINDS if k in prof)
    if args.kernels:
        for k, v in sorted(prof.items(), key=lambda kv: -kv[1]["ms"]):
            print("%-16s launches %4d  %9.3f ms/step  %8.1f GB/s" % (
                k, v["launches"], v["ms"] / args.steps, v["bytes"] / max(v["ms"], 1e-9) / 1e6), file=sys.stderr)
        for o, v in sorted(per_order.items()):
            print("order %d: %9.3f ms/step  %8.1f GB/s" % (o, v["ms"] / args.steps,
                                                           v["bytes"] / max(v["ms"], 1e-9) / 1e6), file=sys.stderr)

    res = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Mcells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic (seeded Gaussian linear field, BBKS P0, sigma8=0.8)",
        "config": {"workload": "%s: %s, %s, cut 2/3 k_Nyq%s" % (args.workload, desc, args.dtype,
                                                                 ", 15 P_mn pairs in %d bins" % nbins if spectra else ""),
                   "n": n, "box": box, "z": z, "nmax": nmax, "kc": grid.kc,
                   "autotuned": ({k: v[0] for k, v in tuning.items()} if tuning else None)},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(dom, args), "launch_ms": round(d["ms"] / d["launches"], 3),
                     "algorithmic_gb_per_launch": round(d["bytes"] / d["launches"] / 1e9, 3)},
        "fft_hbm_gbs": round(fft_b / (fft_ms / 1000.0) / 1e9, 1) if fft_ms > 0 else None,
        "kernel_ms_per_step": round(kern_ms / args.steps, 3),
        "path_gbs": round(sum(v["bytes"] for v in prof.values()) / (kern_ms / 1000.0) / 1e9, 1),
        # kernel time of each order's passes (order 1 with the linear field; the product pass of
        # order n, which also finishes the z inverse of order n - 1, counts for order n)
        "per_order_mcells_s": {str(o): round(n ** 3 / (v["ms"] / args.steps / 1000.0) / 1e6, 1)
                               for o, v in sorted(per_order.items()) if o > 0},
        "per_order_gbs": {str(o): round(v["bytes"] / (v["ms"] / 1000.0) / 1e9, 1)
                          for o, v in sorted(per_order.items()) if o > 0},
        "estimators_ms_per_step": round(per_order.get(0, {"ms": 0.0})["ms"] / args.steps, 3),
    }
    if dtype == g.F32 and not args.no_fp64:
        # the FP64 leg, outside the timed region: the FP32 results wait in host memory
        import gc
        host32 = {"delta": [t.cpu() for t in out.delta], "theta": [t.cpu() for t in out.theta], "sum": total.cpu(),
                  "pk": pk.cpu().numpy() if pk is not None else None}
        del out, total, pk, ctx
        gc.collect()
        torch.cuda.empty_cache()
        if spectra:
            f64 = fp64_leg(args, host32)
            f64["speedup_fp32_over_fp64"] = round(value / f64["value"], 3)
            res["fp64"] = f64
        del host32
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline()
        res["cpu_baseline_1thread"] = cpu_baseline(n_sample=128, threads=1)
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
