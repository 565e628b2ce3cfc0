"""Batched realisations of several grid sizes in one captured HIP graph
(gridspt_batch_*), against the FP64 oracle run realisation by realisation.

Each realisation r of a group is the oracle's linear field with Philox stream
lin.stream + r, pushed through the oracle's recursion, spectra and
bispectrum; the batch's realisation means and standard deviations are checked
against numpy statistics of those oracle values.  Tolerances are those of the
single-call parity tests (FP64 1e-12, FP32 1e-5 relative L2 per order).
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


def _group(n, box, nreal, nmax, dtype, seed, stream0, bisp):
    cut = g.cut_n2max(n, box)
    grid = g.Grid(n, box, g.cube_kc(cut), dtype)
    amp = oracle.sigma8_amp(0.8, NS, GAMMA)
    lp = g.LinearSpectrum(amp=amp, ns=NS, gamma=GAMMA, growth=0.7, n2max=cut, seed=seed, stream=stream0)
    edges = g.linear_edges(12, n, 3, cut)
    pairs = [(a, b) for a in range(nmax) for b in range(a, nmax)]
    tris = terms = None
    if bisp:
        tris = [(b, b, b) for b in range(2, 7)] + [(b, b, 1) for b in range(3, 7)]
        terms = []
        for t in range(len(tris)):
            terms += [(0, 0, 1, t), (0, 1, 0, t), (1, 0, 0, t)]
            if nmax >= 3:
                terms += [(0, 1, 2, t), (1, 1, 1, t)]
    return g.BatchGroup(grid, nreal, nmax, cut, lp, pairs, edges, tris, terms)


def _oracle_group(bg):
    """Per realisation: fields, spectra and bispectrum terms from the oracle."""
    grid, lp = bg.grid, bg.lin
    res = []
    for r in range(bg.nreal):
        d1 = oracle.linear_field(grid.n, grid.box, lp.amp, lp.ns, lp.gamma, lp.growth, lp.n2max, lp.seed,
                                 lp.stream + r)
        rd, rt, rdk, rtk = oracle.orders(d1, grid.box, bg.nmax, lp.n2max, bg.n2max2)
        pk, km, nm = oracle.power(list(rdk), grid.box, bg.pairs, bg.edges)
        bk = nt = sbk = None
        if bg.tris is not None:
            bk, nt = oracle.bispectrum(list(rdk), grid.box, bg.tris, bg.terms, bg.edges)
            # the same triangle sums with |delta(k)| factors: the scale of each term's error
            sbk, _ = oracle.bispectrum([np.abs(x) for x in rdk], grid.box, bg.tris, bg.terms, bg.edges)
        res.append(dict(delta=rd, theta=rt, dk=rdk, pk=pk, km=km, nm=nm, bk=bk, nt=nt, sbk=sbk))
    return res


def _groups(dtype):
    return [_group(32, 200.0, 3, 3, dtype, 21, 5, True),
            _group(48, 300.0, 2, 3, dtype, 22, 0, True),
            _group(64, 500.0, 2, 2, dtype, 23, 9, False)]


@pytest.mark.parametrize("dtype", [g.F64, g.F32])
def test_batch_matches_oracle_per_realisation(ctx, dtype):
    groups = _groups(dtype)
    b = g.Batch(ctx, groups)
    b.run()
    ctx.sync()
    tol = TOL[dtype]
    for gi, bg in enumerate(groups):
        print("group", gi, "N", bg.grid.n, "nreal", bg.nreal, flush=True)
        ref = _oracle_group(bg)
        for r in range(bg.nreal):
            for i in range(bg.nmax):
                ed = rel_l2(b.buffer(gi, r, g.BATCH_DELTA, i).cpu().numpy(), ref[r]["delta"][i])
                et = rel_l2(b.buffer(gi, r, g.BATCH_THETA, i).cpu().numpy(), ref[r]["theta"][i])
                ek = rel_l2(cube_from_tensor(b.buffer(gi, r, g.BATCH_DELTA_K, i)),
                            half_to_cube(ref[r]["dk"][i], bg.grid.kc))
                assert ed < tol and et < tol and ek < tol, (gi, r, i + 1, ed, et, ek)
            pk = b.buffer(gi, r, g.BATCH_PK).cpu().numpy()
            scale = np.abs(ref[r]["pk"]).max(axis=1, keepdims=True)
            assert np.all(np.abs(pk - ref[r]["pk"]) <= 10 * tol * scale), (gi, r)
            if bg.tris is not None:
                bk = b.buffer(gi, r, g.BATCH_BK).cpu().numpy()
                has = ref[r]["nt"][np.asarray(bg.terms)[:, 3]] > 0
                assert np.all(np.abs(bk - ref[r]["bk"])[has] <= (1e-12 if dtype == g.F64 else 1e-5) *
                              ref[r]["sbk"][has]), (gi, r)
        # realisation statistics
        o = b.out[gi]
        pks = np.stack([x["pk"] for x in ref])
        m, sd = pks.mean(axis=0), pks.std(axis=0, ddof=1)
        scale = np.abs(pks).max(axis=(0, 2))[:, None]
        assert np.all(np.abs(o["pk_mean"].cpu().numpy() - m) <= 10 * tol * scale)
        assert np.all(np.abs(o["pk_std"].cpu().numpy() - sd) <= 100 * tol * scale)
        assert np.array_equal(o["nmodes"].cpu().numpy(), ref[0]["nm"])
        assert np.allclose(o["kmean"].cpu().numpy(), ref[0]["km"], rtol=1e-12, atol=0)
        if bg.tris is not None:
            bks = np.stack([x["bk"] for x in ref])
            sc = np.abs(bks).max()
            btol = 1e-10 if dtype == g.F64 else 1e-4
            assert np.all(np.abs(o["bk_mean"].cpu().numpy() - bks.mean(axis=0)) <= btol * sc)
            assert np.all(np.abs(o["bk_std"].cpu().numpy() - bks.std(axis=0, ddof=1)) <= 10 * btol * sc)
            assert np.array_equal(o["ntriangles"].cpu().numpy(), ref[0]["nt"])


def test_batch_graph_replays_and_eager_agree_bitwise(ctx):
    """Graph replays give identical results, with eager work and syncs between
    replays, and the eager path gives the same bits as the graph."""
    groups = _groups(g.F32)
    b = g.Batch(ctx, groups)
    e = g.Batch(ctx, groups, eager=True)
    b.run()
    ctx.sync()
    first = [{k: v.clone() for k, v in o.items()} for o in b.out]
    f0 = b.buffer(1, 1, g.BATCH_DELTA, 2).clone()
    for _ in range(3):
        torch.zeros(1 << 20, device="cuda").add_(1.0)  # unrelated eager work between replays
        for o in b.out:
            for v in o.values():
                v.zero_()
        b.run()
        ctx.sync()
        for o, f in zip(b.out, first):
            for k in o:
                assert torch.equal(o[k], f[k]), k
        assert torch.equal(b.buffer(1, 1, g.BATCH_DELTA, 2), f0)
    e.run()
    ctx.sync()
    for o, f in zip(e.out, first):
        for k in o:
            assert torch.equal(o[k], f[k]), k


def test_batch_autotuned_variants_stay_within_tolerance(ctx):
    """The autotuner picks per pass kind among the compiled variants (rows per
    block, radix split); every choice computes the same fields to tolerance."""
    groups = [_group(64, 500.0, 4, 3, g.F32, 31, 0, False), _group(96, 600.0, 2, 3, g.F32, 32, 0, False)]
    ref = g.Batch(ctx, groups)
    tuned = g.Batch(ctx, groups, tune=True)
    ref.run()
    tuned.run()
    ctx.sync()
    allowed = {64: {0, 1, 4, 5}, 96: {0, 1, 2}}
    for gi, bg in enumerate(groups):
        tu = tuned.tuning(gi)
        print("tuning N=%d:" % bg.grid.n, tu, flush=True)
        assert tu and all(v in allowed[bg.grid.n] for v, _ in tu.values())
        for r in range(bg.nreal):
            for i in range(bg.nmax):
                a = tuned.buffer(gi, r, g.BATCH_DELTA, i).double()
                c = ref.buffer(gi, r, g.BATCH_DELTA, i).double()
                assert (torch.linalg.vector_norm(a - c) / torch.linalg.vector_norm(c)).item() < 2e-6


def test_batch_workload_size_classes(ctx):
    """The batch's own size classes and setup (128^3, 192^3 and 256^3 with
    L = 1000 Mpc/h, z = 1, n <= 4, FP32, 20 bins, the tree-level bispectrum of
    20 equilateral and 19 squeezed triangles, autotuned launch variants), with
    2, 2 and 1 realisations in one graph: every realisation's delta_n and
    theta_n against the oracle run realisation by realisation, its spectra in
    every bin (bound derived from the field tolerance, as for the benchmark
    step), and the bispectrum of the two lowest shells against direct
    triangle enumeration, with exact triangle counts."""
    box, nmax, nbins = 1000.0, 4, 20
    dz = oracle.growth(0.279, 0.721, 1.0)
    amp = oracle.sigma8_amp(0.8, NS, GAMMA)
    groups = []
    for i, (n, nreal) in enumerate(((128, 2), (192, 2), (256, 1))):
        cut = g.cut_n2max(n, box)
        grid = g.Grid(n, box, g.cube_kc(cut), g.F32)
        lp = g.LinearSpectrum(amp=amp, ns=NS, gamma=GAMMA, growth=dz, n2max=cut, seed=40 + i, stream=0)
        edges = g.linear_edges(nbins, n, 3, cut)
        pairs = [(a, b) for a in range(nmax) for b in range(a, nmax)]
        tris = [(b, b, b) for b in range(nbins)] + [(b, b, 0) for b in range(1, nbins)]
        terms = [c + (t,) for t in range(len(tris)) for c in ((0, 0, 1), (0, 1, 0), (1, 0, 0))]
        groups.append(g.BatchGroup(grid, nreal, nmax, cut, lp, pairs, edges, tris, terms))
    b = g.Batch(ctx, groups, tune=True)
    b.run()
    ctx.sync()
    t = TOL[g.F32]
    for gi, bg in enumerate(groups):
        grid, lp = bg.grid, bg.lin
        low = [k for k, tr in enumerate(bg.tris) if max(tr) <= 1]
        low_terms = [c + (j,) for j, k in enumerate(low) for c in ((0, 0, 1), (0, 1, 0), (1, 0, 0))]
        nt = b.out[gi]["ntriangles"].cpu().numpy()
        for r in range(bg.nreal):
            d1 = oracle.linear_field(grid.n, grid.box, lp.amp, lp.ns, lp.gamma, lp.growth, lp.n2max, lp.seed,
                                     lp.stream + r)
            rd, rt, rdk, _ = oracle.orders(d1, grid.box, nmax, lp.n2max, bg.n2max2)
            for i in range(nmax):
                ed = rel_l2(b.buffer(gi, r, g.BATCH_DELTA, i).cpu().numpy(), rd[i])
                et = rel_l2(b.buffer(gi, r, g.BATCH_THETA, i).cpu().numpy(), rt[i])
                print("batch N=%d realisation %d order %d: rel L2 delta %.2e theta %.2e" % (grid.n, r, i + 1, ed, et),
                      flush=True)
                assert ed < t and et < t, (grid.n, r, i + 1, ed, et)
            rpk, _, rnm = oracle.power(list(rdk), grid.box, bg.pairs, bg.edges)
            pbar = [oracle.power([rdk[a]], grid.box, [(0, 0)], [1, lp.n2max + 1])[0][0, 0] for a in range(nmax)]
            pk = b.buffer(gi, r, g.BATCH_PK).cpu().numpy()
            ok = rnm > 0
            for p, (a, c) in enumerate(bg.pairs):
                paa, pcc = rpk[bg.pairs.index((a, a))], rpk[bg.pairs.index((c, c))]
                bound = t * (np.sqrt(paa * pbar[c]) + np.sqrt(pbar[a] * pcc)) + t * t * np.sqrt(pbar[a] * pbar[c])
                assert np.all(np.abs(pk[p] - rpk[p])[ok] <= bound[ok]), (grid.n, r, a + 1, c + 1)
            rbk, rnt = oracle.bispectrum(list(rdk[:2]), grid.box, [bg.tris[k] for k in low], low_terms, bg.edges)
            sbk, _ = oracle.bispectrum([np.abs(x) for x in rdk[:2]], grid.box, [bg.tris[k] for k in low], low_terms,
                                       bg.edges)
            assert np.array_equal(nt[low], rnt), grid.n
            bk = b.buffer(gi, r, g.BATCH_BK).cpu().numpy()
            got = np.concatenate([bk[3 * k: 3 * k + 3] for k in low])
            has = np.repeat(rnt > 0, 3)
            assert np.all(np.abs(got - rbk)[has] <= 1e-5 * sbk[has]), grid.n
        assert np.array_equal(nt, np.rint(nt))
