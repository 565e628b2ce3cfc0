"""CPU tests of the C ABI: the library loads, exports every symbol the header
declares, its host helpers agree with exact arithmetic and quadrature, and
argument validation fails before any GPU work (no GPU needed)."""
import ctypes
import math
import os
import re
from fractions import Fraction

import numpy as np
import pytest
from scipy import integrate

import paper_1807_04215_amd as g

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gridspt.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gridspt_\w+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = g.lib()
    syms = declared_symbols()
    assert len(syms) >= 20
    for s in syms:
        assert hasattr(lib, s), s


def test_status_strings_and_version():
    lib = g.lib()
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert lib.gridspt_status_string(code)
    assert b"NaN" in lib.gridspt_status_string(-6)
    assert lib.gridspt_version() >= 100


@pytest.mark.parametrize("n", [6, 16, 64, 192, 256, 512, 1024])
def test_strict_cut_is_exact(n):
    c = g.cut_n2max(n, 1000.0)
    assert 9 * c < n * n <= 9 * (c + 1)


def test_absolute_cut_matches_paper_reading():
    # |k| <= kcut with kcut = 4/3 h/Mpc on 512^3, L = 1000: floor((kcut L / 2 pi)^2)
    c = g.cut_n2max(512, 1000.0, 4.0 / 3.0)
    x = (4.0 / 3.0) * 1000.0 / (2 * math.pi)
    assert c == math.floor(x * x)
    assert g.cube_kc(c) == math.isqrt(c)


def test_cube_kc_integer_sqrt():
    for v in [1, 2, 3, 4, 8, 9, 455, 7281, 116508, 10 ** 12 - 1, 10 ** 12]:
        assert g.cube_kc(v) == math.isqrt(v)


@pytest.mark.parametrize("n,nbins", [(64, 32), (256, 64), (192, 20), (1024, 64)])
def test_linear_edges_exact(n, nbins):
    cut = g.cut_n2max(n, 1.0)
    e = g.linear_edges(nbins, n, 3, cut)
    assert e[0] == 1 and e[-1] == min((n * n) // 9 + 1, cut + 1)
    for b in range(1, nbins):
        t = Fraction(b * n, 3 * nbins) ** 2
        want = max(1, math.ceil(t))
        assert e[b] == want, b


def test_sigma8_and_growth_against_scipy():
    ns, gam = 0.96, 0.21

    def p0(k, a):
        q = k / gam
        t = math.log1p(2.34 * q) / (2.34 * q) * (1 + 3.89 * q + (16.1 * q) ** 2 + (5.46 * q) ** 3 + (6.71 * q) ** 4) ** -0.25
        return a * k ** ns * t * t

    def s2(a):
        f = lambda lk: (math.exp(lk) ** 3 * p0(math.exp(lk), a)
                        * (3 * (math.sin(8 * math.exp(lk)) - 8 * math.exp(lk) * math.cos(8 * math.exp(lk)))
                           / (8 * math.exp(lk)) ** 3) ** 2)
        v, _ = integrate.quad(f, math.log(1e-6), math.log(1e4), limit=4000, epsabs=0, epsrel=1e-12)
        return v / (2 * math.pi ** 2)

    a = g.sigma8_amp(0.8, ns, gam)
    assert math.isclose(math.sqrt(s2(a)), 0.8, rel_tol=1e-9)
    assert math.isclose(g.growth(1.0, 0.0, 1.0), 0.5, rel_tol=1e-12)
    om, ol = 0.279, 0.721
    e = lambda x: math.sqrt(om / x ** 3 + ol)
    d = lambda aa: e(aa) * integrate.quad(lambda x: 1 / (x * e(x)) ** 3, 0, aa, epsabs=0, epsrel=1e-13)[0]
    assert math.isclose(g.growth(om, ol, 1.0), d(0.5) / d(1.0), rel_tol=1e-10)


def _grid(n=64, kc=21, dtype=0, box=500.0):
    return g._Grid(n, dtype, box, kc, 0)


def test_validation_before_any_gpu_work():
    lib = g.lib()
    h = ctypes.c_void_p()
    assert lib.gridspt_create(ctypes.byref(h), None) == 0
    try:
        G = _grid()
        ws = ctypes.c_void_p(4096 * 256)       # aligned but never touched: validation fails first
        d = (ctypes.c_void_p * 3)(4096 * 512, 4096 * 768, 4096 * 1024)
        # nmax out of range
        assert lib.gridspt_orders(h, ctypes.byref(G), 0, 455, 455, ws, d, d, None, None, ws, 1 << 40) == -1
        assert lib.gridspt_orders(h, ctypes.byref(G), 6, 455, 455, ws, d, d, None, None, ws, 1 << 40) == -1
        # cut at or beyond Nyquist, or outside the cube
        assert lib.gridspt_orders(h, ctypes.byref(G), 3, 1024, 455, ws, d, d, None, None, ws, 1 << 40) == -1
        assert lib.gridspt_orders(h, ctypes.byref(G), 3, 455, 600, ws, d, d, None, None, ws, 1 << 40) == -1
        # misaligned pointer
        bad = (ctypes.c_void_p * 3)(4096 * 512 + 4, 4096 * 768, 4096 * 1024)
        assert lib.gridspt_orders(h, ctypes.byref(G), 3, 455, 455, ws, bad, d, None, None, ws, 1 << 40) == -4
        # workspace too small / missing
        assert lib.gridspt_orders(h, ctypes.byref(G), 3, 455, 455, ws, d, d, None, None, ws, 1024) == -3
        assert lib.gridspt_orders(h, ctypes.byref(G), 3, 455, 455, ws, d, d, None, None, None, 1 << 40) == -3
        # grid: odd, non power of two, kc too large, bad dtype, bad box
        assert lib.gridspt_workspace_bytes(ctypes.byref(_grid(n=63)), 3, 0) == -1
        assert lib.gridspt_workspace_bytes(ctypes.byref(_grid(n=144, kc=47)), 3, 0) == -2  # 9 * 16: not built
        assert lib.gridspt_workspace_bytes(ctypes.byref(_grid(n=200, kc=60)), 3, 0) == -2  # factor 5
        assert lib.gridspt_workspace_bytes(ctypes.byref(_grid(n=192, kc=63)), 3, 0) > 0    # 3 * 64: radix-3 plan
        assert lib.gridspt_workspace_bytes(ctypes.byref(_grid(n=48, kc=15)), 3, 0) > 0
        assert lib.gridspt_workspace_bytes(ctypes.byref(_grid(kc=32)), 3, 0) == -1
        assert lib.gridspt_workspace_bytes(ctypes.byref(_grid(dtype=7)), 3, 0) == -1
        assert lib.gridspt_workspace_bytes(ctypes.byref(_grid(box=-1.0)), 3, 0) == -1
        # power: bad pair index, decreasing edges, edge[0] = 0
        f = (ctypes.c_void_p * 2)(4096 * 512, 4096 * 768)
        pairs = (ctypes.c_int32 * 2)(0, 2)
        edges = (ctypes.c_int64 * 3)(1, 5, 9)
        out = ctypes.c_void_p(4096 * 2048)
        assert lib.gridspt_power(h, ctypes.byref(G), 2, f, 1, pairs, 2, edges, out, None, None, ws, 1 << 30) == -1
        pairs = (ctypes.c_int32 * 2)(0, 1)
        dec = (ctypes.c_int64 * 3)(1, 9, 5)
        assert lib.gridspt_power(h, ctypes.byref(G), 2, f, 1, pairs, 2, dec, out, None, None, ws, 1 << 30) == -1
        zero = (ctypes.c_int64 * 3)(0, 5, 9)
        assert lib.gridspt_power(h, ctypes.byref(G), 2, f, 1, pairs, 2, zero, out, None, None, ws, 1 << 30) == -1
        # bispectrum: shells beyond the cube, term pointing at a missing triangle
        tb = (ctypes.c_int32 * 3)(0, 0, 1)
        tm = (ctypes.c_int32 * 4)(0, 0, 0, 1)
        assert lib.gridspt_bispectrum(h, ctypes.byref(G), 2, f, 1, tb, 1, tm, 2, edges, out, out, ws, 1 << 30) == -1
        far = (ctypes.c_int64 * 3)(1, 5, 600)
        tm = (ctypes.c_int32 * 4)(0, 0, 0, 0)
        assert lib.gridspt_bispectrum(h, ctypes.byref(G), 2, f, 1, tb, 1, tm, 2, far, out, out, ws, 1 << 30) == -1
        # linear field: non-positive Gamma
        lp = g._LinPk(1.0, 0.96, 0.0, 1.0, 455, 1, 0)
        assert lib.gridspt_linear_field(h, ctypes.byref(G), ctypes.byref(lp), ws, None, ws, 1 << 40) == -1
        # grid flags: only GRIDSPT_CHECK_FINITE is defined
        G2 = _grid()
        G2.flags = 2
        assert lib.gridspt_orders(h, ctypes.byref(G2), 3, 455, 455, ws, d, d, None, None, ws, 1 << 40) == -1
        assert lib.gridspt_workspace_bytes(ctypes.byref(G), 3, 2) == -1
        # half layout: misaligned or missing pointers
        assert lib.gridspt_spectrum_half(h, ctypes.byref(G), ctypes.c_void_p(4096 * 256 + 8), ws) == -4
        assert lib.gridspt_spectrum_half(h, ctypes.byref(G), ws, None) == -4
        assert lib.gridspt_spectrum_half(None, ctypes.byref(G), ws, ws) == -1
    finally:
        lib.gridspt_destroy(h)


def test_workspace_flags_and_profile_orders():
    """The finiteness check's flag word is part of every workspace, so the flag
    does not change the size; a fresh context reports no per-order timing."""
    lib = g.lib()
    G = _grid()
    base = lib.gridspt_workspace_bytes(ctypes.byref(G), 3, 0)
    assert base > 0
    assert lib.gridspt_workspace_bytes(ctypes.byref(G), 3, g.CHECK_FINITE) == base
    G.flags = g.CHECK_FINITE
    assert lib.gridspt_workspace_bytes(ctypes.byref(G), 3, 0) == base
    h = ctypes.c_void_p()
    assert lib.gridspt_create(ctypes.byref(h), None) == 0
    try:
        ms = (ctypes.c_double * 9)()
        assert lib.gridspt_profile_orders(h, 9, ms, None) == 0
        assert all(v == 0.0 for v in ms)
        assert lib.gridspt_profile_orders(None, 9, ms, None) == -1
    finally:
        lib.gridspt_destroy(h)


def test_bispectrum_rejects_triangles_that_close_only_modulo_n():
    """Eq. 22-23 sum over exactly closed triangles; the FFT estimator closes them
    modulo N.  A triangle whose three shell radii add up to N or more could
    close through a wrap, so the call rejects it; below N it proceeds (here
    to the workspace check, with no device work)."""
    lib = g.lib()
    h = ctypes.c_void_p()
    assert lib.gridspt_create(ctypes.byref(h), None) == 0
    try:
        G = _grid(n=64, kc=31)
        f = (ctypes.c_void_p * 1)(4096 * 512)
        out = ctypes.c_void_p(4096 * 2048)
        ws = ctypes.c_void_p(4096 * 256)
        edges = (ctypes.c_int64 * 3)(1, 400, 962)     # shell radii 19 and 31
        for tri, want in (((0, 0, 0), -3), ((0, 0, 1), -1), ((1, 1, 1), -1), ((1, 0, 0), -1)):
            tb = (ctypes.c_int32 * 3)(*tri)
            tm = (ctypes.c_int32 * 4)(0, 0, 0, 0)
            rc = lib.gridspt_bispectrum(h, ctypes.byref(G), 1, f, 1, tb, 1, tm, 2, edges, out, out, ws, 1024)
            assert rc == want, (tri, rc)
        # the same rule for a batch group (19 + 19 + 31 = 69 >= 64)
        grp, keep = _bgroup(n=64, kc=31, n2=961, edges=(1, 400, 962), tris=(0, 0, 1), terms=(0, 0, 0, 0))
        assert lib.gridspt_batch_workspace_bytes(1, ctypes.byref(grp)) == -1
        grp, keep = _bgroup(n=64, kc=31, n2=961, edges=(1, 400, 962), tris=(0, 0, 0), terms=(0, 0, 0, 0))
        assert lib.gridspt_batch_workspace_bytes(1, ctypes.byref(grp)) > 0
    finally:
        lib.gridspt_destroy(h)


def test_set_tuning_accepts_only_compiled_variants():
    """gridspt_set_tuning pins a compiled launch variant (host-side bookkeeping, no GPU work)."""
    lib = g.lib()
    h = ctypes.c_void_p()
    assert lib.gridspt_create(ctypes.byref(h), None) == 0
    try:
        f32_64 = _grid(n=64, kc=21, dtype=g.F32)
        f64_64 = _grid(n=64, kc=21, dtype=g.F64)
        f32_96 = _grid(n=96, kc=31, dtype=g.F32)
        f32_48 = _grid(n=48, kc=15, dtype=g.F32)
        assert lib.gridspt_set_tuning(None, ctypes.byref(f32_64), 0) == -1
        for v, want in ((0, 0), (1, 0), (4, 0), (5, 0), (2, -1), (3, -1), (8, -1)):
            assert lib.gridspt_set_tuning(h, ctypes.byref(f32_64), v) == want, v
        assert lib.gridspt_set_tuning(h, ctypes.byref(f64_64), 1) == -1
        assert lib.gridspt_set_tuning(h, ctypes.byref(f32_96), 2) == 0
        assert lib.gridspt_set_tuning(h, ctypes.byref(f32_96), 4) == -1
        assert lib.gridspt_set_tuning(h, ctypes.byref(f32_48), 1) == -1
        assert lib.gridspt_set_tuning(h, ctypes.byref(_grid(n=63)), 0) == -1
        # the pinned variant is what the context reports for every tuned pass kind
        assert lib.gridspt_set_tuning(h, ctypes.byref(f32_64), 5) == 0
        var = (ctypes.c_int32 * 16)()
        k = lib.gridspt_tuning(h, ctypes.byref(f32_64), 16, None, var, None)
        assert k > 0 and all(var[i] == 5 for i in range(k))
        k = lib.gridspt_tuning(h, ctypes.byref(f32_96), 16, None, var, None)
        assert k > 0 and all(var[i] == 2 for i in range(k))
    finally:
        lib.gridspt_destroy(h)


def test_workspace_sizes_follow_layout():
    G = _grid(n=1024, kc=341, dtype=0, box=2000.0)
    n, kz, ky = 1024, 342, 683
    a = max(4 * kz * n * n, 5 * kz * n * ky) * 8
    b = max(4 * kz * ky * n, 5 * n * n * kz) * 8
    u = 9 * n ** 3 * 4                # u_1 .. u_3: the order-5 product pass holds u_4 in registers
    got = g.lib().gridspt_workspace_bytes(ctypes.byref(G), 5, 0)
    amp = (341 + 1) ** 2 * 8          # radial amplitude table
    assert a + b + u + amp <= got <= a + b + u + amp + 5 * 256 + n * 8
    assert g.lib().gridspt_cube_elems(ctypes.byref(G)) == kz * ky * ky


def _bgroup(n=32, kc=10, nreal=2, nmax=3, n2=100, pairs=(0, 0), edges=(1, 10, 50, 101), tris=None, terms=None):
    import numpy as np
    keep = [np.asarray(pairs, dtype=np.int32), np.asarray(edges, dtype=np.int64)]
    tb = np.asarray(tris if tris is not None else [], dtype=np.int32)
    tt = np.asarray(terms if terms is not None else [], dtype=np.int32)
    keep += [tb, tt]
    grp = g._BatchGroup(g._Grid(n, 0, 200.0, kc, 0), nreal, nmax, n2, g._LinPk(1.0, 0.96, 0.21, 1.0, n2, 1, 0),
                        keep[0].size // 2, keep[0].ctypes.data, keep[1].size - 1, keep[1].ctypes.data,
                        tb.size // 3, tb.ctypes.data if tb.size else None, tt.size // 4,
                        tt.ctypes.data if tt.size else None)
    return grp, keep


def test_batch_validation_and_layout():
    """Batch plans are validated and laid out on the host (no device work)."""
    lib = g.lib()
    grp, keep = _bgroup()
    one = lib.gridspt_batch_workspace_bytes(1, ctypes.byref(grp))
    assert one > 0 and one % 256 == 0
    # twice the realisations: twice the arena
    grp2, keep2 = _bgroup(nreal=4)
    assert lib.gridspt_batch_workspace_bytes(1, ctypes.byref(grp2)) == 2 * one
    # the per-realisation arena holds at least the fields, workspace and spectra
    n, nmax = 32, 3
    assert one // 2 >= g.lib().gridspt_workspace_bytes(ctypes.byref(g._Grid(n, 0, 200.0, 10, 0)), nmax, 0) \
        + (2 * nmax - 1) * n ** 3 * 4
    arr = (g._BatchGroup * 2)(grp, grp2)
    assert lib.gridspt_batch_workspace_bytes(2, arr) == 3 * one
    # invalid: pair index beyond nmax, nreal 0, nmax 6, mask beyond the cube, bad size, bad term
    for kw in (dict(pairs=(0, 3)), dict(nreal=0), dict(nmax=6), dict(n2=200), dict(n=144, kc=10),
               dict(tris=(0, 0, 1), terms=(0, 0, 0, 1))):
        bad, k = _bgroup(**kw)
        rc = lib.gridspt_batch_workspace_bytes(1, ctypes.byref(bad))
        assert rc in (-1, -2), (kw, rc)
    assert lib.gridspt_batch_workspace_bytes(0, ctypes.byref(grp)) == -1
    # create: missing outputs or workspace are rejected before any device work
    h = ctypes.c_void_p()
    assert lib.gridspt_create(ctypes.byref(h), None) == 0
    try:
        out = g._BatchOut()
        b = ctypes.c_void_p()
        ws = ctypes.c_void_p(4096 * 256)
        assert lib.gridspt_batch_create(h, 1, ctypes.byref(grp), ctypes.byref(out), ws, one, 0, ctypes.byref(b)) == -1
        out.pk_mean = 4096 * 512
        assert lib.gridspt_batch_create(h, 1, ctypes.byref(grp), ctypes.byref(out), ws, one - 256, 0,
                                        ctypes.byref(b)) == -3
        out.pk_std = 4096 * 512 + 8
        assert lib.gridspt_batch_create(h, 1, ctypes.byref(grp), ctypes.byref(out), ws, one, 0, ctypes.byref(b)) == -4
        assert lib.gridspt_batch_create(h, 1, ctypes.byref(grp), ctypes.byref(out), ws, one, 8, ctypes.byref(b)) == -1
        assert not b.value
    finally:
        lib.gridspt_destroy(h)


class _HostCtx:
    """Stands in for a Context in host-only checks of the binding's argument tests."""
    device = None

    def _uses(self, t):
        raise AssertionError("a rejected tensor reached the stream bookkeeping")


def test_binding_rejects_wrong_tensors_before_any_call():
    """Every tensor address the binding passes on is checked first: a wrong
    dtype (FP32 into an F64 grid), shape (a smaller out= buffer), layout (a
    transposed view) or device (a CPU tensor) raises instead of reaching a
    kernel that would read or write past the allocation."""
    import torch
    ctx = _HostCtx()
    grid = g.Grid(16, 100.0, 5, g.F64)
    ok = torch.zeros(grid.real_shape, dtype=torch.float64)
    with pytest.raises(TypeError, match="dtype"):
        g._real(ctx, grid, ok.float(), "delta1")
    with pytest.raises(ValueError, match="shape"):
        g._real(ctx, grid, torch.zeros((16, 16, 8), dtype=torch.float64), "out")
    with pytest.raises(ValueError, match="shape"):
        g._cube(ctx, grid, torch.zeros((6, 11, 11), dtype=torch.float64), "out_k")   # no trailing complex axis
    with pytest.raises(ValueError, match="contiguous"):
        g._real(ctx, grid, ok.transpose(0, 2), "delta1")
    with pytest.raises(ValueError, match="GPU"):
        g._real(ctx, grid, ok, "delta1")
    with pytest.raises(ValueError, match="missing"):
        g._real_array(ctx, grid, [None, ok], "delta")
    with pytest.raises(TypeError):
        g._real(ctx, grid, ok.numpy(), "delta1")
