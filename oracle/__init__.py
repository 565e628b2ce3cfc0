"""GridSPT reference oracle -- test infrastructure only.

A plain double-precision CPU implementation of the GridSPT hot path (Taruya,
Nishimichi & Jeong 2018, arXiv:1807.04215), in C (``gridspt_oracle.c``) with
this thin ctypes wrapper.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import it; the GPU library never does.

Layouts: real fields are ``float64[N, N, N]`` indexed ``[ix, iy, iz]``;
spectra are the half layout ``complex128[N, N, N//2 + 1]`` with the forward
transform normalised by ``N**-3`` (Sec. II C, Eq. 17).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gridspt_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP over pencils); returns the .so path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        lib = ctypes.CDLL(_LIB)
        c_i64p = ctypes.POINTER(ctypes.c_int64)
        c_dp = ctypes.c_void_p
        lib.or_set_threads.argtypes = [ctypes.c_int]
        lib.or_set_threads.restype = ctypes.c_int
        lib.or_fft3d.argtypes = [ctypes.c_int, c_dp, ctypes.c_int]
        lib.or_philox4x64_10.argtypes = [c_dp, c_dp, c_dp]
        lib.or_unit_gaussian.argtypes = [ctypes.c_uint64] * 3
        lib.or_unit_gaussian.restype = ctypes.c_double
        lib.or_bbks.argtypes = [ctypes.c_double]
        lib.or_bbks.restype = ctypes.c_double
        lib.or_p0.argtypes = [ctypes.c_double] * 4
        lib.or_p0.restype = ctypes.c_double
        lib.or_sigma_r.argtypes = [ctypes.c_double] * 4
        lib.or_sigma_r.restype = ctypes.c_double
        lib.or_sigma8_amp.argtypes = [ctypes.c_double] * 3
        lib.or_sigma8_amp.restype = ctypes.c_double
        lib.or_growth.argtypes = [ctypes.c_double] * 3
        lib.or_growth.restype = ctypes.c_double
        lib.or_linear_field.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint64, c_dp]
        lib.or_linear_field.restype = ctypes.c_int
        for name in ("or_orders_dform", "or_orders_pform"):
            f = getattr(lib, name)
            f.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int64,
                          ctypes.c_int64, c_dp, c_dp, c_dp, c_dp, c_dp]
            f.restype = ctypes.c_int
        lib.or_power.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int, c_dp,
                                 ctypes.c_int, c_dp, ctypes.c_int, c_i64p, c_dp, c_dp, c_dp]
        lib.or_power.restype = ctypes.c_int
        lib.or_bispectrum.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int, c_dp,
                                      ctypes.c_int, c_dp, ctypes.c_int, c_dp, ctypes.c_int,
                                      c_i64p, c_dp, c_dp]
        lib.or_bispectrum.restype = ctypes.c_int
        lib.or_sum_orders.argtypes = [ctypes.c_long, ctypes.c_int, c_dp, c_dp, c_dp]
        lib.or_group_gaussians.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, c_dp]
        lib.or_linear_modes.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_double, ctypes.c_int64, ctypes.c_uint64,
                                        ctypes.c_uint64, ctypes.c_int, c_dp, c_dp]
        lib.or_linear_modes.restype = ctypes.c_int
        lib.or_noise_field.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_int64, c_dp, c_dp]
        lib.or_noise_field.restype = ctypes.c_int
        lib.or_adjoint_dform.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int64,
                                         ctypes.c_int64, c_dp, c_dp, c_dp]
        lib.or_adjoint_dform.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def set_threads(n: int = 0) -> int:
    """Set the OpenMP thread count (0 keeps the default); returns the count in use."""
    return _load().or_set_threads(int(n))


# --------------------------------------------------------------------------
# transforms and generator
# --------------------------------------------------------------------------

def fft3d(a: np.ndarray, sign: int = -1) -> np.ndarray:
    """Unnormalised 3D DFT of a full complex cube (sign -1 forward, +1 inverse)."""
    out = np.ascontiguousarray(a, dtype=np.complex128).copy()
    _load().or_fft3d(out.shape[0], _ptr(out), int(sign))
    return out


def forward(f: np.ndarray) -> np.ndarray:
    """Half-layout spectrum N^-3 sum_x f(x) e^{-ik.x} of a real cube (oracle DFT)."""
    n = f.shape[0]
    full = fft3d(f.astype(np.complex128), -1) / float(n) ** 3
    return np.ascontiguousarray(full[:, :, : n // 2 + 1])


def philox4x64_10(ctr, key) -> np.ndarray:
    c = np.asarray(ctr, dtype=np.uint64).copy()
    k = np.asarray(key, dtype=np.uint64).copy()
    out = np.zeros(4, dtype=np.uint64)
    _load().or_philox4x64_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def unit_gaussian(seed: int, stream: int, cell: int) -> float:
    return _load().or_unit_gaussian(seed, stream, cell)


def bbks(q: float) -> float:
    return _load().or_bbks(float(q))


def p0(k: float, amp: float, ns: float, gamma: float) -> float:
    return _load().or_p0(float(k), float(amp), float(ns), float(gamma))


def sigma_r(R: float, amp: float, ns: float, gamma: float) -> float:
    return _load().or_sigma_r(float(R), float(amp), float(ns), float(gamma))


def sigma8_amp(sigma8: float, ns: float, gamma: float) -> float:
    return _load().or_sigma8_amp(float(sigma8), float(ns), float(gamma))


def growth(om: float, ol: float, z: float) -> float:
    return _load().or_growth(float(om), float(ol), float(z))


def group_gaussians(seed: int, stream: int, q: int) -> np.ndarray:
    out = np.zeros(4)
    _load().or_group_gaussians(seed, stream, q, _ptr(out))
    return out


# --------------------------------------------------------------------------
# hot path
# --------------------------------------------------------------------------

def linear_modes(n: int, box: float, amp: float, ns: float, gamma: float, growth_d: float, n2max1: int,
                 seed: int, modes, stream: int = 0) -> np.ndarray:
    """The linear field's spectrum at single signed modes by the direct DFT
    sum over all n^3 noise cells (no FFT); for sampling large grids."""
    m = np.ascontiguousarray(np.asarray(modes, dtype=np.int32).reshape(-1))
    out = np.zeros(m.size // 3, dtype=np.complex128)
    _load().or_linear_modes(n, box, amp, ns, gamma, growth_d, int(n2max1), int(seed), int(stream),
                            m.size // 3, _ptr(m), _ptr(out))
    return out


def linear_field(n: int, box: float, amp: float, ns: float, gamma: float, growth_d: float,
                 n2max1: int, seed: int, stream: int = 0) -> np.ndarray:
    """Step (1) of Sec. II C: seeded Gaussian delta_1(x) with L^3<|d(k)|^2> = D^2 P0."""
    out = np.zeros((n, n, n), dtype=np.float64)
    rc = _load().or_linear_field(n, box, amp, ns, gamma, growth_d, int(n2max1), int(seed),
                                 int(stream), _ptr(out))
    if rc != 0:
        raise MemoryError("oracle linear_field failed")
    return out


def noise_field(w: np.ndarray, box: float, amp: float, ns: float, gamma: float, growth_d: float,
                n2max1: int) -> np.ndarray:
    """Step (1) of Sec. II C from a given white-noise field w(x)."""
    wc = np.ascontiguousarray(w, dtype=np.float64)
    out = np.zeros_like(wc)
    if _load().or_noise_field(wc.shape[0], box, amp, ns, gamma, growth_d, int(n2max1), _ptr(wc), _ptr(out)) != 0:
        raise MemoryError("oracle noise_field failed")
    return out


def adjoint(w: np.ndarray, box: float, amp: float, ns: float, gamma: float, growth_d: float, nmax: int,
            n2max1: int, n2max2: int, gdelta) -> np.ndarray:
    """Reverse mode of noise -> delta_1..delta_nmax (linear field and D-form
    recursion): the gradient dJ/dw(x) of a scalar J given gdelta[n-1] = dJ/d delta_n(x)."""
    wc = np.ascontiguousarray(w, dtype=np.float64)
    n = wc.shape[0]
    g = np.ascontiguousarray(np.asarray(gdelta, dtype=np.float64).reshape(nmax, n, n, n))
    out = np.zeros_like(wc)
    if _load().or_adjoint_dform(n, box, amp, ns, gamma, growth_d, nmax, int(n2max1), int(n2max2), _ptr(wc),
                                _ptr(g), _ptr(out)) != 0:
        raise MemoryError("oracle adjoint failed")
    return out


def orders(delta1: np.ndarray, box: float, nmax: int, n2max1: int, n2max2: int,
           form: str = "D", spectra: bool = True):
    """Recursion of Eq. 10/11 up to order nmax.

    Returns (delta, theta, delta_k, theta_k): real arrays [nmax, N, N, N] and,
    if ``spectra``, half-layout spectra [nmax, N, N, N//2+1] (else None).
    ``form`` "D" is the divergence form, "P" the paper's literal products.
    """
    d1 = np.ascontiguousarray(delta1, dtype=np.float64)
    n = d1.shape[0]
    delta = np.zeros((nmax, n, n, n), dtype=np.float64)
    theta = np.zeros_like(delta)
    dk = tk = None
    if spectra:
        dk = np.zeros((nmax, n, n, n // 2 + 1), dtype=np.complex128)
        tk = np.zeros_like(dk)
    fn = _load().or_orders_dform if form.upper() == "D" else _load().or_orders_pform
    rc = fn(n, float(box), int(nmax), int(n2max1), int(n2max2), _ptr(d1), _ptr(delta),
            _ptr(theta), _ptr(dk) if spectra else None, _ptr(tk) if spectra else None)
    if rc != 0:
        raise RuntimeError("oracle orders failed")
    return delta, theta, dk, tk


def _ptr_array(fields):
    arrs = [np.ascontiguousarray(f, dtype=np.complex128) for f in fields]
    ptrs = (ctypes.c_void_p * len(arrs))(*[a.ctypes.data for a in arrs])
    return arrs, ptrs


def power(fields_k, box: float, pairs, edges):
    """Shell-averaged cross spectra (Eq. 19-21 with the L^3 factor).

    fields_k: list of half-layout spectra; pairs: [(a, b), ...]; edges: nbins+1
    integer n^2 thresholds.  Returns (pk [npairs, nbins], kmean, nmodes).
    """
    arrs, ptrs = _ptr_array(fields_k)
    n = arrs[0].shape[0]
    pr = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1))
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int64))
    nb = e.size - 1
    npairs = pr.size // 2
    pk = np.zeros((npairs, nb))
    km = np.zeros(nb)
    nm = np.zeros(nb)
    rc = _load().or_power(n, float(box), len(arrs), ptrs, npairs, _ptr(pr), nb,
                          e.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _ptr(pk), _ptr(km), _ptr(nm))
    if rc != 0:
        raise ValueError("oracle power: bad pair index")
    return pk, km, nm


def bispectrum(fields_k, box: float, tris, terms, edges):
    """Closed-triangle sums (Eq. 22/23) by direct enumeration.

    tris: [(b1, b2, b3), ...]; terms: [(fa, fb, fc, tri), ...].
    Returns (bk [nterms], ntriangles [ntri]).
    """
    arrs, ptrs = _ptr_array(fields_k)
    n = arrs[0].shape[0]
    tb = np.ascontiguousarray(np.asarray(tris, dtype=np.int32).reshape(-1))
    tt = np.ascontiguousarray(np.asarray(terms, dtype=np.int32).reshape(-1))
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int64))
    bk = np.zeros(tt.size // 4)
    nt = np.zeros(tb.size // 3)
    rc = _load().or_bispectrum(n, float(box), len(arrs), ptrs, tb.size // 3, _ptr(tb), tt.size // 4,
                               _ptr(tt), e.size - 1, e.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                               _ptr(bk), _ptr(nt))
    if rc != 0:
        raise ValueError("oracle bispectrum: bad bin, field or triangle index")
    return bk, nt


def sum_orders(delta: np.ndarray, coef) -> np.ndarray:
    d = np.ascontiguousarray(delta, dtype=np.float64)
    c = np.ascontiguousarray(np.asarray(coef, dtype=np.float64))
    nmax = d.shape[0]
    out = np.zeros(d.shape[1:])
    _load().or_sum_orders(out.size, nmax, _ptr(d), _ptr(c), _ptr(out))
    return out


# --------------------------------------------------------------------------
# integer helpers (the readings of the cut and of the bins)
# --------------------------------------------------------------------------

def cut_n2max_strict(n: int) -> int:
    """Strict 2/3 rule: keep |n| < N/3, i.e. n^2 <= ceil(N^2 / 9) - 1."""
    return -(-n * n // 9) - 1


def cut_n2max_abs(n: int, box: float, kcut: float) -> int:
    """Absolute cut |k| <= kcut: n^2 <= floor((kcut L / 2 pi)^2)."""
    return int(np.floor((kcut * box / (2.0 * np.pi)) ** 2))


def linear_edges(nbins: int, kmax_num: int, kmax_den: int, n2max: int):
    """Linear bins on [0, k_max], k_max = (num/den) k_F, left-closed, last bin
    closed at min(k_max, cut); k = 0 excluded.  Exact integer arithmetic."""
    e = [1]
    for b in range(1, nbins):
        num = b * b * kmax_num * kmax_num
        den = nbins * nbins * kmax_den * kmax_den
        e.append(-(-num // den))
    e.append(min(kmax_num * kmax_num // (kmax_den * kmax_den) + 1, n2max + 1))
    return np.asarray(e, dtype=np.int64)


from .sparse import sparse_orders  # noqa: E402  (pure-Python Fourier-space recursion)
