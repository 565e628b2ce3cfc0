"""GridSPT on MI355X: Python binding of libgridspt (include/gridspt.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``csrc/``.  PyTorch provides device memory and the stream.  The
binding raises if the library is missing; there is no CPU fallback.

Layouts (see include/gridspt.h): real fields are ``[N, N, N]`` tensors
indexed ``[x, y, z]``; spectra are cube-layout complex tensors of shape
``[Kc + 1, 2Kc + 1, 2Kc + 1]`` indexed ``[kz, ky, kx]`` with the two last axes
in fftfreq order, stored as real tensors with a trailing axis of 2.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgridspt.so")

F32, F64 = 0, 1
CHECK_FINITE = 1  # grid flag: input fields are checked for NaN / infinity (GRIDSPT_ENONFINITE)
_STATUS = {0: "ok", -1: "invalid argument", -2: "unsupported configuration", -3: "workspace too small",
           -4: "null or misaligned device pointer", -5: "HIP runtime error",
           -6: "an input field holds a NaN or an infinity"}
ENONFINITE = -6


class GridSPTError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__("%s: %s (status %d)" % (where, _STATUS.get(status, "unknown"), status))
        self.status = status


class _Grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("dtype", ctypes.c_int32), ("box", ctypes.c_double),
                ("kc", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class _LinPk(ctypes.Structure):
    _fields_ = [("amp", ctypes.c_double), ("ns", ctypes.c_double), ("gamma", ctypes.c_double),
                ("growth", ctypes.c_double), ("n2max", ctypes.c_int64), ("seed", ctypes.c_uint64),
                ("stream", ctypes.c_uint64)]


class _BatchGroup(ctypes.Structure):
    _fields_ = [("grid", _Grid), ("nreal", ctypes.c_int32), ("nmax", ctypes.c_int32), ("n2max2", ctypes.c_int64),
                ("lin", _LinPk), ("npairs", ctypes.c_int32), ("pairs", ctypes.c_void_p), ("nbins", ctypes.c_int32),
                ("edge_n2", ctypes.c_void_p), ("ntri", ctypes.c_int32), ("tri_bins", ctypes.c_void_p),
                ("nterms", ctypes.c_int32), ("terms", ctypes.c_void_p)]


class _BatchOut(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("pk_mean", "pk_std", "kmean", "nmodes", "bk_mean", "bk_std",
                                               "ntriangles")]


BATCH_TUNE, BATCH_EAGER = 1, 2
BATCH_DELTA, BATCH_THETA, BATCH_DELTA_K, BATCH_PK, BATCH_BK = 0, 1, 2, 3, 4

_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libgridspt.so is not built (run __graft_entry__.build() or "
                              "python paper_1807_04215_amd/build.py)")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        gp = ctypes.POINTER(_Grid)
        sig = {
            "gridspt_create": ([ctypes.POINTER(vp), vp], ctypes.c_int),
            "gridspt_destroy": ([vp], None),
            "gridspt_sync": ([vp], ctypes.c_int),
            "gridspt_status_string": ([ctypes.c_int], ctypes.c_char_p),
            "gridspt_version": ([], i32),
            "gridspt_cut_n2max": ([i32, dbl, dbl], i64),
            "gridspt_cube_kc": ([i64], i32),
            "gridspt_cube_elems": ([gp], i64),
            "gridspt_linear_edges": ([i32, i64, i64, i64, vp], ctypes.c_int),
            "gridspt_sigma8_amp": ([dbl, dbl, dbl, ctypes.POINTER(dbl)], ctypes.c_int),
            "gridspt_growth": ([dbl, dbl, dbl, ctypes.POINTER(dbl)], ctypes.c_int),
            "gridspt_workspace_bytes": ([gp, i32, ctypes.c_uint32], i64),
            "gridspt_spectrum_half": ([vp, gp, vp, vp], ctypes.c_int),
            "gridspt_profile_orders": ([vp, i32, vp, vp], ctypes.c_int),
            "gridspt_linear_field": ([vp, gp, ctypes.POINTER(_LinPk), vp, vp, vp, i64], ctypes.c_int),
            "gridspt_forward": ([vp, gp, i64, vp, vp, vp, i64], ctypes.c_int),
            "gridspt_orders": ([vp, gp, i32, i64, i64, vp, vp, vp, vp, vp, vp, i64], ctypes.c_int),
            "gridspt_sum_orders": ([vp, gp, i32, vp, vp, vp], ctypes.c_int),
            "gridspt_power_workspace_bytes": ([gp, i32, i32], i64),
            "gridspt_power": ([vp, gp, i32, vp, i32, vp, i32, vp, vp, vp, vp, vp, i64], ctypes.c_int),
            "gridspt_power_static": ([vp, gp, i32, vp, i32, vp, i32, vp, vp, vp, vp], ctypes.c_int),
            "gridspt_bispectrum_workspace_bytes": ([gp, i32, vp, i32, vp], i64),
            "gridspt_bispectrum": ([vp, gp, i32, vp, i32, vp, i32, vp, i32, vp, vp, vp, vp, i64], ctypes.c_int),
            "gridspt_batch_workspace_bytes": ([i32, ctypes.POINTER(_BatchGroup)], i64),
            "gridspt_batch_create": ([vp, i32, ctypes.POINTER(_BatchGroup), ctypes.POINTER(_BatchOut), vp, i64,
                                      ctypes.c_uint32, ctypes.POINTER(vp)], ctypes.c_int),
            "gridspt_batch_run": ([vp], ctypes.c_int),
            "gridspt_batch_destroy": ([vp], None),
            "gridspt_batch_buffer": ([vp, i32, i32, i32, i32, ctypes.POINTER(vp)], ctypes.c_int),
            "gridspt_batch_tuning": ([vp, i32, i32, vp, vp, vp], ctypes.c_int),
            "gridspt_orders_linear": ([vp, gp, ctypes.POINTER(_LinPk), i32, i64, vp, vp, vp, vp, vp, i64],
                                      ctypes.c_int),
            "gridspt_tune_orders": ([vp, gp, ctypes.POINTER(_LinPk), i32, i64, vp, vp, vp, vp, vp, i64], ctypes.c_int),
            "gridspt_tuning": ([vp, gp, i32, vp, vp, vp], ctypes.c_int),
            "gridspt_set_tuning": ([vp, gp, i32], ctypes.c_int),
            "gridspt_pform_workspace_bytes": ([gp, i32], i64),
            "gridspt_orders_pform": ([vp, gp, i32, i64, i64, vp, vp, vp, vp, vp, vp, i64], ctypes.c_int),
            "gridspt_smooth": ([vp, gp, i32, vp, vp, i32, dbl, vp, vp, i64], ctypes.c_int),
            "gridspt_stats_workspace_bytes": ([i32, i32, i32], i64),
            "gridspt_field_stats": ([vp, gp, i32, vp, i32, dbl, dbl, i32, vp, vp, vp, vp, vp, i64], ctypes.c_int),
            "gridspt_noise_field": ([vp, gp, ctypes.POINTER(_LinPk), vp, vp, vp, vp, i64], ctypes.c_int),
            "gridspt_adjoint_workspace_bytes": ([gp, i32], i64),
            "gridspt_adjoint": ([vp, gp, ctypes.POINTER(_LinPk), i32, i64, vp, vp, vp, vp, vp, i64], ctypes.c_int),
            "gridspt_set_profiling": ([vp, i32], ctypes.c_int),
            "gridspt_profile_read": ([vp, i32, vp, vp, vp, vp], ctypes.c_int),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _check(rc: int, where: str) -> int:
    if rc < 0:
        raise GridSPTError(rc, where)
    return rc


# --------------------------------------------------------------------------
# host helpers
# --------------------------------------------------------------------------

def cut_n2max(n: int, box: float, kcut: float = 0.0) -> int:
    """Mask threshold: kcut <= 0 is the strict 2/3 rule, else |k| <= kcut."""
    return _check(lib().gridspt_cut_n2max(n, box, kcut), "cut_n2max")


def cube_kc(n2max: int) -> int:
    return _check(lib().gridspt_cube_kc(n2max), "cube_kc")


def linear_edges(nbins: int, kmax_num: int, kmax_den: int, n2max: int):
    import numpy as np
    e = np.zeros(nbins + 1, dtype=np.int64)
    _check(lib().gridspt_linear_edges(nbins, kmax_num, kmax_den, n2max, e.ctypes.data), "linear_edges")
    return e


def sigma8_amp(sigma8: float, ns: float, gamma: float) -> float:
    out = ctypes.c_double()
    _check(lib().gridspt_sigma8_amp(sigma8, ns, gamma, ctypes.byref(out)), "sigma8_amp")
    return out.value


def growth(om: float, ol: float, z: float) -> float:
    out = ctypes.c_double()
    _check(lib().gridspt_growth(om, ol, z, ctypes.byref(out)), "growth")
    return out.value


# --------------------------------------------------------------------------
# grid, context, workspace
# --------------------------------------------------------------------------

@dataclass(frozen=True)
class Grid:
    n: int
    box: float
    kc: int
    dtype: int = F32
    flags: int = 0  # CHECK_FINITE or 0

    @property
    def cstruct(self) -> _Grid:
        return _Grid(self.n, self.dtype, float(self.box), self.kc, self.flags)

    @property
    def real_shape(self):
        return (self.n,) * 3

    @property
    def real_dtype(self):
        return torch.float64 if self.dtype == F64 else torch.float32

    @property
    def cube_shape(self):
        return (self.kc + 1, 2 * self.kc + 1, 2 * self.kc + 1, 2)


@dataclass
class LinearSpectrum:
    amp: float
    ns: float = 0.96
    gamma: float = 0.21
    growth: float = 1.0
    n2max: int = 0
    seed: int = 1
    stream: int = 0


# --------------------------------------------------------------------------
# tensor checks: every address handed to the library belongs to a contiguous
# GPU tensor of the dtype and shape the call expects (a wrong one would make a
# kernel read or write past its allocation)
# --------------------------------------------------------------------------

def _addr(ctx: "Context", t: torch.Tensor, name: str, dtype, shape) -> int:
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s: expected a torch.Tensor, got %s" % (name, type(t).__name__))
    if t.dtype != dtype:
        raise TypeError("%s: dtype %s, expected %s" % (name, t.dtype, dtype))
    if tuple(t.shape) != tuple(shape):
        raise ValueError("%s: shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))
    if not t.is_contiguous():
        raise ValueError("%s: must be contiguous" % name)
    if t.device.type != "cuda":
        raise ValueError("%s: must be a GPU tensor (got device %s)" % (name, t.device))
    if t.device != ctx.device:
        raise ValueError("%s: on %s, but the context's stream is on %s" % (name, t.device, ctx.device))
    ctx._uses(t)
    return t.data_ptr()


def _real(ctx, grid, t, name):
    return ctypes.c_void_p(_addr(ctx, t, name, grid.real_dtype, grid.real_shape))


def _cube(ctx, grid, t, name):
    return ctypes.c_void_p(_addr(ctx, t, name, grid.real_dtype, grid.cube_shape))


def _f64(ctx, t, name, shape):
    if t is None:
        return None
    return ctypes.c_void_p(_addr(ctx, t, name, torch.float64, shape))


def _real_array(ctx, grid, ts, name, allow_none=False):
    arr = (ctypes.c_void_p * len(ts))()
    for i, t in enumerate(ts):
        if t is None:
            if not allow_none:
                raise ValueError("%s[%d]: missing" % (name, i))
            arr[i] = None
        else:
            arr[i] = _addr(ctx, t, "%s[%d]" % (name, i), grid.real_dtype, grid.real_shape)
    return arr


def _cube_array(ctx, grid, ts, name, allow_none=False):
    arr = (ctypes.c_void_p * len(ts))()
    for i, t in enumerate(ts):
        if t is None:
            if not allow_none:
                raise ValueError("%s[%d]: missing" % (name, i))
            arr[i] = None
        else:
            arr[i] = _addr(ctx, t, "%s[%d]" % (name, i), grid.real_dtype, grid.cube_shape)
    return arr


class Context:
    """A libgridspt context bound to a torch stream (default: current stream).

    Outputs and the workspace the binding allocates come from the context's
    stream; tensors the caller passes are marked as used on it when it is
    not the current stream, so that freeing them waits for its work."""

    def __init__(self, stream: Optional[torch.cuda.Stream] = None):
        s = stream if stream is not None else torch.cuda.current_stream()
        self.stream = s
        self.device = s.device if s.device.index is not None else torch.device("cuda", torch.cuda.current_device())
        h = ctypes.c_void_p()
        _check(lib().gridspt_create(ctypes.byref(h), ctypes.c_void_p(s.cuda_stream)), "create")
        self._h = h
        self._ws = None

    def _uses(self, t: torch.Tensor) -> None:
        if self.stream != torch.cuda.current_stream(self.device):
            t.record_stream(self.stream)

    def empty(self, shape, dtype) -> torch.Tensor:
        """A new tensor allocated on the context's stream."""
        with torch.cuda.stream(self.stream):
            return torch.empty(shape, dtype=dtype, device=self.device)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.gridspt_destroy(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def sync(self):
        _check(lib().gridspt_sync(self._h), "sync")

    def workspace(self, nbytes: int) -> torch.Tensor:
        """A device scratch buffer of at least nbytes, reused across calls
        (allocated on the context's stream, so a regrown buffer's memory is
        reused only after the stream's earlier work)."""
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = None
            self._ws = self.empty(max(int(nbytes), 256), torch.uint8)
        return self._ws

    def _work(self, nbytes: int):
        ws = self.workspace(nbytes)
        return ctypes.c_void_p(ws.data_ptr()), ws.numel()

    # ---- profiling ----
    def set_profiling(self, enable: bool):
        _check(lib().gridspt_set_profiling(self._h, 1 if enable else 0), "set_profiling")

    def profile_read(self):
        import numpy as np
        m = 32
        names = ctypes.create_string_buffer(32 * m)
        launches = np.zeros(m, dtype=np.int64)
        ms = np.zeros(m)
        by = np.zeros(m)
        k = _check(lib().gridspt_profile_read(self._h, m, names, launches.ctypes.data, ms.ctypes.data,
                                              by.ctypes.data), "profile_read")
        out = {}
        for i in range(k):
            nm = names.raw[32 * i: 32 * (i + 1)].split(b"\0", 1)[0].decode()
            out[nm] = {"launches": int(launches[i]), "ms": float(ms[i]), "bytes": float(by[i])}
        return out

    def profile_orders(self):
        """{order: {"ms", "bytes"}} of the last profile_read (order 0: launches of no order)."""
        import numpy as np
        m = 9
        ms = np.zeros(m)
        by = np.zeros(m)
        top = _check(lib().gridspt_profile_orders(self._h, m, ms.ctypes.data, by.ctypes.data), "profile_orders")
        return {i: {"ms": float(ms[i]), "bytes": float(by[i])} for i in range(min(top, m - 1) + 1)}


def workspace_bytes(grid: Grid, nmax: int, flags: int = 0) -> int:
    g = grid.cstruct
    return _check(lib().gridspt_workspace_bytes(ctypes.byref(g), nmax, flags), "workspace_bytes")


def _new_real(ctx: Optional[Context], grid: Grid) -> torch.Tensor:
    if ctx is not None:
        return ctx.empty(grid.real_shape, grid.real_dtype)
    return torch.empty(grid.real_shape, dtype=grid.real_dtype, device="cuda")


def _new_cube(ctx: Optional[Context], grid: Grid) -> torch.Tensor:
    if ctx is not None:
        return ctx.empty(grid.cube_shape, grid.real_dtype)
    return torch.empty(grid.cube_shape, dtype=grid.real_dtype, device="cuda")


# --------------------------------------------------------------------------
# hot path
# --------------------------------------------------------------------------

def linear_field(ctx: Context, grid: Grid, lp: LinearSpectrum, out: Optional[torch.Tensor] = None,
                 out_k: Optional[torch.Tensor] = None, spectrum: bool = False):
    """Seeded Gaussian delta_1 (step 1 of Sec. II C).  Returns delta1 or (delta1, delta1_k)."""
    out = out if out is not None else _new_real(ctx, grid)
    if spectrum and out_k is None:
        out_k = _new_cube(ctx, grid)
    g = grid.cstruct
    c = _linpk(lp)
    ws, nws = ctx._work(workspace_bytes(grid, 1))
    _check(lib().gridspt_linear_field(ctx.handle, ctypes.byref(g), ctypes.byref(c), _real(ctx, grid, out, "out"),
                                      _cube(ctx, grid, out_k, "out_k") if out_k is not None else None, ws, nws),
           "linear_field")
    return (out, out_k) if (spectrum or out_k is not None) else out


def _linpk(lp: LinearSpectrum) -> _LinPk:
    return _LinPk(lp.amp, lp.ns, lp.gamma, lp.growth, lp.n2max, lp.seed, lp.stream)


def noise_field(ctx: Context, grid: Grid, lp: LinearSpectrum, noise: torch.Tensor,
                out: Optional[torch.Tensor] = None, out_k: Optional[torch.Tensor] = None):
    """delta_1 from a given white-noise field (step 1 of Sec. II C without the draw)."""
    out = out if out is not None else _new_real(ctx, grid)
    g = grid.cstruct
    c = _linpk(lp)
    ws, nws = ctx._work(workspace_bytes(grid, 1))
    _check(lib().gridspt_noise_field(ctx.handle, ctypes.byref(g), ctypes.byref(c), _real(ctx, grid, noise, "noise"),
                                     _real(ctx, grid, out, "out"),
                                     _cube(ctx, grid, out_k, "out_k") if out_k is not None else None, ws, nws),
           "noise_field")
    return out


def adjoint(ctx: Context, grid: Grid, lp: LinearSpectrum, nmax: int, n2max2: int, delta_k, theta_k, gdelta,
            out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """dJ/dw for a scalar J of delta_1..delta_nmax, given gdelta[n-1] = dJ/d delta_n
    and the forward run's spectra delta_k, theta_k (orders < nmax)."""
    if len(gdelta) != nmax:
        raise ValueError("adjoint: %d gradients for nmax = %d" % (len(gdelta), nmax))
    out = out if out is not None else _new_real(ctx, grid)
    g = grid.cstruct
    c = _linpk(lp)
    need = _check(lib().gridspt_adjoint_workspace_bytes(ctypes.byref(g), nmax), "adjoint_workspace_bytes")
    ws, nws = ctx._work(need)
    nk = max(nmax - 1, 1)
    dk = _cube_array(ctx, grid, list(delta_k[:nk]), "delta_k") if nmax > 1 else None
    tk = _cube_array(ctx, grid, [None] + list(theta_k[1:nk]), "theta_k", allow_none=True) if nmax > 2 else None
    gd = _real_array(ctx, grid, list(gdelta), "gdelta")
    _check(lib().gridspt_adjoint(ctx.handle, ctypes.byref(g), ctypes.byref(c), nmax, n2max2, dk, tk, gd,
                                 _real(ctx, grid, out, "out"), ws, nws), "adjoint")
    return out


class NoiseToOrders(torch.autograd.Function):
    """w -> (delta_1, ..., delta_nmax): the linear field from the noise w and
    the recursion, differentiable in w.  The forward keeps only the spectra
    of orders < nmax (per-order checkpoints); the backward regenerates the
    real fields from them and runs the hand-written reverse mode."""

    @staticmethod
    def forward(fctx, w, gctx, grid, lp, nmax, n2max2):
        d1 = noise_field(gctx, grid, lp, w.contiguous())
        out = orders(gctx, grid, nmax, lp.n2max, n2max2, d1, spectra=nmax > 1)
        keep = []
        if nmax > 1:
            keep = list(out.delta_k[:nmax - 1]) + list(out.theta_k[1:nmax - 1])
        fctx.save_for_backward(*keep)
        fctx.meta = (gctx, grid, lp, nmax, n2max2)
        return tuple(out.delta)

    @staticmethod
    def backward(fctx, *grads):
        gctx, grid, lp, nmax, n2max2 = fctx.meta
        saved = fctx.saved_tensors
        dk = list(saved[:nmax - 1]) if nmax > 1 else []
        tk = ([dk[0]] + list(saved[nmax - 1:])) if nmax > 2 else dk
        gdelta = [(g.contiguous() if g is not None else gctx.empty(grid.real_shape, grid.real_dtype).zero_())
                  for g in grads]
        gw = adjoint(gctx, grid, lp, nmax, n2max2, dk, tk, gdelta)
        return gw, None, None, None, None, None


def orders_from_noise(w: torch.Tensor, ctx: Context, grid: Grid, lp: LinearSpectrum, nmax: int, n2max2: int):
    """Differentiable (delta_1, ..., delta_nmax) of the white-noise field w."""
    return NoiseToOrders.apply(w, ctx, grid, lp, nmax, n2max2)


def forward(ctx: Context, grid: Grid, n2max: int, field: torch.Tensor, out_k: Optional[torch.Tensor] = None):
    """Masked forward transform of a real field into the cube layout."""
    out_k = out_k if out_k is not None else _new_cube(ctx, grid)
    g = grid.cstruct
    ws, nws = ctx._work(workspace_bytes(grid, 1))
    _check(lib().gridspt_forward(ctx.handle, ctypes.byref(g), n2max, _real(ctx, grid, field, "field"),
                                 _cube(ctx, grid, out_k, "out_k"), ws, nws), "forward")
    return out_k


def spectrum_half(ctx: Context, grid: Grid, cube: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """A cube spectrum in the half layout [ix, iy, iz, 2] (N x N x (N/2 + 1) complex,
    zero outside the cube), the layout of numpy's rfftn of an [x, y, z] field."""
    shape = (grid.n, grid.n, grid.n // 2 + 1, 2)
    out = out if out is not None else ctx.empty(shape, grid.real_dtype)
    g = grid.cstruct
    _check(lib().gridspt_spectrum_half(ctx.handle, ctypes.byref(g), _cube(ctx, grid, cube, "cube"),
                                       ctypes.c_void_p(_addr(ctx, out, "out", grid.real_dtype, shape))),
           "spectrum_half")
    return out


class Orders:
    """Outputs of gridspt_orders: lists delta, theta (real) and delta_k, theta_k (cube or None)."""

    def __init__(self, delta, theta, delta_k, theta_k):
        self.delta, self.theta, self.delta_k, self.theta_k = delta, theta, delta_k, theta_k


def alloc_orders(grid: Grid, nmax: int, spectra: bool = True, ctx: Optional[Context] = None) -> Orders:
    delta = [_new_real(ctx, grid) for _ in range(nmax)]
    theta = [delta[0]] + [_new_real(ctx, grid) for _ in range(nmax - 1)]
    dk = [_new_cube(ctx, grid) for _ in range(nmax)] if spectra else None
    tk = ([dk[0]] + [_new_cube(ctx, grid) for _ in range(nmax - 1)]) if spectra else None
    return Orders(delta, theta, dk, tk)


def _order_args(ctx: Context, grid: Grid, nmax: int, out: Orders):
    """Checked address arrays of an Orders output set (theta[0] and spectra entries may be None)."""
    if len(out.delta) != nmax or len(out.theta) != nmax:
        raise ValueError("orders: %d / %d output fields for nmax = %d" % (len(out.delta), len(out.theta), nmax))
    d = _real_array(ctx, grid, out.delta, "delta")
    if any(x is None for x in out.theta[1:]):
        raise ValueError("orders: theta[1:] must all be given")
    t = _real_array(ctx, grid, out.theta, "theta", allow_none=True)  # theta[0] (= delta_1) may be None
    dk = tk = None
    if out.delta_k is not None:
        if len(out.delta_k) != nmax:
            raise ValueError("orders: %d delta_k entries for nmax = %d" % (len(out.delta_k), nmax))
        dk = _cube_array(ctx, grid, out.delta_k, "delta_k", allow_none=True)
    if out.theta_k is not None:
        if len(out.theta_k) != nmax:
            raise ValueError("orders: %d theta_k entries for nmax = %d" % (len(out.theta_k), nmax))
        tk = _cube_array(ctx, grid, out.theta_k, "theta_k", allow_none=True)
    return d, t, dk, tk


def orders(ctx: Context, grid: Grid, nmax: int, n2max1: int, n2max2: int, delta1: torch.Tensor,
           out: Optional[Orders] = None, spectra: bool = True) -> Orders:
    """Recursion of Eq. 10/11 up to nmax (delta_1 input is masked with W1 here)."""
    out = out if out is not None else alloc_orders(grid, nmax, spectra, ctx)
    g = grid.cstruct
    ws, nws = ctx._work(workspace_bytes(grid, nmax))
    d, t, dk, tk = _order_args(ctx, grid, nmax, out)
    _check(lib().gridspt_orders(ctx.handle, ctypes.byref(g), nmax, n2max1, n2max2,
                                _real(ctx, grid, delta1, "delta1"), d, t, dk, tk, ws, nws), "orders")
    return out


def orders_linear(ctx: Context, grid: Grid, lp: LinearSpectrum, nmax: int, n2max2: int,
                  out: Optional[Orders] = None, spectra: bool = True) -> Orders:
    """Seeded linear field and orders 1..nmax in one pass sequence (delta[0] = delta_1)."""
    out = out if out is not None else alloc_orders(grid, nmax, spectra, ctx)
    g = grid.cstruct
    c = _linpk(lp)
    ws, nws = ctx._work(workspace_bytes(grid, nmax))
    d, t, dk, tk = _order_args(ctx, grid, nmax, out)
    _check(lib().gridspt_orders_linear(ctx.handle, ctypes.byref(g), ctypes.byref(c), nmax, n2max2, d, t, dk, tk,
                                       ws, nws), "orders_linear")
    return out


def set_tuning(ctx: Context, grid: Grid, variant: int) -> None:
    """Pin launch variant `variant` for every pass of this grid's size and precision."""
    g = grid.cstruct
    _check(lib().gridspt_set_tuning(ctx.handle, ctypes.byref(g), int(variant)), "set_tuning")


def tune_orders(ctx: Context, grid: Grid, lp: LinearSpectrum, nmax: int, n2max2: int,
                out: Optional[Orders] = None):
    """Autotune the pass variants of this grid for the context; returns {kind: (variant, ms)}."""
    import numpy as np
    out = out if out is not None else alloc_orders(grid, nmax, True, ctx)
    g = grid.cstruct
    c = _linpk(lp)
    ws, nws = ctx._work(workspace_bytes(grid, nmax))
    d, t, dk, tk = _order_args(ctx, grid, nmax, out)
    _check(lib().gridspt_tune_orders(ctx.handle, ctypes.byref(g), ctypes.byref(c), nmax, n2max2, d, t, dk, tk,
                                     ws, nws), "tune_orders")
    m = 16
    names = ctypes.create_string_buffer(32 * m)
    var = np.zeros(m, dtype=np.int32)
    ms = np.zeros(m)
    k = _check(lib().gridspt_tuning(ctx.handle, ctypes.byref(g), m, names, var.ctypes.data, ms.ctypes.data),
               "tuning")
    return {names.raw[32 * i: 32 * (i + 1)].split(b"\0", 1)[0].decode(): (int(var[i]), float(ms[i]))
            for i in range(k)}


def orders_pform(ctx: Context, grid: Grid, nmax: int, n2max1: int, n2max2: int, delta1: torch.Tensor,
                 out: Optional[Orders] = None, spectra: bool = True) -> Orders:
    """The recursion with the printed (P-form) sources of Eq. 10; outputs as orders()."""
    out = out if out is not None else alloc_orders(grid, nmax, spectra, ctx)
    g = grid.cstruct
    need = _check(lib().gridspt_pform_workspace_bytes(ctypes.byref(g), nmax), "pform_workspace_bytes")
    ws, nws = ctx._work(need)
    d, t, dk, tk = _order_args(ctx, grid, nmax, out)
    _check(lib().gridspt_orders_pform(ctx.handle, ctypes.byref(g), nmax, n2max1, n2max2,
                                      _real(ctx, grid, delta1, "delta1"), d, t, dk, tk, ws, nws), "orders_pform")
    return out


def smooth(ctx: Context, grid: Grid, fields_k: Sequence[torch.Tensor], coef: Sequence[float], radius: float,
           cumulative: bool = True, out: Optional[Sequence[torch.Tensor]] = None):
    """Gaussian-smoothed real fields of cube spectra: cumulative sums sum_{i<=j} coef_i F_i
    (the truncated series) or each coef_j F_j; at most five."""
    import numpy as np
    out = list(out) if out is not None else [_new_real(ctx, grid) for _ in fields_k]
    if len(out) != len(fields_k) or len(coef) < len(fields_k):
        raise ValueError("smooth: %d spectra, %d outputs, %d coefficients" % (len(fields_k), len(out), len(coef)))
    c = np.ascontiguousarray(np.asarray(coef, dtype=np.float64))
    g = grid.cstruct
    ws, nws = ctx._work(workspace_bytes(grid, 1))
    _check(lib().gridspt_smooth(ctx.handle, ctypes.byref(g), len(fields_k), _cube_array(ctx, grid, fields_k, "fields_k"),
                                c.ctypes.data, 1 if cumulative else 0, float(radius),
                                _real_array(ctx, grid, out, "out"), ws, nws), "smooth")
    return out


def field_stats(ctx: Context, grid: Grid, fields: Sequence[torch.Tensor], nbins: int = 0, lo: float = -1.0,
                hi: float = 1.0, nbins2: int = 0):
    """(moments [nf, 4], corr [nf, nf], counts [nf, nbins] or None, joint [nf-1, nbins2, nbins2] or None)."""
    nf = len(fields)
    f64 = torch.float64
    mom = ctx.empty((nf, 4), f64)
    cor = ctx.empty((nf, nf), f64)
    cnt = ctx.empty((nf, nbins), f64) if nbins > 0 else None
    jnt = ctx.empty((nf - 1, nbins2, nbins2), f64) if (nbins2 > 0 and nf > 1) else None
    g = grid.cstruct
    need = _check(lib().gridspt_stats_workspace_bytes(nf, nbins, nbins2 if jnt is not None else 0),
                  "stats_workspace_bytes")
    ws, nws = ctx._work(need)
    _check(lib().gridspt_field_stats(ctx.handle, ctypes.byref(g), nf, _real_array(ctx, grid, fields, "fields"),
                                     nbins, float(lo), float(hi), nbins2, _f64(ctx, mom, "moments", mom.shape),
                                     _f64(ctx, cor, "corr", cor.shape),
                                     _f64(ctx, cnt, "counts", cnt.shape) if cnt is not None else None,
                                     _f64(ctx, jnt, "joint", jnt.shape) if jnt is not None else None, ws, nws),
           "field_stats")
    return mom, cor, cnt, jnt


def sum_orders(ctx: Context, grid: Grid, delta: Sequence[torch.Tensor], coef: Sequence[float],
               out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """FP64 sum_n coef[n] delta_n(x) (the truncated series of Eq. 8)."""
    import numpy as np
    if len(coef) < len(delta):
        raise ValueError("sum_orders: %d fields, %d coefficients" % (len(delta), len(coef)))
    out = out if out is not None else ctx.empty(grid.real_shape, torch.float64)
    c = np.ascontiguousarray(np.asarray(coef, dtype=np.float64))
    g = grid.cstruct
    _check(lib().gridspt_sum_orders(ctx.handle, ctypes.byref(g), len(delta), _real_array(ctx, grid, delta, "delta"),
                                    c.ctypes.data, _f64(ctx, out, "out", grid.real_shape)), "sum_orders")
    return out


def power(ctx: Context, grid: Grid, fields_k: Sequence[torch.Tensor], pairs, edges):
    """Shell-averaged cross spectra; returns (pk [npairs, nbins], kmean, nmodes) as float64 tensors."""
    import numpy as np
    pr = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1))
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int64))
    npairs, nb = pr.size // 2, e.size - 1
    pk = ctx.empty((npairs, nb), torch.float64)
    km = ctx.empty(nb, torch.float64)
    nm = ctx.empty(nb, torch.float64)
    g = grid.cstruct
    need = _check(lib().gridspt_power_workspace_bytes(ctypes.byref(g), npairs, nb), "power_workspace_bytes")
    ws, nws = ctx._work(need)
    _check(lib().gridspt_power(ctx.handle, ctypes.byref(g), len(fields_k), _cube_array(ctx, grid, fields_k, "fields_k"),
                               npairs, pr.ctypes.data, nb, e.ctypes.data, _f64(ctx, pk, "pk", pk.shape),
                               _f64(ctx, km, "kmean", km.shape), _f64(ctx, nm, "nmodes", nm.shape), ws, nws), "power")
    return pk, km, nm


def power_static(ctx: Context, grid: Grid, fields_k: Sequence[torch.Tensor], pairs, edges, out=None):
    """power() through gridspt_power_static: no workspace, the library's own
    scratch array.  out: optional (pk, kmean, nmodes) float64 tensors to fill
    (so that the call itself allocates nothing)."""
    import numpy as np
    pr = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1))
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int64))
    npairs, nb = pr.size // 2, e.size - 1
    if out is None:
        out = (ctx.empty((npairs, nb), torch.float64), ctx.empty(nb, torch.float64), ctx.empty(nb, torch.float64))
    pk, km, nm = out
    g = grid.cstruct
    _check(lib().gridspt_power_static(ctx.handle, ctypes.byref(g), len(fields_k),
                                      _cube_array(ctx, grid, fields_k, "fields_k"), npairs, pr.ctypes.data, nb,
                                      e.ctypes.data, _f64(ctx, pk, "pk", (npairs, nb)), _f64(ctx, km, "kmean", (nb,)),
                                      _f64(ctx, nm, "nmodes", (nb,))), "power_static")
    return pk, km, nm


def bispectrum(ctx: Context, grid: Grid, fields_k: Sequence[torch.Tensor], tris, terms, edges):
    """FFT-estimator bispectra; returns (bk [nterms], ntriangles [ntri]) as float64 tensors."""
    import numpy as np
    tb = np.ascontiguousarray(np.asarray(tris, dtype=np.int32).reshape(-1))
    tt = np.ascontiguousarray(np.asarray(terms, dtype=np.int32).reshape(-1))
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int64))
    ntri, nterms, nb = tb.size // 3, tt.size // 4, e.size - 1
    bk = ctx.empty(nterms, torch.float64)
    nt = ctx.empty(ntri, torch.float64)
    g = grid.cstruct
    need = _check(lib().gridspt_bispectrum_workspace_bytes(ctypes.byref(g), ntri, tb.ctypes.data, nterms,
                                                           tt.ctypes.data), "bispectrum_workspace_bytes")
    ws, nws = ctx._work(need)
    _check(lib().gridspt_bispectrum(ctx.handle, ctypes.byref(g), len(fields_k),
                                    _cube_array(ctx, grid, fields_k, "fields_k"), ntri, tb.ctypes.data, nterms,
                                    tt.ctypes.data, nb, e.ctypes.data, _f64(ctx, bk, "bk", bk.shape),
                                    _f64(ctx, nt, "ntriangles", nt.shape), ws, nws), "bispectrum")
    return bk, nt


# --------------------------------------------------------------------------
# batches of realisations (one captured graph)
# --------------------------------------------------------------------------

@dataclass
class BatchGroup:
    """nreal realisations of one grid: linear field (Philox stream lin.stream + r),
    orders 1..nmax, spectra of the delta_n pairs and optional bispectrum terms."""
    grid: Grid
    nreal: int
    nmax: int
    n2max2: int
    lin: LinearSpectrum
    pairs: Sequence
    edges: Sequence
    tris: Optional[Sequence] = None
    terms: Optional[Sequence] = None


class Batch:
    """gridspt_batch_*: every group's passes launched once over all its
    realisations, the groups as parallel branches of one HIP graph, ending in
    realisation means and standard deviations of P and B."""

    def __init__(self, ctx: Context, groups: Sequence[BatchGroup], tune: bool = False, eager: bool = False):
        import numpy as np
        self.ctx = ctx
        self.groups = list(groups)
        ng = len(self.groups)
        self._keep = []
        cg = (_BatchGroup * ng)()
        self.out = []
        co = (_BatchOut * ng)()
        for i, bg in enumerate(self.groups):
            pr = np.ascontiguousarray(np.asarray(bg.pairs, dtype=np.int32).reshape(-1))
            e = np.ascontiguousarray(np.asarray(bg.edges, dtype=np.int64))
            tb = np.ascontiguousarray(np.asarray(bg.tris if bg.tris is not None else [], dtype=np.int32).reshape(-1))
            tt = np.ascontiguousarray(np.asarray(bg.terms if bg.terms is not None else [], dtype=np.int32).reshape(-1))
            self._keep += [pr, e, tb, tt]
            lp = bg.lin
            cg[i] = _BatchGroup(bg.grid.cstruct, bg.nreal, bg.nmax, bg.n2max2,
                                _LinPk(lp.amp, lp.ns, lp.gamma, lp.growth, lp.n2max, lp.seed, lp.stream),
                                pr.size // 2, pr.ctypes.data, e.size - 1, e.ctypes.data, tb.size // 3,
                                tb.ctypes.data if tb.size else None, tt.size // 4, tt.ctypes.data if tt.size else None)
            npairs, nb, ntri, nterms = pr.size // 2, e.size - 1, tb.size // 3, tt.size // 4
            dev = dict(device=ctx.device, dtype=torch.float64)
            with torch.cuda.stream(ctx.stream):  # the outputs belong to the context's stream
                o = {"pk_mean": torch.zeros((npairs, nb), **dev), "pk_std": torch.zeros((npairs, nb), **dev),
                     "kmean": torch.zeros(nb, **dev), "nmodes": torch.zeros(nb, **dev)}
                if ntri:
                    o.update(bk_mean=torch.zeros(nterms, **dev), bk_std=torch.zeros(nterms, **dev),
                             ntriangles=torch.zeros(ntri, **dev))
            self.out.append(o)
            co[i] = _BatchOut(*[o[k].data_ptr() if k in o else None for k, _ in _BatchOut._fields_])
        self._cg, self._co = cg, co
        need = _check(lib().gridspt_batch_workspace_bytes(ng, cg), "batch_workspace_bytes")
        self.work = ctx.empty(max(int(need), 256), torch.uint8)
        flags = (BATCH_TUNE if tune else 0) | (BATCH_EAGER if eager else 0)
        h = ctypes.c_void_p()
        _check(lib().gridspt_batch_create(ctx.handle, ng, cg, co, ctypes.c_void_p(self.work.data_ptr()),
                                          self.work.numel(), flags, ctypes.byref(h)), "batch_create")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.gridspt_batch_destroy(h)
            self._h = None

    def run(self):
        _check(lib().gridspt_batch_run(self._h), "batch_run")

    def buffer(self, group: int, real: int, what: int, index: int = 0) -> torch.Tensor:
        """A view of one realisation's buffer inside the batch workspace."""
        import numpy as np
        p = ctypes.c_void_p()
        _check(lib().gridspt_batch_buffer(self._h, group, real, what, index, ctypes.byref(p)), "batch_buffer")
        bg = self.groups[group]
        g = bg.grid
        off = p.value - self.work.data_ptr()
        if what in (BATCH_DELTA, BATCH_THETA):
            shape, dt = (g.n,) * 3, g.real_dtype
        elif what == BATCH_DELTA_K:
            shape, dt = g.cube_shape, g.real_dtype
        elif what == BATCH_PK:
            shape, dt = (int(np.asarray(bg.pairs).size // 2), len(bg.edges) - 1), torch.float64
        else:
            shape, dt = (int(np.asarray(bg.terms).size // 4),), torch.float64
        nbytes = int(torch.tensor([], dtype=dt).element_size())
        for d in shape:
            nbytes *= d
        return self.work[off: off + nbytes].view(dt).view(shape)

    def tuning(self, group: int):
        """{kind: (variant, ms)} chosen by the autotuner for a group."""
        import numpy as np
        m = 32
        names = ctypes.create_string_buffer(32 * m)
        var = np.zeros(m, dtype=np.int32)
        ms = np.zeros(m)
        k = _check(lib().gridspt_batch_tuning(self._h, group, m, names, var.ctypes.data, ms.ctypes.data),
                   "batch_tuning")
        out = {}
        for i in range(k):
            nm = names.raw[32 * i: 32 * (i + 1)].split(b"\0", 1)[0].decode()
            out[nm] = (int(var[i]), float(ms[i]))
        return out
