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
_STATUS = {0: "ok", -1: "invalid argument", -2: "unsupported configuration", -3: "workspace too small",
           -4: "null or misaligned device pointer", -5: "HIP runtime error"}


class GridSPTError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__("%s: %s (status %d)" % (where, _STATUS.get(status, "unknown"), status))
        self.status = status


class _Grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("dtype", ctypes.c_int32), ("box", ctypes.c_double),
                ("kc", ctypes.c_int32), ("reserved", ctypes.c_int32)]


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
            "gridspt_workspace_bytes": ([gp, i32], i64),
            "gridspt_linear_field": ([vp, gp, ctypes.POINTER(_LinPk), vp, vp, vp, i64], ctypes.c_int),
            "gridspt_forward": ([vp, gp, i64, vp, vp, vp, i64], ctypes.c_int),
            "gridspt_orders": ([vp, gp, i32, i64, i64, vp, vp, vp, vp, vp, vp, i64], ctypes.c_int),
            "gridspt_sum_orders": ([vp, gp, i32, vp, vp, vp], ctypes.c_int),
            "gridspt_power_workspace_bytes": ([gp, i32, i32], i64),
            "gridspt_power": ([vp, gp, i32, vp, i32, vp, i32, vp, vp, vp, vp, vp, i64], ctypes.c_int),
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

    @property
    def cstruct(self) -> _Grid:
        return _Grid(self.n, self.dtype, float(self.box), self.kc, 0)

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


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _ptr_array(ts: Sequence[Optional[torch.Tensor]]):
    arr = (ctypes.c_void_p * len(ts))()
    for i, t in enumerate(ts):
        arr[i] = t.data_ptr() if t is not None else None
    return arr


class Context:
    """A libgridspt context bound to a torch stream (default: current stream)."""

    def __init__(self, stream: Optional[torch.cuda.Stream] = None):
        s = stream if stream is not None else torch.cuda.current_stream()
        self.stream = s
        h = ctypes.c_void_p()
        _check(lib().gridspt_create(ctypes.byref(h), ctypes.c_void_p(s.cuda_stream)), "create")
        self._h = h
        self._ws = None

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
        """A device scratch buffer of at least nbytes, reused across calls."""
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = None
            self._ws = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device="cuda")
        return self._ws

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


def workspace_bytes(grid: Grid, nmax: int) -> int:
    g = grid.cstruct
    return _check(lib().gridspt_workspace_bytes(ctypes.byref(g), nmax), "workspace_bytes")


def _new_real(grid: Grid) -> torch.Tensor:
    return torch.empty((grid.n,) * 3, dtype=grid.real_dtype, device="cuda")


def _new_cube(grid: Grid) -> torch.Tensor:
    return torch.empty(grid.cube_shape, dtype=grid.real_dtype, device="cuda")


# --------------------------------------------------------------------------
# hot path
# --------------------------------------------------------------------------

def linear_field(ctx: Context, grid: Grid, lp: LinearSpectrum, out: Optional[torch.Tensor] = None,
                 out_k: Optional[torch.Tensor] = None, spectrum: bool = False):
    """Seeded Gaussian delta_1 (step 1 of Sec. II C).  Returns delta1 or (delta1, delta1_k)."""
    out = out if out is not None else _new_real(grid)
    if spectrum and out_k is None:
        out_k = _new_cube(grid)
    g = grid.cstruct
    c = _LinPk(lp.amp, lp.ns, lp.gamma, lp.growth, lp.n2max, lp.seed, lp.stream)
    nb = workspace_bytes(grid, 1)
    ws = ctx.workspace(nb)
    _check(lib().gridspt_linear_field(ctx.handle, ctypes.byref(g), ctypes.byref(c), _ptr(out), _ptr(out_k),
                                      _ptr(ws), ws.numel()), "linear_field")
    return (out, out_k) if (spectrum or out_k is not None) else out


def _linpk(lp: LinearSpectrum) -> _LinPk:
    return _LinPk(lp.amp, lp.ns, lp.gamma, lp.growth, lp.n2max, lp.seed, lp.stream)


def noise_field(ctx: Context, grid: Grid, lp: LinearSpectrum, noise: torch.Tensor,
                out: Optional[torch.Tensor] = None, out_k: Optional[torch.Tensor] = None):
    """delta_1 from a given white-noise field (step 1 of Sec. II C without the draw)."""
    out = out if out is not None else _new_real(grid)
    g = grid.cstruct
    c = _linpk(lp)
    ws = ctx.workspace(workspace_bytes(grid, 1))
    _check(lib().gridspt_noise_field(ctx.handle, ctypes.byref(g), ctypes.byref(c), _ptr(noise), _ptr(out),
                                     _ptr(out_k), _ptr(ws), ws.numel()), "noise_field")
    return out


def adjoint(ctx: Context, grid: Grid, lp: LinearSpectrum, nmax: int, n2max2: int, delta_k, theta_k, gdelta,
            out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """dJ/dw for a scalar J of delta_1..delta_nmax, given gdelta[n-1] = dJ/d delta_n
    and the forward run's spectra delta_k, theta_k (orders < nmax)."""
    out = out if out is not None else _new_real(grid)
    g = grid.cstruct
    c = _linpk(lp)
    need = _check(lib().gridspt_adjoint_workspace_bytes(ctypes.byref(g), nmax), "adjoint_workspace_bytes")
    ws = ctx.workspace(need)
    nk = max(nmax - 1, 1)
    dk = _ptr_array(list(delta_k[:nk])) if nmax > 1 else None
    tk = _ptr_array([None] + list(theta_k[1:nk])) if nmax > 2 else None
    gd = _ptr_array(list(gdelta))
    _check(lib().gridspt_adjoint(ctx.handle, ctypes.byref(g), ctypes.byref(c), nmax, n2max2, dk, tk, gd, _ptr(out),
                                 _ptr(ws), ws.numel()), "adjoint")
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
        gdelta = [(g.contiguous() if g is not None else torch.zeros((grid.n,) * 3, dtype=grid.real_dtype,
                                                                    device="cuda")) for g in grads]
        gw = adjoint(gctx, grid, lp, nmax, n2max2, dk, tk, gdelta)
        return gw, None, None, None, None, None


def orders_from_noise(w: torch.Tensor, ctx: Context, grid: Grid, lp: LinearSpectrum, nmax: int, n2max2: int):
    """Differentiable (delta_1, ..., delta_nmax) of the white-noise field w."""
    return NoiseToOrders.apply(w, ctx, grid, lp, nmax, n2max2)


def forward(ctx: Context, grid: Grid, n2max: int, field: torch.Tensor, out_k: Optional[torch.Tensor] = None):
    """Masked forward transform of a real field into the cube layout."""
    out_k = out_k if out_k is not None else _new_cube(grid)
    g = grid.cstruct
    ws = ctx.workspace(workspace_bytes(grid, 1))
    _check(lib().gridspt_forward(ctx.handle, ctypes.byref(g), n2max, _ptr(field), _ptr(out_k), _ptr(ws),
                                 ws.numel()), "forward")
    return out_k


class Orders:
    """Outputs of gridspt_orders: lists delta, theta (real) and delta_k, theta_k (cube or None)."""

    def __init__(self, delta, theta, delta_k, theta_k):
        self.delta, self.theta, self.delta_k, self.theta_k = delta, theta, delta_k, theta_k


def alloc_orders(grid: Grid, nmax: int, spectra: bool = True) -> Orders:
    delta = [_new_real(grid) for _ in range(nmax)]
    theta = [delta[0]] + [_new_real(grid) for _ in range(nmax - 1)]
    dk = [_new_cube(grid) for _ in range(nmax)] if spectra else None
    tk = ([dk[0]] + [_new_cube(grid) for _ in range(nmax - 1)]) if spectra else None
    return Orders(delta, theta, dk, tk)


def orders(ctx: Context, grid: Grid, nmax: int, n2max1: int, n2max2: int, delta1: torch.Tensor,
           out: Optional[Orders] = None, spectra: bool = True) -> Orders:
    """Recursion of Eq. 10/11 up to nmax (delta_1 input is masked with W1 here)."""
    out = out if out is not None else alloc_orders(grid, nmax, spectra)
    g = grid.cstruct
    ws = ctx.workspace(workspace_bytes(grid, nmax))
    d = _ptr_array(out.delta)
    t = _ptr_array(out.theta)
    dk = _ptr_array(out.delta_k) if out.delta_k is not None else None
    tk = _ptr_array(out.theta_k) if out.theta_k is not None else None
    _check(lib().gridspt_orders(ctx.handle, ctypes.byref(g), nmax, n2max1, n2max2, _ptr(delta1), d, t, dk, tk,
                                _ptr(ws), ws.numel()), "orders")
    return out


def orders_linear(ctx: Context, grid: Grid, lp: LinearSpectrum, nmax: int, n2max2: int,
                  out: Optional[Orders] = None, spectra: bool = True) -> Orders:
    """Seeded linear field and orders 1..nmax in one pass sequence (delta[0] = delta_1)."""
    out = out if out is not None else alloc_orders(grid, nmax, spectra)
    g = grid.cstruct
    c = _linpk(lp)
    ws = ctx.workspace(workspace_bytes(grid, nmax))
    d = _ptr_array(out.delta)
    t = _ptr_array(out.theta)
    dk = _ptr_array(out.delta_k) if out.delta_k is not None else None
    tk = _ptr_array(out.theta_k) if out.theta_k is not None else None
    _check(lib().gridspt_orders_linear(ctx.handle, ctypes.byref(g), ctypes.byref(c), nmax, n2max2, d, t, dk, tk,
                                       _ptr(ws), ws.numel()), "orders_linear")
    return out


def set_tuning(ctx: Context, grid: Grid, variant: int) -> None:
    """Pin launch variant `variant` for every pass of this grid's size and precision."""
    g = grid.cstruct
    _check(lib().gridspt_set_tuning(ctx.handle, ctypes.byref(g), int(variant)), "set_tuning")


def tune_orders(ctx: Context, grid: Grid, lp: LinearSpectrum, nmax: int, n2max2: int,
                out: Optional[Orders] = None):
    """Autotune the pass variants of this grid for the context; returns {kind: (variant, ms)}."""
    import numpy as np
    out = out if out is not None else alloc_orders(grid, nmax, True)
    g = grid.cstruct
    c = _linpk(lp)
    ws = ctx.workspace(workspace_bytes(grid, nmax))
    dk = _ptr_array(out.delta_k) if out.delta_k is not None else None
    tk = _ptr_array(out.theta_k) if out.theta_k is not None else None
    _check(lib().gridspt_tune_orders(ctx.handle, ctypes.byref(g), ctypes.byref(c), nmax, n2max2,
                                     _ptr_array(out.delta), _ptr_array(out.theta), dk, tk, _ptr(ws), ws.numel()),
           "tune_orders")
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
    out = out if out is not None else alloc_orders(grid, nmax, spectra)
    g = grid.cstruct
    need = _check(lib().gridspt_pform_workspace_bytes(ctypes.byref(g), nmax), "pform_workspace_bytes")
    ws = ctx.workspace(need)
    d = _ptr_array(out.delta)
    t = _ptr_array(out.theta)
    dk = _ptr_array(out.delta_k) if out.delta_k is not None else None
    tk = _ptr_array(out.theta_k) if out.theta_k is not None else None
    _check(lib().gridspt_orders_pform(ctx.handle, ctypes.byref(g), nmax, n2max1, n2max2, _ptr(delta1), d, t, dk, tk,
                                      _ptr(ws), ws.numel()), "orders_pform")
    return out


def smooth(ctx: Context, grid: Grid, fields_k: Sequence[torch.Tensor], coef: Sequence[float], radius: float,
           cumulative: bool = True, out: Optional[Sequence[torch.Tensor]] = None):
    """Gaussian-smoothed real fields of cube spectra: cumulative sums sum_{i<=j} coef_i F_i
    (the truncated series) or each coef_j F_j; at most five."""
    import numpy as np
    out = list(out) if out is not None else [_new_real(grid) for _ in fields_k]
    c = np.ascontiguousarray(np.asarray(coef, dtype=np.float64))
    g = grid.cstruct
    ws = ctx.workspace(workspace_bytes(grid, 1))
    _check(lib().gridspt_smooth(ctx.handle, ctypes.byref(g), len(fields_k), _ptr_array(fields_k), c.ctypes.data,
                                1 if cumulative else 0, float(radius), _ptr_array(out), _ptr(ws), ws.numel()),
           "smooth")
    return out


def field_stats(ctx: Context, grid: Grid, fields: Sequence[torch.Tensor], nbins: int = 0, lo: float = -1.0,
                hi: float = 1.0, nbins2: int = 0):
    """(moments [nf, 4], corr [nf, nf], counts [nf, nbins] or None, joint [nf-1, nbins2, nbins2] or None)."""
    nf = len(fields)
    dev = dict(device="cuda", dtype=torch.float64)
    mom = torch.empty((nf, 4), **dev)
    cor = torch.empty((nf, nf), **dev)
    cnt = torch.empty((nf, nbins), **dev) if nbins > 0 else None
    jnt = torch.empty((nf - 1, nbins2, nbins2), **dev) if (nbins2 > 0 and nf > 1) else None
    g = grid.cstruct
    need = _check(lib().gridspt_stats_workspace_bytes(nf, nbins, nbins2 if jnt is not None else 0),
                  "stats_workspace_bytes")
    ws = ctx.workspace(need)
    _check(lib().gridspt_field_stats(ctx.handle, ctypes.byref(g), nf, _ptr_array(fields), nbins, float(lo), float(hi),
                                     nbins2, _ptr(mom), _ptr(cor), _ptr(cnt), _ptr(jnt), _ptr(ws), ws.numel()),
           "field_stats")
    return mom, cor, cnt, jnt


def sum_orders(ctx: Context, grid: Grid, delta: Sequence[torch.Tensor], coef: Sequence[float],
               out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """FP64 sum_n coef[n] delta_n(x) (the truncated series of Eq. 8)."""
    import numpy as np
    out = out if out is not None else torch.empty((grid.n,) * 3, dtype=torch.float64, device="cuda")
    c = np.ascontiguousarray(np.asarray(coef, dtype=np.float64))
    g = grid.cstruct
    _check(lib().gridspt_sum_orders(ctx.handle, ctypes.byref(g), len(delta), _ptr_array(delta), c.ctypes.data,
                                    _ptr(out)), "sum_orders")
    return out


def power(ctx: Context, grid: Grid, fields_k: Sequence[torch.Tensor], pairs, edges):
    """Shell-averaged cross spectra; returns (pk [npairs, nbins], kmean, nmodes) as float64 tensors."""
    import numpy as np
    pr = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1))
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int64))
    npairs, nb = pr.size // 2, e.size - 1
    pk = torch.empty((npairs, nb), dtype=torch.float64, device="cuda")
    km = torch.empty(nb, dtype=torch.float64, device="cuda")
    nm = torch.empty(nb, dtype=torch.float64, device="cuda")
    g = grid.cstruct
    need = _check(lib().gridspt_power_workspace_bytes(ctypes.byref(g), npairs, nb), "power_workspace_bytes")
    ws = ctx.workspace(need)
    _check(lib().gridspt_power(ctx.handle, ctypes.byref(g), len(fields_k), _ptr_array(fields_k), npairs,
                               pr.ctypes.data, nb, e.ctypes.data, _ptr(pk), _ptr(km), _ptr(nm), _ptr(ws),
                               ws.numel()), "power")
    return pk, km, nm


def bispectrum(ctx: Context, grid: Grid, fields_k: Sequence[torch.Tensor], tris, terms, edges):
    """FFT-estimator bispectra; returns (bk [nterms], ntriangles [ntri]) as float64 tensors."""
    import numpy as np
    tb = np.ascontiguousarray(np.asarray(tris, dtype=np.int32).reshape(-1))
    tt = np.ascontiguousarray(np.asarray(terms, dtype=np.int32).reshape(-1))
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int64))
    ntri, nterms, nb = tb.size // 3, tt.size // 4, e.size - 1
    bk = torch.empty(nterms, dtype=torch.float64, device="cuda")
    nt = torch.empty(ntri, dtype=torch.float64, device="cuda")
    g = grid.cstruct
    need = _check(lib().gridspt_bispectrum_workspace_bytes(ctypes.byref(g), ntri, tb.ctypes.data, nterms,
                                                           tt.ctypes.data), "bispectrum_workspace_bytes")
    ws = ctx.workspace(need)
    _check(lib().gridspt_bispectrum(ctx.handle, ctypes.byref(g), len(fields_k), _ptr_array(fields_k), ntri,
                                    tb.ctypes.data, nterms, tt.ctypes.data, nb, e.ctypes.data, _ptr(bk), _ptr(nt),
                                    _ptr(ws), ws.numel()), "bispectrum")
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
            dev = dict(device="cuda", dtype=torch.float64)
            o = {"pk_mean": torch.zeros((npairs, nb), **dev), "pk_std": torch.zeros((npairs, nb), **dev),
                 "kmean": torch.zeros(nb, **dev), "nmodes": torch.zeros(nb, **dev)}
            if ntri:
                o.update(bk_mean=torch.zeros(nterms, **dev), bk_std=torch.zeros(nterms, **dev),
                         ntriangles=torch.zeros(ntri, **dev))
            self.out.append(o)
            co[i] = _BatchOut(*[o[k].data_ptr() if k in o else None for k, _ in _BatchOut._fields_])
        self._cg, self._co = cg, co
        need = _check(lib().gridspt_batch_workspace_bytes(ng, cg), "batch_workspace_bytes")
        self.work = torch.empty(max(int(need), 256), dtype=torch.uint8, device="cuda")
        flags = (BATCH_TUNE if tune else 0) | (BATCH_EAGER if eager else 0)
        h = ctypes.c_void_p()
        _check(lib().gridspt_batch_create(ctx.handle, ng, cg, co, _ptr(self.work), self.work.numel(), flags,
                                          ctypes.byref(h)), "batch_create")
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
