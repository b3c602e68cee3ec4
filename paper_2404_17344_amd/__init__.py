"""Fast additive-kernel matvecs on AMD MI355X (gfx950).

Python face of ``libaddk.so`` (C ABI in ``include/addk.h``).  This module only
marshals arguments: every step of the products runs in the library's HIP
kernels.  Torch supplies device memory and the current stream.

Layout: an (N, R) tensor ``V`` is handed to the library as a column-major
N x R matrix (its transpose is made contiguous), results come back as (N, R)
views of column-major buffers.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np

from . import _lib
from ._lib import (ADDK_FP32, ADDK_FP64, ADDK_GAUSSIAN, ADDK_MATERN12, ADDK_MATERN32, AddkError,  # noqa: F401
                   ADDK_COEF_SAMPLED, ADDK_TORUS_PAPER, ADDK_NO_ACCURACY_CHECK, ADDK_KNOB_SPREAD_MFMA,
                   ADDK_KNOB_INTERP_DENSE_MFMA, ADDK_KNOB_INTERP_TILE_MFMA, ADDK_KNOB_ALL_MFMA,
                   ADDK_KNOB_SPREAD_SPLIT, ADDK_KNOB_ALL, ADDK_KNOB_SPARSE_ATOMIC)

__all__ = ["Plan", "Batch", "AddkError", "addk_matvec", "torus_period", "window_ft", "choose_n", "choose_n_for",
           "KernelMatvec", "tune_cache_clear"]


def tune_cache_clear():
    """Forget the knobs recorded by every autotune of the process (addk_tune_cache_clear)."""
    _lib.check(_lib.load().addk_tune_cache_clear(), "addk_tune_cache_clear")

_KERNELS = {"gaussian": ADDK_GAUSSIAN, "matern12": ADDK_MATERN12, "matern32": ADDK_MATERN32,
            ADDK_GAUSSIAN: ADDK_GAUSSIAN, ADDK_MATERN12: ADDK_MATERN12, ADDK_MATERN32: ADDK_MATERN32}
_PREC = {"fp64": ADDK_FP64, "fp32": ADDK_FP32, ADDK_FP64: ADDK_FP64, ADDK_FP32: ADDK_FP32}


def _torch():
    import torch
    return torch


def _stream(stream=None) -> ctypes.c_void_p:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _colmajor(V):
    """(N,) or (N, R) float64 CUDA tensor -> contiguous (R, N) tensor (column-major N x R)."""
    torch = _torch()
    if not isinstance(V, torch.Tensor) or not V.is_cuda:
        raise TypeError("expected a CUDA tensor")
    if V.dtype != torch.float64:
        raise TypeError("expected float64 (the ABI takes FP64 inputs and outputs)")
    if V.dim() == 1:
        V = V[:, None]
    return V.t().contiguous()


def torus_period(kernel, L: float, ell: float, n: int, paper_rule: bool = False, dmax: int = 3) -> float:
    lib = _lib.load()
    T = ctypes.c_double()
    _lib.check(lib.addk_torus_period(_KERNELS[kernel], L, ell, n, ADDK_TORUS_PAPER if paper_rule else 0, dmax,
                                     ctypes.byref(T)), "addk_torus_period")
    return T.value


def window_ft(m: int, n_os: int, oversampling: float, k: float) -> float:
    lib = _lib.load()
    v = ctypes.c_double()
    _lib.check(lib.addk_window_ft(m, n_os, oversampling, k, ctypes.byref(v)), "addk_window_ft")
    return v.value


def choose_n(kernel, L: float, ell: float, m: int = 6, oversampling: float = 2.0, tol: float = 1e-5):
    """Smallest supported bandwidth n meeting tol for one window (extent L, length scale l).

    Returns (n, error estimate); raises AddkError (ACCURACY) when none does."""
    lib = _lib.load()
    n = ctypes.c_int32()
    err = ctypes.c_double()
    _lib.check(lib.addk_choose_n(_KERNELS[kernel], float(L), float(ell), int(m), float(oversampling), float(tol),
                                 ctypes.byref(n), ctypes.byref(err)), "addk_choose_n")
    return n.value, err.value


def _win_arrays(windows):
    off = [0]
    feat = []
    for w in windows:
        feat.extend(int(f) for f in w)
        off.append(len(feat))
    return (ctypes.c_int32 * len(off))(*off), (ctypes.c_int32 * max(1, len(feat)))(*feat)


def choose_n_for(X, windows: Sequence[Sequence[int]], ell, kernel="gaussian", m: int = 6,
                 oversampling: float = 2.0, tol: float = 1e-5, with_estimate: bool = False):
    """Bandwidth for a whole plan (addk_choose_n_windows): the largest per-window
    choice.  X: (N, D) host array or CUDA tensor.  Returns n, or (n, estimate)."""
    lib = _lib.load()
    torch = _torch()
    if isinstance(X, torch.Tensor):
        Xk = X.detach().to(torch.float64).contiguous()
        N, D = Xk.shape
        xptr = Xk.data_ptr() if N else None
        st = _stream()
    else:
        Xk = np.ascontiguousarray(np.asarray(X, dtype=np.float64))
        N, D = Xk.shape
        xptr = Xk.ctypes.data if N else None
        st = ctypes.c_void_p(0)
    off_a, feat_a = _win_arrays(windows)
    ell_a = np.ascontiguousarray(np.broadcast_to(np.asarray(ell, dtype=np.float64), (len(windows),)))
    n = ctypes.c_int32()
    err = ctypes.c_double()
    _lib.check(lib.addk_choose_n_windows(_KERNELS[kernel], N, D, xptr, D, len(windows), off_a, feat_a,
                                         ell_a.ctypes.data_as(_lib._pd), int(m), float(oversampling), float(tol),
                                         ctypes.byref(n), ctypes.byref(err), st), "addk_choose_n_windows")
    return (n.value, err.value) if with_estimate else n.value


class Plan:
    """A plan for y = sum_w sigma_w^2 K_w v over fixed points and windows."""

    def __init__(self, X, windows: Sequence[Sequence[int]], ell, sigma, kernel="gaussian", n: int = 64,
                 m: int = 6, oversampling: float = 2.0, precision="fp64", coef: str = "analytic",
                 torus: str = "auto", check_accuracy: bool = True, dense_kernels: bool = True, matrix_cores: bool = True,
                 targets=None, near_field: bool = False, stream=None):
        """X: sources (N, D), host array or CUDA tensor.  targets: optional (Nt, D)
        prediction points; the plan's products then map N-row V to Nt-row Y.
        near_field (Matern kernels only): regularised multipliers on an image-free
        torus plus a direct sum over close pairs (ADDK_NEAR_FIELD), which
        brings the products to ~1e-5 of the direct sum."""
        lib = _lib.load()
        torch = _torch()

        def _points(A):
            if isinstance(A, torch.Tensor):
                At = A.detach().to(torch.float64).contiguous()
                return At, At.shape[0], At.shape[1], (At.data_ptr() if At.shape[0] else None)
            An = np.ascontiguousarray(np.asarray(A, dtype=np.float64))
            return An, An.shape[0], An.shape[1], (An.ctypes.data if An.shape[0] else None)

        self._xkeep, N, D, xptr = _points(X)
        if targets is not None:
            self._tkeep, Nt, Dt, tptr = _points(targets)
            if Dt != D:
                raise ValueError("targets must have the sources' number of features")
        self.P = len(windows)
        self.N = int(N)  # rows of V
        self.N_out = int(Nt) if targets is not None else int(N)  # rows of Y
        self.windows = [list(w) for w in windows]
        off_a, feat_a = _win_arrays(windows)
        ell_a = np.ascontiguousarray(np.broadcast_to(np.asarray(ell, dtype=np.float64), (self.P,)))
        sig_a = np.ascontiguousarray(np.broadcast_to(np.asarray(sigma, dtype=np.float64), (self.P,)))
        flags = 0
        if coef == "sampled":
            flags |= ADDK_COEF_SAMPLED
        if torus == "paper":
            flags |= ADDK_TORUS_PAPER
        if not check_accuracy:
            flags |= ADDK_NO_ACCURACY_CHECK
        if not dense_kernels:
            flags |= _lib.ADDK_TILE_KERNELS_ONLY
        if not matrix_cores:
            flags |= _lib.ADDK_VECTOR_ALU_ONLY
        if near_field:
            flags |= _lib.ADDK_NEAR_FIELD
        h = ctypes.c_void_p()
        st = _stream(stream) if torch.cuda.is_available() else ctypes.c_void_p(0)
        if targets is None:
            _lib.check(lib.addk_plan_create(ctypes.byref(h), N, D, xptr, D, self.P, off_a, feat_a, _KERNELS[kernel],
                                            ell_a.ctypes.data_as(_lib._pd), sig_a.ctypes.data_as(_lib._pd), n, m,
                                            float(oversampling), _PREC[precision], flags, st), "addk_plan_create")
        else:
            _lib.check(lib.addk_plan_create_targets(ctypes.byref(h), N, Nt, D, xptr, D, tptr, D, self.P, off_a,
                                                    feat_a, _KERNELS[kernel], ell_a.ctypes.data_as(_lib._pd),
                                                    sig_a.ctypes.data_as(_lib._pd), n, m, float(oversampling),
                                                    _PREC[precision], flags, st), "addk_plan_create_targets")
        self._h = h
        self._lib = lib
        self.kernel = _KERNELS[kernel]
        self.precision = _PREC[precision]
        self.ell = ell_a.copy()
        self.sigma = sig_a.copy()

    # -- lifetime
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.check(self._lib.addk_plan_destroy(self._h), "addk_plan_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    # -- facts
    def query(self):
        info = _lib.AddkPlanInfo()
        T = (ctypes.c_double * self.P)()
        eta = (ctypes.c_double * self.P)()
        dims = (ctypes.c_int32 * self.P)()
        _lib.check(self._lib.addk_plan_query(self._h, ctypes.byref(info), T, eta, dims), "addk_plan_query")
        return {"N": info.N, "P": info.P, "n": info.n, "m": info.m, "n_os": info.n_os,
                "precision": info.precision, "kernel": info.kernel, "workspace_bytes": info.workspace_bytes,
                "err_estimate": info.err_estimate, "T": list(T), "eta": list(eta), "d": list(dims),
                "dense_points": info.dense_points, "tile_points": info.tile_points,
                "knobs": info.knobs, "tuned": bool(info.tuned), "n_sources": info.n_sources,
                "n_targets": info.n_targets}

    def gsi_theta(self, v, stream=None) -> np.ndarray:
        """Per-window variance contributions theta (P, 8) by support mask (see addk_gsi)."""
        vc = _colmajor(v)
        if vc.shape[0] != 1:
            raise ValueError("gsi takes one right-hand side")
        th = np.zeros(8 * self.P)
        _lib.check(self._lib.addk_gsi(self._h, vc.data_ptr(), th.ctypes.data_as(_lib._pd), _stream(stream)),
                   "addk_gsi")
        return th.reshape(self.P, 8)

    def gsi(self, v, stream=None) -> dict:
        """Global sensitivity indices {feature tuple: rho} over all windows and
        their subsets (addk_gsi_indices)."""
        vc = _colmajor(v)
        if vc.shape[0] != 1:
            raise ValueError("gsi takes one right-hand side")
        cap = 7 * self.P
        subsets = (ctypes.c_int32 * (3 * cap))()
        rho = np.zeros(cap)
        count = ctypes.c_int32()
        _lib.check(self._lib.addk_gsi_indices(self._h, vc.data_ptr(), cap, subsets, rho.ctypes.data_as(_lib._pd),
                                              ctypes.byref(count), _stream(stream)), "addk_gsi_indices")
        return {tuple(f for f in subsets[3 * j:3 * j + 3] if f >= 0): float(rho[j]) for j in range(count.value)}

    def autotune(self, R: int, nout: int = 1, reps: int = 3, stream=None) -> int:
        """Time the kernel-variant combinations on this plan and keep the fastest (ADDK_KNOB_* mask)."""
        k = ctypes.c_uint32()
        _lib.check(self._lib.addk_plan_autotune(self._h, int(R), int(nout), int(reps), ctypes.byref(k),
                                                _stream(stream)), "addk_plan_autotune")
        return k.value

    def set_knobs(self, knobs: int):
        """Run with these ADDK_KNOB_* (as if tuned; addk_plan_set_knobs)."""
        _lib.check(self._lib.addk_plan_set_knobs(self._h, int(knobs)), "addk_plan_set_knobs")

    def cached_knobs(self, R: int, nout: int = 1):
        """The knobs the tuning cache holds for this plan's shape at (R, nout), or None."""
        k, found = ctypes.c_uint32(), ctypes.c_int32()
        _lib.check(self._lib.addk_tune_cache_lookup(self._h, int(R), int(nout), ctypes.byref(k), ctypes.byref(found)),
                   "addk_tune_cache_lookup")
        return k.value if found.value else None

    def update_params(self, ell, sigma, stream=None):
        ell_a = np.ascontiguousarray(np.broadcast_to(np.asarray(ell, dtype=np.float64), (self.P,)))
        sig_a = np.ascontiguousarray(np.broadcast_to(np.asarray(sigma, dtype=np.float64), (self.P,)))
        _lib.check(self._lib.addk_plan_update_params(self._h, ell_a.ctypes.data_as(_lib._pd),
                                                     sig_a.ctypes.data_as(_lib._pd), _stream(stream)),
                   "addk_plan_update_params")
        self.ell, self.sigma = ell_a.copy(), sig_a.copy()

    # -- stage timing (HIP events recorded around every stage launch)
    def profile(self, enable: bool = True):
        _lib.check(self._lib.addk_plan_profile(self._h, 1 if enable else 0), "addk_plan_profile")

    def profile_read(self):
        """{stage name: (total_ms, launches)} since the last read (synchronises)."""
        ms = (ctypes.c_double * _lib.ADDK_NSTAGES)()
        cnt = (ctypes.c_int32 * _lib.ADDK_NSTAGES)()
        _lib.check(self._lib.addk_plan_profile_read(self._h, ms, cnt), "addk_plan_profile_read")
        return {self._lib.addk_stage_name(s).decode(): (ms[s], cnt[s]) for s in range(_lib.ADDK_NSTAGES)}

    # -- products
    def matvec(self, V, out=None, stream=None):
        torch = _torch()
        Vc = _colmajor(V)
        R = Vc.shape[0]
        Yc = out if out is not None else torch.empty((R, self.N_out), dtype=torch.float64, device=Vc.device)
        _lib.check(self._lib.addk_matvec(self._h, R, Vc.data_ptr(), max(self.N, 1), Yc.data_ptr(),
                                         max(self.N_out, 1), _stream(stream)), "addk_matvec")
        return Yc.t()

    def matvec_noalloc(self, V, out, stream=None):
        """K V into the caller's column-major (R, N) buffer ``out`` with no device
        allocation: the workspace is the library's fixed per-GPU array."""
        Vc = _colmajor(V)
        R = Vc.shape[0]
        if tuple(out.shape) != (R, self.N_out) or not out.is_contiguous():
            raise ValueError("out must be a contiguous (R, N_out) float64 CUDA tensor")
        _lib.check(self._lib.addk_matvec_noalloc(self._h, R, Vc.data_ptr(), max(self.N, 1), out.data_ptr(),
                                                 max(self.N_out, 1), _stream(stream)), "addk_matvec_noalloc")
        return out.t()

    def cg(self, Y, beta: float, tol: float = 1e-3, maxit: int = 500, X0=None, stream=None):
        """Solve (K + beta I) X = Y by conjugate gradients (eq. (9)); returns (X, iterations, relres)."""
        torch = _torch()
        Yc = _colmajor(Y)
        R = Yc.shape[0]
        Xc = _colmajor(X0).clone() if X0 is not None else torch.zeros_like(Yc)
        it = ctypes.c_int32()
        rel = np.zeros(R)
        _lib.check(self._lib.addk_cg(self._h, float(beta), R, Yc.data_ptr(), max(self.N, 1), Xc.data_ptr(),
                                     max(self.N, 1), float(tol), int(maxit), ctypes.byref(it),
                                     rel.ctypes.data_as(_lib._pd), _stream(stream)), "addk_cg")
        return Xc.t(), it.value, rel

    def dmatvec(self, V, want_y=True, want_dell=True, want_dsigma=True, stream=None):
        """Returns (Y, dY_dell, dY_dsigma) with dY_* of shape (P, N, R) (None where not requested)."""
        torch = _torch()
        Vc = _colmajor(V)
        R = Vc.shape[0]
        dev = Vc.device
        Y = torch.empty((R, self.N_out), dtype=torch.float64, device=dev) if want_y else None
        dl = torch.empty((self.P, R, self.N_out), dtype=torch.float64, device=dev) if want_dell else None
        ds = torch.empty((self.P, R, self.N_out), dtype=torch.float64, device=dev) if want_dsigma else None
        p = lambda t: t.data_ptr() if t is not None else None  # noqa: E731
        _lib.check(self._lib.addk_dmatvec(self._h, R, Vc.data_ptr(), max(self.N, 1), p(dl), p(ds), p(Y),
                                          max(self.N_out, 1), _stream(stream)), "addk_dmatvec")
        t2 = lambda t: t.transpose(1, 2) if t is not None else None  # noqa: E731
        return (Y.t() if Y is not None else None), t2(dl), t2(ds)

    def vjp(self, V, G, want_v=True, want_params=True, stream=None):
        """Gradients of <G, K V>: (K G, d/dl_w, d/dsigma_w)."""
        torch = _torch()
        Gc = _colmajor(G)
        R = Gc.shape[0]
        Vc = _colmajor(V) if want_params else None
        dev = Gc.device
        gV = torch.empty((R, self.N), dtype=torch.float64, device=dev) if want_v else None
        gl = torch.empty((self.P,), dtype=torch.float64, device=dev) if want_params else None
        gs = torch.empty((self.P,), dtype=torch.float64, device=dev) if want_params else None
        p = lambda t: t.data_ptr() if t is not None else None  # noqa: E731
        _lib.check(self._lib.addk_vjp(self._h, R, p(Vc), max(self.N, 1), Gc.data_ptr(), max(self.N, 1), p(gV),
                                      max(self.N, 1), p(gl), p(gs), _stream(stream)), "addk_vjp")
        return (gV.t() if gV is not None else None), gl, gs


class Batch:
    """Many plans multiplied together with bound device buffers, replayed as one hipGraph."""

    def __init__(self, plans: Sequence[Plan], R: int, stream=None):
        torch = _torch()
        lib = _lib.load()
        self.plans = list(plans)
        self.R = R
        self.V = [torch.zeros((R, p.N), dtype=torch.float64, device="cuda") for p in self.plans]
        self.Y = [torch.zeros((R, p.N), dtype=torch.float64, device="cuda") for p in self.plans]
        n = len(self.plans)
        hp = (ctypes.c_void_p * n)(*[p.handle.value for p in self.plans])
        vp = (ctypes.c_void_p * n)(*[t.data_ptr() for t in self.V])
        yp = (ctypes.c_void_p * n)(*[t.data_ptr() for t in self.Y])
        ld = (ctypes.c_int64 * n)(*[max(p.N, 1) for p in self.plans])
        h = ctypes.c_void_p()
        torch.cuda.synchronize()
        _lib.check(lib.addk_batch_create(ctypes.byref(h), n, hp, R, vp, ld, yp, ld, _stream(stream)),
                   "addk_batch_create")
        self._h = h
        self._lib = lib

    def set_inputs(self, Vs):
        for dst, src in zip(self.V, Vs):
            dst.copy_(_colmajor(src))

    def outputs(self):
        return [y.t() for y in self.Y]

    def launch(self, stream=None):
        _lib.check(self._lib.addk_batch_launch(self._h, _stream(stream)), "addk_batch_launch")

    def autotune(self, reps: int = 3, stream=None) -> int:
        """Time the kernel-variant combinations on the graph, keep (and re-capture) the fastest."""
        k = ctypes.c_uint32()
        _lib.check(self._lib.addk_batch_autotune(self._h, int(reps), ctypes.byref(k), _stream(stream)),
                   "addk_batch_autotune")
        return k.value

    def run_eager(self, stream=None):
        _lib.check(self._lib.addk_batch_run_eager(self._h, _stream(stream)), "addk_batch_run_eager")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.check(self._lib.addk_batch_destroy(self._h), "addk_batch_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def addk_matvec(plan: Plan, V):
    return plan.matvec(V)


from .autograd import KernelMatvec  # noqa: E402
