"""ctypes wrapper of ``direct.c`` (plain FP64 direct sums).  TEST INFRASTRUCTURE ONLY.

The C source follows the kernel definitions of eq. (3) and eqs. (7)-(8), the l- and
sigma-derivatives of the section "Implementing the NFFT approach" (Gaussian)
and of "Extension to other kernels" (Matern-1/2, and the Matern-3/2 kernel that
section names as a further kernel).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "direct.c")
_lib = None


def build_oracle(force: bool = True) -> str:
    """Compile direct.c with gcc (IEEE math, no fast-math) into liboracle.so."""
    if force or not os.path.exists(lib_path):
        tmp = lib_path + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, lib_path)
    return lib_path


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(lib_path):
            build_oracle(force=True)
        lib = ctypes.CDLL(lib_path)
        d = ctypes.POINTER(ctypes.c_double)
        i32 = ctypes.POINTER(ctypes.c_int32)
        i64 = ctypes.POINTER(ctypes.c_int64)
        lib.oracle_direct.restype = ctypes.c_int
        lib.oracle_direct.argtypes = [ctypes.c_int64, ctypes.c_int32, d, ctypes.c_int64,
                                      ctypes.c_int32, i32, i32, ctypes.c_int32, d, d,
                                      ctypes.c_int32, d, ctypes.c_int64,
                                      ctypes.c_int64, i64, d, ctypes.c_int64, d, d]
        lib.oracle_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def oracle_threads() -> int:
    return int(_load().oracle_num_threads())


def _ptr(a, ty):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ty))


def oracle_direct(X: np.ndarray, windows: Sequence[Sequence[int]], kernel: int,
                  ell, sigma, V: np.ndarray, rows: Optional[np.ndarray] = None,
                  want_derivs: bool = False):
    """Direct FP64 sums.

    Returns ``Y`` of shape (nrows, R) and, if ``want_derivs``, also
    ``dY_dl`` and ``dY_ds`` of shape (P, nrows, R):

        Y       = sum_w sigma_w^2 K_w V
        dY_dl_w = sigma_w^2 (dK_w/dl_w) V
        dY_ds_w = 2 sigma_w K_w V
    """
    X = np.ascontiguousarray(X, dtype=np.float64)
    N, D = X.shape
    V = np.asarray(V, dtype=np.float64)
    if V.ndim == 1:
        V = V[:, None]
    Vf = np.asfortranarray(V)
    R = Vf.shape[1]
    off = [0]
    feat = []
    for w in windows:
        feat.extend(int(f) for f in w)
        off.append(len(feat))
    off_a = np.asarray(off, dtype=np.int32)
    feat_a = np.asarray(feat, dtype=np.int32)
    P = len(windows)
    ell_a = np.ascontiguousarray(np.broadcast_to(np.asarray(ell, dtype=np.float64), (P,)))
    sig_a = np.ascontiguousarray(np.broadcast_to(np.asarray(sigma, dtype=np.float64), (P,)))
    if rows is None:
        nrows = N
        rows_a = None
    else:
        rows_a = np.ascontiguousarray(rows, dtype=np.int64)
        nrows = rows_a.shape[0]
        if nrows and (rows_a.min() < 0 or rows_a.max() >= N):
            raise ValueError("row index out of range")
    ldy = max(nrows, 1)
    Y = np.zeros((R, ldy), dtype=np.float64)
    dl = np.zeros((P, R, ldy), dtype=np.float64) if want_derivs else None
    ds = np.zeros((P, R, ldy), dtype=np.float64) if want_derivs else None
    rc = _load().oracle_direct(N, D, _ptr(X, ctypes.c_double), D, P,
                               _ptr(off_a, ctypes.c_int32), _ptr(feat_a, ctypes.c_int32),
                               int(kernel), _ptr(ell_a, ctypes.c_double), _ptr(sig_a, ctypes.c_double),
                               R, _ptr(Vf, ctypes.c_double), max(N, 1), nrows,
                               _ptr(rows_a, ctypes.c_int64), _ptr(Y, ctypes.c_double), ldy,
                               _ptr(dl, ctypes.c_double), _ptr(ds, ctypes.c_double))
    if rc != 0:
        raise ValueError("oracle_direct rejected its arguments (code %d)" % rc)
    Yo = Y[:, :nrows].T.copy()
    if not want_derivs:
        return Yo
    return Yo, np.transpose(dl[:, :, :nrows], (0, 2, 1)).copy(), np.transpose(ds[:, :, :nrows], (0, 2, 1)).copy()


def oracle_vjp(X, windows, kernel, ell, sigma, V, G):
    """Gradients of L = <G, K V> (Frobenius) w.r.t. V, l_w and sigma_w.

    K is symmetric, so dL/dV = K G; dL/dl_w = <G, dK/dl_w V>;
    dL/dsigma_w = <G, 2 sigma_w K_w V>.
    """
    gV = oracle_direct(X, windows, kernel, ell, sigma, G)
    _, dl, ds = oracle_direct(X, windows, kernel, ell, sigma, V, want_derivs=True)
    G = np.asarray(G, dtype=np.float64).reshape(dl.shape[1], dl.shape[2])
    gl = np.einsum("wir,ir->w", dl, G)
    gs = np.einsum("wir,ir->w", ds, G)
    return gV, gl, gs
