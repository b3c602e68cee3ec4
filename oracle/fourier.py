"""Fourier-side steps of the NFFT fast summation, written out plainly (FP64, NumPy).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Every function follows a passage of the paper:

* Continuous Fourier transforms of the kernels: the Gaussian's closed form
  (eq. (FT_gauss) in the proof of Theorem 1, tensor product in d dimensions as
  in the proof of Theorem 1); the derivative kernel's transform via
  eq. (ghat) and the tensor split of the "Derivative Gaussian kernel"
  subsection.  The Matern-1/2 kernel of "Extension to other kernels" has no
  transform in the paper; the textbook transform of exp(-|x|/l) in R^d is
  used (a reading, listed in the design notes).  The same holds for the
  Matern-3/2 kernel (1 + sqrt3 r/l) e^{-sqrt3 r/l}, which that subsection names
  as a further kernel: its transform is the Matern spectral density with
  smoothness 3/2.
* Periodised Fourier coefficients on a torus of period T:
  - ``coeffs_sampled``: discrete coefficients from n^d equidistant kernel
    samples of the simple periodic continuation (Lemma 1, "Fourier theory"
    subsection on periodisation);
  - ``coeffs_analytic``: the continuous transform sampled at k/T (periodisation
    by summation, Poisson's formula) -- the reading used by default.
* The trigonometric sum of eq. (6): h~(x_i) = sum_k c_k a_k e^{2 pi i k x_i}
  with a_k = sum_j v_j e^{-2 pi i k x_j}, evaluated by brute force (a
  non-uniform DFT, no window functions, no FFT).  Its real part is taken: the
  kernel is real and the index set I_n is not symmetric about 0.
* Error bounds of Theorem 1, Remark 1, Theorem 2 and Remark 2 (Fourier
  approximation error section).  Where the statement of Theorem 1 and its
  proof differ for l >= 1/2, the proof's (larger) value is used.
* Global sensitivity indices (Algorithm 1 of the global sensitivity analysis
  section): per window, the coefficients c_k S(k, W) of the trigonometric
  approximation, split by the support of k.  Windows may have any length
  d <= 3 and their own l and torus period (the paper's remark that this case
  is analogous); S(k, W) is evaluated by brute force.
"""
from __future__ import annotations

import math
from typing import Sequence

import numpy as np
from scipy.special import erfc as _erfc, wofz as _wofz

GAUSSIAN = 1
MATERN12 = 3
MATERN32 = 5

# ----------------------------------------------------------------------------
# kernels and their continuous Fourier transforms


def kernel_value(kernel: int, r2, ell: float):
    """kappa(r): Gaussian exp(-r^2/(2l^2)) (eq. (3)); Matern-1/2 exp(-r/l);
    Matern-3/2 (1 + a r) exp(-a r) with a = sqrt(3)/l."""
    r2 = np.asarray(r2, dtype=np.float64)
    if kernel == GAUSSIAN:
        return np.exp(-r2 / (2.0 * ell * ell))
    if kernel == MATERN32:
        ar = np.sqrt(3.0 * r2) / ell
        return (1.0 + ar) * np.exp(-ar)
    return np.exp(-np.sqrt(r2) / ell)


def kernel_der_value(kernel: int, r2, ell: float):
    """The implementation derivative kernels.

    Gaussian (eq. (implement_der_gaussian_kernel)): r^2/(2 l^2) exp(-r^2/(2 l^2)),
    so that dK/dl = (2/l) K_der.  Matern-1/2 ("der_laplacian_rbf"): (r/l) exp(-r/l),
    so that dK/dl = (1/l) K_der.  Matern-3/2, by the same convention
    (K_der = l dK/dl): (a r)^2 exp(-a r) = 3 (r/l)^2 exp(-a r).
    """
    r2 = np.asarray(r2, dtype=np.float64)
    if kernel == GAUSSIAN:
        return r2 / (2.0 * ell * ell) * np.exp(-r2 / (2.0 * ell * ell))
    if kernel == MATERN32:
        ar = np.sqrt(3.0 * r2) / ell
        return ar * ar * np.exp(-ar)
    r = np.sqrt(r2)
    return r / ell * np.exp(-r / ell)


def der_scale(kernel: int, ell: float) -> float:
    """dK_w/dl_w = der_scale * K_der_w (Gaussian 2/l, Matern 1/l)."""
    return 2.0 / ell if kernel == GAUSSIAN else 1.0 / ell


_MATERN_CD = {1: 2.0, 2: 2.0 * math.pi, 3: 8.0 * math.pi}
# Matern-3/2: int_{R^d} (1 + a|x|) e^{-a|x|} dx = c_d l^d with a = sqrt(3)/l
_MATERN32_CD = {1: 4.0 / math.sqrt(3.0), 2: 2.0 * math.pi, 3: 32.0 * math.pi / 3.0 ** 1.5}


def kernel_ft(kernel: int, xi2, ell: float, d: int):
    """Continuous Fourier transform int_{R^d} kappa(x) e^{-2 pi i xi.x} dx at |xi|^2 = xi2."""
    xi2 = np.asarray(xi2, dtype=np.float64)
    if kernel == GAUSSIAN:
        return (ell * math.sqrt(2.0 * math.pi)) ** d * np.exp(-2.0 * math.pi ** 2 * ell * ell * xi2)
    u = 4.0 * math.pi ** 2 * ell * ell * xi2
    if kernel == MATERN32:
        return _MATERN32_CD[d] * ell ** d / (1.0 + u / 3.0) ** ((d + 3) / 2.0)
    return _MATERN_CD[d] * ell ** d / (1.0 + u) ** ((d + 1) / 2.0)


def kernel_der_ft(kernel: int, xi2, ell: float, d: int):
    """Fourier transform of the implementation derivative kernel.

    Gaussian: (d/2 - 2 pi^2 l^2 |xi|^2) times the Gaussian's transform
    (eq. (ghat) per coordinate, summed over the tensor split).
    Matern-1/2: l * d/dl of the transform = (d - (d+1) u/(1+u)) times it,
    u = 4 pi^2 l^2 |xi|^2.  Matern-3/2: l * d/dl of its transform =
    (d - (d+3) (u/3)/(1 + u/3)) times it.
    """
    xi2 = np.asarray(xi2, dtype=np.float64)
    base = kernel_ft(kernel, xi2, ell, d)
    if kernel == GAUSSIAN:
        return (d / 2.0 - 2.0 * math.pi ** 2 * ell * ell * xi2) * base
    u = 4.0 * math.pi ** 2 * ell * ell * xi2
    if kernel == MATERN32:
        return (d - (d + 3) * (u / 3.0) / (1.0 + u / 3.0)) * base
    return (d - (d + 1) * u / (1.0 + u)) * base


# ----------------------------------------------------------------------------
# torus period


def torus_period_auto(kernel: int, L: float, ell: float, n: int) -> float:
    """Per-window torus period T (a reading: the paper leaves the regularisation open).

    Differences of points lie in [-L, L] per coordinate.  Periodisation by
    summation adds images at distance >= T - L; truncating to |k| < n/2 drops
    modes of size ~ kappa_hat(n/(2T)).  For the Gaussian both errors are
    balanced, exp(-(T-L)^2/(2 l^2)) = exp(-2 pi^2 l^2 (n/2)^2 / T^2), giving
    T = (L + sqrt(L^2 + 4 pi l^2 n)) / 2.  For Matern-1/2 the image error
    exp(-(T-L)/l) is set to the algebraic truncation level ~ 1/n:
    T = L + l ln n.  For Matern-3/2 (coefficients decaying like |k|^-(d+3),
    truncation ~ n^-3) the image factor exp(-sqrt3 (T-L)/l) is set to n^-3:
    T = L + sqrt3 l ln n.
    """
    if kernel == GAUSSIAN:
        return 0.5 * (L + math.sqrt(L * L + 4.0 * math.pi * ell * ell * n))
    if kernel == MATERN32:
        return L + math.sqrt(3.0) * ell * math.log(n)
    return L + ell * math.log(n)


def torus_period_paper(Lmax: float, dmax: int) -> float:
    """Prescaling rule of the "Scaling the data" section.

    Data scaled into [-1/4, 1/4]^d (extent 1/2) is divided by sqrt(d_max)
    and placed on the unit torus; in the data's own units that is a period
    T = 2 Lmax sqrt(d_max) for a maximal per-coordinate extent Lmax.
    """
    return 2.0 * Lmax * math.sqrt(dmax)


# ----------------------------------------------------------------------------
# periodised coefficients


def modes(n: int) -> np.ndarray:
    """The index set I_n = {-n/2, ..., n/2 - 1} ("Fourier theory" subsection)."""
    return np.arange(-n // 2, n // 2)


def _k2_grid(n: int, d: int) -> np.ndarray:
    k = modes(n).astype(np.float64)
    grids = np.meshgrid(*([k] * d), indexing="ij")
    return sum(g * g for g in grids)


def coeffs_analytic(kernel: int, ell: float, T: float, n: int, d: int, der: bool = False) -> np.ndarray:
    """b_k = T^{-d} kappa_hat(k / T), k in I_n^d: Fourier coefficients of the
    T-periodisation by summation (Poisson).  Array axes are k_i + n/2."""
    xi2 = _k2_grid(n, d) / (T * T)
    f = kernel_der_ft if der else kernel_ft
    return f(kernel, xi2, ell, d) / T ** d


def coeffs_sampled(kernel: int, ell: float, T: float, n: int, d: int, der: bool = False) -> np.ndarray:
    """c^_k = n^{-d} sum_{j in I_n^d} kappa(T j / n) e^{-2 pi i j.k / n} (Lemma 1),
    the discrete coefficients of the simple periodic continuation on
    [-T/2, T/2)^d.  Real because the samples are even.  Axes are k_i + n/2."""
    j = modes(n).astype(np.float64) * (T / n)
    grids = np.meshgrid(*([j] * d), indexing="ij")
    r2 = sum(g * g for g in grids)
    samp = kernel_der_value(kernel, r2, ell) if der else kernel_value(kernel, r2, ell)
    # index j in I_n sits at array position j + n/2; move j = 0 to position 0
    samp0 = np.fft.ifftshift(samp)
    c = np.fft.fftn(samp0) / n ** d
    return np.fft.fftshift(c).real.copy()


def truncated_gauss_coeff_1d(k, ell: float) -> np.ndarray:
    """c_k of the simple periodic continuation of exp(-r^2/(2l^2)) on [-1/2, 1/2)
    in the closed form l sqrt(2 pi) e^{-2 pi^2 k^2 l^2} Re erf(1/(2 sqrt2 l) + i pi k sqrt2 l)
    ("Fourier theory" subsection).  Evaluated through the Faddeeva function
    w(z) = e^{-z^2} erfc(-iz) so that large k do not overflow:
    erf(z) = 1 - e^{-z^2} w(iz)."""
    k = np.asarray(k, dtype=np.float64)
    x = 1.0 / (2.0 * math.sqrt(2.0) * ell)
    y = math.pi * k * math.sqrt(2.0) * ell
    # e^{-y^2} Re erf(x + i y) = e^{-y^2} - Re(e^{-x^2 - 2 i x y} w(-y + i x))
    val = np.exp(-y * y) - np.real(np.exp(-x * x - 2j * x * y) * _wofz(-y + 1j * x))
    return ell * math.sqrt(2.0 * math.pi) * val


# ----------------------------------------------------------------------------
# brute-force trigonometric sums (eq. (6))

_CHUNK = 4096


def _adjoint_ndft(xt: np.ndarray, v: np.ndarray, n: int) -> np.ndarray:
    """a_k = sum_j v_j exp(-2 pi i k.x_j), k in I_n^d (the inner sum of eq. (6))."""
    N, d = xt.shape
    ks = modes(n).astype(np.float64)
    a = np.zeros((n,) * d, dtype=np.complex128)
    for s in range(0, N, _CHUNK):
        e = slice(s, min(N, s + _CHUNK))
        E = [np.exp(-2j * np.pi * np.outer(xt[e, i], ks)) for i in range(d)]
        vv = v[e].astype(np.complex128)
        if d == 1:
            a += E[0].T @ vv
        elif d == 2:
            a += (E[0] * vv[:, None]).T @ E[1]
        else:
            M = (E[0] * vv[:, None])[:, :, None] * E[1][:, None, :]
            a += (M.reshape(M.shape[0], n * n).T @ E[2]).reshape(n, n, n)
    return a


def _forward_ndft(xt: np.ndarray, h: np.ndarray, n: int) -> np.ndarray:
    """y_i = sum_k h_k exp(2 pi i k.x_i) (the outer sum of eq. (6))."""
    N, d = xt.shape
    ks = modes(n).astype(np.float64)
    y = np.zeros(N, dtype=np.complex128)
    for s in range(0, N, _CHUNK):
        e = slice(s, min(N, s + _CHUNK))
        F = [np.exp(2j * np.pi * np.outer(xt[e, i], ks)) for i in range(d)]
        if d == 1:
            y[e] = F[0] @ h
        elif d == 2:
            y[e] = np.sum((F[0] @ h) * F[1], axis=1)
        else:
            Q = (h.reshape(n * n, n) @ F[2].T).reshape(n, n, -1)
            y[e] = np.einsum("ia,ib,abi->i", F[0], F[1], Q)
    return y


def trig_sum(coef: np.ndarray, xt: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Real part of sum_{k in I_n^d} coef_k (sum_j v_j e^{-2 pi i k.x_j}) e^{2 pi i k.x_i}
    evaluated at the same points x_i = x_j (torus coordinates xt, shape (N, d))."""
    n = coef.shape[0]
    a = _adjoint_ndft(xt, v, n)
    return _forward_ndft(xt, coef * a, n).real


def window_geometry(Xw: np.ndarray):
    """Bounding-box centre and maximal per-coordinate extent L of a window's points."""
    lo = Xw.min(axis=0)
    hi = Xw.max(axis=0)
    return 0.5 * (lo + hi), float(np.max(hi - lo)) if Xw.shape[0] else 0.0


def fast_sum_oracle(X: np.ndarray, windows: Sequence[Sequence[int]], kernel: int, ell, sigma,
                    V: np.ndarray, n: int, periods=None, mode: str = "analytic",
                    want_derivs: bool = False):
    """The paper's approximate matvec with the NFFTs replaced by exact NDFTs.

    For each window: torus coordinates x~ = (x - centre) / T, coefficients of
    kappa (and of the derivative kernel), the trigonometric sum of eq. (6),
    then the window sum with sigma_w^2 (Y), sigma_w^2 * der_scale (dY/dl_w)
    and 2 sigma_w (dY/dsigma_w).  ``periods`` gives T_w (default: the
    automatic rule).  Returns Y (N, R) [, dY_dl (P, N, R), dY_ds (P, N, R)].
    """
    V = np.asarray(V, dtype=np.float64)
    if V.ndim == 1:
        V = V[:, None]
    N, R = V.shape
    P = len(windows)
    ell = np.broadcast_to(np.asarray(ell, dtype=np.float64), (P,))
    sigma = np.broadcast_to(np.asarray(sigma, dtype=np.float64), (P,))
    Y = np.zeros((N, R))
    dl = np.zeros((P, N, R))
    ds = np.zeros((P, N, R))
    for w, feats in enumerate(windows):
        Xw = np.asarray(X, dtype=np.float64)[:, list(feats)]
        d = Xw.shape[1]
        c, L = window_geometry(Xw)
        T = periods[w] if periods is not None else torus_period_auto(kernel, L, ell[w], n)
        xt = (Xw - c) / T
        cf = coeffs_analytic if mode == "analytic" else coeffs_sampled
        ck = cf(kernel, ell[w], T, n, d)
        cd = cf(kernel, ell[w], T, n, d, der=True) if want_derivs else None
        for r in range(R):
            kv = trig_sum(ck, xt, V[:, r])
            Y[:, r] += sigma[w] ** 2 * kv
            ds[w, :, r] = 2.0 * sigma[w] * kv
            if want_derivs:
                dl[w, :, r] = sigma[w] ** 2 * der_scale(kernel, ell[w]) * trig_sum(cd, xt, V[:, r])
    if want_derivs:
        return Y, dl, ds
    return Y


# ----------------------------------------------------------------------------
# global sensitivity indices (Algorithm 1)


def gsi_theta_oracle(X: np.ndarray, windows: Sequence[Sequence[int]], kernel: int, ell, v: np.ndarray, n: int,
                     periods=None, mode: str = "analytic") -> np.ndarray:
    """theta[w, mask] = sum of |c_k S(k, W_w)|^2 over k in I_n^d whose nonzero
    entries are exactly the bits of mask (bit i: i-th feature of the window),
    with S(k, W) = sum_j v_j e^{2 pi i k.x~_j^W} on the window's torus (step 2 of
    Algorithm 1) and c_k the window's periodised coefficients.  Mask 0 is the
    constant term.  Returns an array (P, 8)."""
    X = np.asarray(X, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64).reshape(-1)
    P = len(windows)
    ell = np.broadcast_to(np.asarray(ell, dtype=np.float64), (P,))
    theta = np.zeros((P, 8))
    for w, feats in enumerate(windows):
        Xw = X[:, list(feats)]
        d = Xw.shape[1]
        c, L = window_geometry(Xw)
        T = periods[w] if periods is not None else torus_period_auto(kernel, L, ell[w], n)
        xt = (Xw - c) / T
        cf = coeffs_analytic if mode == "analytic" else coeffs_sampled
        ck = cf(kernel, ell[w], T, n, d)
        S = np.conj(_adjoint_ndft(xt, v, n))  # real v: sum_j v_j e^{+2 pi i k.x_j}
        vals = np.abs(ck * S) ** 2
        grids = np.meshgrid(*([modes(n)] * d), indexing="ij")
        mask = sum((g != 0).astype(np.int64) << i for i, g in enumerate(grids))
        for m in range(1 << d):
            theta[w, m] = vals[mask == m].sum()
    return theta


def gsi_oracle(X: np.ndarray, windows: Sequence[Sequence[int]], kernel: int, ell, v: np.ndarray, n: int,
               periods=None) -> dict:
    """Steps 1-4 of Algorithm 1: theta summed over windows for every nonempty
    feature subset of every window, divided by the total variance."""
    theta = gsi_theta_oracle(X, windows, kernel, ell, v, n, periods)
    acc = {}
    for w, feats in enumerate(windows):
        for m in range(1, 1 << len(feats)):
            key = tuple(sorted(feats[i] for i in range(len(feats)) if m >> i & 1))
            acc[key] = acc.get(key, 0.0) + theta[w, m]
    total = sum(acc.values())
    return {k: val / total for k, val in acc.items()}


# ----------------------------------------------------------------------------
# error bounds (Theorems 1, 2 and Remarks 1, 2).  Here n is the paper's grid size
# per dimension (its m), the kernel length scale is relative to the unit torus.


def eta(ell: float, n: int) -> float:
    return ell * math.pi * n / math.sqrt(2.0)


def gamma_bound(et: float, ell: float) -> float:
    tail = math.exp(-1.0 / (8 * ell * ell)) / et ** 2 if ell < 0.5 else 2.0 * ell * math.exp(-0.5) / et ** 2
    return ell * math.sqrt(2 * math.pi) * math.exp(-et ** 2) + tail


def A_bound(et: float, ell: float) -> float:
    if ell < 0.5:
        tail = math.exp(-1.0 / (8 * ell * ell)) / (math.sqrt(2.0) * ell * math.pi * et)
    else:
        tail = math.sqrt(2.0) * math.exp(-0.5) / (math.pi * et)
    return math.exp(-et ** 2) / (2 * et * math.sqrt(math.pi)) + tail


_ELL_XI = 0.5 * math.sqrt(2.0 / (5.0 + math.sqrt(17.0)))


def xi_bound(et: float, ell: float) -> float:
    if ell <= _ELL_XI:
        tail = math.exp(-1.0 / (8 * ell * ell)) / (8 * et ** 2 * ell ** 2)
    else:
        tail = 1.0 / et ** 2 + 3 * ell / (2 * et ** 2)
    return (et ** 2 + 0.5) * ell * math.sqrt(2 * math.pi) * math.exp(-et ** 2) + tail


def S_bound(et: float, ell: float) -> float:
    if ell <= _ELL_XI:
        tail = math.exp(-1.0 / (8 * ell * ell)) / (8 * math.sqrt(2.0) * math.pi * ell ** 3 * et)
    else:
        tail = 1.0 / (math.sqrt(2.0) * math.pi * ell * et) + 3.0 / (2 * math.sqrt(2.0) * math.pi * et)
    return (float(_erfc(et)) / 4 + et * math.exp(-et ** 2) / (2 * math.sqrt(math.pi))
            + math.exp(-et ** 2) / (4 * math.sqrt(math.pi) * et) + tail)


def theorem1_bound(ell: float, n: int) -> float:
    """Bound on ||kappa_ERR||_inf for the trivariate Gaussian (Theorem 1), eta >= 1."""
    et = eta(ell, n)
    if et < 1.0:
        raise ValueError("Theorem 1 needs eta >= 1")
    g = gamma_bound(et, ell)
    return 15 * g * (g + 2.5) + 102 * A_bound(et, ell)


def remark1_bound(ell: float, n: int) -> float:
    et = eta(ell, n)
    if et < 1.0:
        raise ValueError("Remark 1 needs eta >= 1")
    return 2 * gamma_bound(et, ell) + 4 * A_bound(et, ell)


def theorem2_bound(ell: float, n: int) -> float:
    """Bound on ||kappa_ERR||_inf for the trivariate derivative Gaussian (Theorem 2)."""
    et = eta(ell, n)
    if et < 1.0:
        raise ValueError("Theorem 2 needs eta >= 1")
    g, A, x, S = gamma_bound(et, ell), A_bound(et, ell), xi_bound(et, ell), S_bound(et, ell)
    return (2.5 * x + 15 * g) * (15 + 12 * g) + 75 * S + 6 * A * (116.0 / 5.0 * S + 87)


def remark2_bound(ell: float, n: int) -> float:
    et = eta(ell, n)
    if et < 1.0:
        raise ValueError("Remark 2 needs eta >= 1")
    return 2 * xi_bound(et, ell) + 4 * S_bound(et, ell)


def measured_fourier_error(kernel_der: bool, ell: float, n: int, d: int, npts: int, seed: int) -> float:
    """max_j |kappa(r_j) - kappa_F(r_j)| for uniform r_j in [-1/2, 1/2]^d, with
    kappa_F the trigonometric polynomial with sampled coefficients on the unit
    torus (the experiment comparing measured errors with the bounds)."""
    rng = np.random.default_rng(seed)
    r = rng.uniform(-0.5, 0.5, size=(npts, d))
    c = coeffs_sampled(GAUSSIAN, ell, 1.0, n, d, der=kernel_der)
    kf = _forward_ndft(r, c.astype(np.complex128), n).real
    r2 = np.sum(r * r, axis=1)
    kv = kernel_der_value(GAUSSIAN, r2, ell) if kernel_der else kernel_value(GAUSSIAN, r2, ell)
    return float(np.max(np.abs(kv - kf)))
