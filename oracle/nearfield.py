"""Near-field corrected fast summation for the Matern kernels (FP64, NumPy).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The Matern-1/2 kernel exp(-r/l) of the "Extension to other kernels"
subsection has a cusp at r = 0, so its Fourier coefficients decay only
algebraically (like |k|^-(d+1)) and a truncated Fourier series of it stays
far from 1e-5.  Fast summation with non-smooth kernels splits the kernel in a
smooth part, summed by the Fourier method, and a compactly supported
near-field part, summed directly over close pairs (the regularisation of
NFFT-based fast summation that the paper builds on; the paper gives no
formulas for it, so every choice below is this implementation's reading):

* Torus.  T = (5/2) L for a window whose points span at most L per coordinate
  (L replaced by l when all points coincide, L = 0).
  The kernel is made T-periodic without images: each coordinate's square x^2
  is replaced by s(x) = x^2 (1 - h) + (T - x)^2 h on [0, T), with h a smooth
  step rising from 0 at x = L to 1 at x = T - L.  s is even and T-periodic,
  equals x^2 for |x| <= L, and so the periodic kernel equals the true kernel
  for every difference of two points of the window.
* Inner regularisation.  Inside r < eps the kernel is replaced by the even
  polynomial p(r) = sum_j a_j (r/eps)^(2j), j = 0..q, whose value and first q
  derivatives at r = eps are those of the kernel.  The near-field kernel is
  K_NE(r) = kappa(r) - p(r) for r < eps and 0 beyond.
* Coefficients.  The smooth periodic kernel K_R = kappa(sqrt(sum s(x_i))) - K_NE(|x|)
  is sampled on M^d points of the torus (M = 2n) and transformed with a DFT,
  as in Lemma 1 with the regularised kernel in place of kappa.
* Product.  K v = (trigonometric sum of eq. (6) with these coefficients)
  + (sum over pairs closer than eps of K_NE(|x_i - x_j|) v_j).

The derivative kernel (r/l) exp(-r/l) gets the same treatment with its own
polynomial.  Parameters: T = 5L/2, eps = 5 T / n, q = 8, step h = the
degree-7 smoothstep t^4 (35 - 84 t + 70 t^2 - 20 t^3).

The Matern-3/2 kernel (1 + a r) e^{-a r}, a = sqrt(3)/l, named in the same
subsection as a further kernel, is smooth at r = 0 only to second order (a
|r|^3 term), so its coefficients decay like |k|^-(d+3) and the truncated
series alone stays near 1e-3; it takes the same correction with the same
parameters, its derivative kernel being (a r)^2 e^{-a r} (= l dkappa/dl).
"""
from __future__ import annotations

import math
from typing import Sequence

import numpy as np

from .fourier import MATERN12, MATERN32, modes, trig_sum, window_geometry, der_scale

NEAR_Q = 8            # matched derivatives at r = eps
NEAR_P = 5.0          # eps = NEAR_P * T / n
FOLD_RATIO = 2.5      # T = FOLD_RATIO * L
SAMPLE_FACTOR = 2     # M = SAMPLE_FACTOR * n samples per axis


def fold_width(L: float, ell: float) -> float:
    """Half-width L_f of the unfolded region: L, or l for a window of identical
    points (L = 0), so that the near-field radius 5 T / n = 12.5 L_f / n stays
    inside the unfolded region for n >= 16."""
    return L if L > 0.0 else ell


def near_period(L: float, ell: float) -> float:
    """Torus period of a near-field window: T = 5 L_f / 2."""
    return FOLD_RATIO * fold_width(L, ell)


def near_radius(T: float, n: int) -> float:
    return NEAR_P * T / n


def smoothstep7(t):
    """t^4 (35 - 84 t + 70 t^2 - 20 t^3) on [0, 1], clamped outside: C^3, and
    smoothstep7(t) + smoothstep7(1 - t) = 1."""
    t = np.clip(np.asarray(t, dtype=np.float64), 0.0, 1.0)
    return t ** 4 * (35.0 - 84.0 * t + 70.0 * t * t - 20.0 * t ** 3)


def fold_sq(x, L: float, T: float):
    """The folded square s(x): even, T-periodic, x^2 for |x| <= L."""
    x = np.mod(np.asarray(x, dtype=np.float64), T)
    if T <= 2.0 * L:
        raise ValueError("fold needs T > 2 L")
    h = smoothstep7((x - L) / (T - 2.0 * L))
    return x * x * (1.0 - h) + (T - x) ** 2 * h


def _kappa(r, ell: float, der: bool, kernel: int = MATERN12):
    r = np.asarray(r, dtype=np.float64)
    if kernel == MATERN32:
        ar = math.sqrt(3.0) * r / ell
        e = np.exp(-ar)
        return ar * ar * e if der else (1.0 + ar) * e
    e = np.exp(-r / ell)
    return r / ell * e if der else e


def _kappa_derivs(r: float, ell: float, der: bool, q: int, kernel: int = MATERN12):
    """d^s/dr^s kappa at r, s = 0..q.

    exp(-r/l): (-1/l)^s e^{-r/l}; (r/l) e^{-r/l}: (-1/l)^s e^{-r/l} (r - s l) / l
    (Leibniz on r * e^{-r/l}).  With a = sqrt(3)/l: (1 + a r) e^{-a r}:
    (-a)^s e^{-a r} (1 + a r - s); (a r)^2 e^{-a r}: (-a)^s e^{-a r}
    ((a r)^2 - 2 s a r + s (s - 1)) (Leibniz on r^2 * e^{-a r})."""
    out = []
    if kernel == MATERN32:
        a = math.sqrt(3.0) / ell
        e = math.exp(-a * r)
        for s in range(q + 1):
            f = (-a) ** s * e
            ar = a * r
            out.append(f * (ar * ar - 2 * s * ar + s * (s - 1)) if der else f * (1.0 + ar - s))
        return np.array(out)
    e = math.exp(-r / ell)
    for s in range(q + 1):
        f = (-1.0 / ell) ** s * e
        out.append(f * (r - s * ell) / ell if der else f)
    return np.array(out)


def taylor_even_poly(ell: float, eps: float, der: bool, q: int = NEAR_Q, kernel: int = MATERN12) -> np.ndarray:
    """a_0..a_q of p(r) = sum_j a_j (r/eps)^(2j) with p^(s)(eps) = kappa^(s)(eps), s <= q.

    In t = r/eps: sum_j a_j (2j)!/(2j-s)! = eps^s kappa^(s)(eps)."""
    A = np.zeros((q + 1, q + 1))
    for s in range(q + 1):
        for j in range(q + 1):
            p = 2 * j
            A[s, j] = math.prod(range(p - s + 1, p + 1)) if s <= p else 0.0
    rhs = _kappa_derivs(eps, ell, der, q, kernel) * np.array([eps ** s for s in range(q + 1)])
    return np.linalg.solve(A, rhs)


def even_poly(a: np.ndarray, t):
    t2 = np.asarray(t, dtype=np.float64) ** 2
    return sum(c * t2 ** j for j, c in enumerate(a))


def near_kernel(r, ell: float, eps: float, a: np.ndarray, der: bool, kernel: int = MATERN12):
    """K_NE(r) = kappa(r) - p(r) for r < eps, 0 beyond."""
    r = np.asarray(r, dtype=np.float64)
    return np.where(r < eps, _kappa(r, ell, der, kernel) - even_poly(a, r / eps), 0.0)


def regularised_samples(ell: float, T: float, L: float, n: int, d: int, der: bool,
                        kernel: int = MATERN12) -> np.ndarray:
    """K_R on the torus points T j / M, j in I_M^d (array index j + M/2)."""
    M = SAMPLE_FACTOR * n
    eps = near_radius(T, n)
    a = taylor_even_poly(ell, eps, der, kernel=kernel)
    x = modes(M).astype(np.float64) * (T / M)
    g = np.meshgrid(*([x] * d), indexing="ij")
    rf = np.sqrt(sum(fold_sq(gi, L, T) for gi in g))
    r0 = np.sqrt(sum(gi * gi for gi in g))  # |x_i| <= T/2: the nearest image
    return _kappa(rf, ell, der, kernel) - near_kernel(r0, ell, eps, a, der, kernel)


def coeffs_regularised(ell: float, T: float, L: float, n: int, d: int, der: bool = False,
                       kernel: int = MATERN12) -> np.ndarray:
    """c_k = M^-d sum_j K_R(T j / M) e^{-2 pi i j.k / M}, k in I_n^d (axes k_i + n/2)."""
    M = SAMPLE_FACTOR * n
    s = regularised_samples(ell, T, L, n, d, der, kernel)
    c = np.fft.fftshift(np.fft.fftn(np.fft.ifftshift(s))).real / M ** d
    sl = slice(M // 2 - n // 2, M // 2 + n // 2)
    return c[(sl,) * d].copy()


def near_field_sum(Xw: np.ndarray, V: np.ndarray, ell: float, eps: float, der: bool,
                   kernel: int = MATERN12) -> np.ndarray:
    """sum over j with |x_i - x_j| < eps of K_NE(|x_i - x_j|) V_j (all i), by blocks of rows."""
    a = taylor_even_poly(ell, eps, der, kernel=kernel)
    N = Xw.shape[0]
    out = np.zeros((N, V.shape[1]))
    for s in range(0, N, 1024):
        e = min(N, s + 1024)
        D = Xw[s:e, None, :] - Xw[None, :, :]
        r = np.sqrt((D * D).sum(-1))
        out[s:e] = near_kernel(r, ell, eps, a, der, kernel) @ V
    return out


def nearfield_fast_sum_oracle(X: np.ndarray, windows: Sequence[Sequence[int]], ell, sigma, V: np.ndarray,
                              n: int, want_derivs: bool = False, kernel: int = MATERN12):
    """Y = sum_w sigma_w^2 K_w V with each K_w V = trigonometric sum (regularised
    coefficients, exact NDFTs) + near-field sum; also sigma_w^2 / l_w K_der,w V
    and 2 sigma_w K_w V.  Returns Y (N, R) [, dY_dl (P, N, R), dY_ds (P, N, R)]."""
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
        Lf = fold_width(L, ell[w])
        T = near_period(L, ell[w])
        eps = near_radius(T, n)
        xt = (Xw - c) / T
        ck = coeffs_regularised(ell[w], T, Lf, n, d, kernel=kernel)
        kv = np.stack([trig_sum(ck, xt, V[:, r]) for r in range(R)], axis=1)
        kv += near_field_sum(Xw, V, ell[w], eps, False, kernel)
        Y += sigma[w] ** 2 * kv
        ds[w] = 2.0 * sigma[w] * kv
        if want_derivs:
            cd = coeffs_regularised(ell[w], T, Lf, n, d, der=True, kernel=kernel)
            kd = np.stack([trig_sum(cd, xt, V[:, r]) for r in range(R)], axis=1)
            kd += near_field_sum(Xw, V, ell[w], eps, True, kernel)
            dl[w] = sigma[w] ** 2 * der_scale(kernel, ell[w]) * kd
    if want_derivs:
        return Y, dl, ds
    return Y
