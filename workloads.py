"""Seeded synthetic inputs shaped like the paper's regression workloads.

This module only draws random numbers and arranges them into problem
descriptions.  It holds none of the method's arithmetic, so both the
independent CPU oracle and the GPU library can be fed from it.

The paper evaluates on tabular regression data sets (z-scored features,
then scaled into [-1/4, 1/4] per feature; "Scaling the Data" section and
the experimental set-up of the numerical-results section).  Those data sets
are not available here; i.i.d. Gaussian or uniform features, min-max scaled
per feature to [-1/4, 1/4], stand in for them with the same scaling.

Every generator uses NumPy's PCG64 (``default_rng(seed)``) and draws in the
fixed order: features X, then right-hand sides V, then per-problem
parameters.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

GAUSSIAN = 1
MATERN12 = 3
MATERN32 = 5


@dataclasses.dataclass
class Problem:
    """One additive-kernel matvec problem (points, windows, parameters, RHS)."""

    name: str
    X: np.ndarray            # (N, D) float64, row-major
    V: np.ndarray            # (N, R) float64
    windows: List[List[int]]  # feature indices of each window, d_w <= 3
    ell: np.ndarray          # (P,) length scales
    sigma: np.ndarray        # (P,) per-window signal amplitudes sigma_w
    kernel: int = GAUSSIAN
    n: int = 64              # Fourier bandwidth per dimension
    m: int = 6               # window half-width in oversampled grid cells
    oversampling: float = 2.0

    @property
    def N(self) -> int:
        return self.X.shape[0]

    @property
    def R(self) -> int:
        return self.V.shape[1]

    @property
    def P(self) -> int:
        return len(self.windows)

    def win_arrays(self):
        off = [0]
        feat: List[int] = []
        for w in self.windows:
            feat.extend(int(f) for f in w)
            off.append(len(feat))
        return np.asarray(off, dtype=np.int32), np.asarray(feat, dtype=np.int32)


def minmax_quarter(Z: np.ndarray) -> np.ndarray:
    """Affinely map every column of Z onto [-1/4, 1/4] (min -> -1/4, max -> 1/4)."""
    lo = Z.min(axis=0, keepdims=True)
    hi = Z.max(axis=0, keepdims=True)
    span = np.where(hi > lo, hi - lo, 1.0)
    return (Z - lo) / span * 0.5 - 0.25


def consecutive_windows(D: int, d: int) -> List[List[int]]:
    return [list(range(s, min(s + d, D))) for s in range(0, D, d)]


def single_window_c1(N: int = 2000, seed: int = 17341, m: int = 4) -> Problem:
    """One d=3 window, uniform features, Gaussian l=0.1, n=32, sigma=2."""
    rng = np.random.default_rng(seed)
    X = minmax_quarter(rng.uniform(0.0, 1.0, size=(N, 3)))
    V = rng.standard_normal(size=(N, 1))
    return Problem("single_window_d3_N%d_n32_m%d" % (N, m), X, V, [[0, 1, 2]],
                   np.array([0.1]), np.array([1.0]), GAUSSIAN, n=32, m=m)


def additive_c2(N: int = 100000, seed: int = 17342, R: int = 1,
                kernel: int = GAUSSIAN) -> Problem:
    """Three d=3 windows over 9 Gaussian features, l = (0.05, 0.1, 0.2), n=64, m=6."""
    rng = np.random.default_rng(seed)
    X = minmax_quarter(rng.standard_normal(size=(N, 9)))
    V = rng.standard_normal(size=(N, R))
    return Problem("additive_3xd3_N%d" % N, X, V, consecutive_windows(9, 3),
                   np.array([0.05, 0.1, 0.2]), np.ones(3), kernel, n=64, m=6)


def derivative_c3(N: int = 100000, seed: int = 17343,
                  kernel: int = GAUSSIAN) -> Problem:
    """Same shape as the additive case; used with K, dK/dl, dK/dsigma and autograd."""
    p = additive_c2(N=N, seed=seed, R=1, kernel=kernel)
    p.name = "derivative_3xd3_N%d_%s" % (N, "gauss" if kernel == GAUSSIAN else "matern12")
    return p


def large_c5(N: int = 1000000, seed: int = 17345, R: int = 16) -> Problem:
    """Five d=3 windows over 15 Gaussian features, l=0.1, 16 RHS, n=64, m=6."""
    rng = np.random.default_rng(seed)
    X = minmax_quarter(rng.standard_normal(size=(N, 15)))
    V = rng.standard_normal(size=(N, R))
    return Problem("large_5xd3_N%d_R%d" % (N, R), X, V, consecutive_windows(15, 3),
                   np.full(5, 0.1), np.ones(5), GAUSSIAN, n=64, m=6)


def batched_c4(n_problems: int = 64, seed: int = 17344, R: int = 8,
               n_min: int = 5000, n_max: int = 200000) -> List[Problem]:
    """Uneven independent problems: N log-uniform, 1-5 windows of mixed d in {1,2,3}.

    Features are i.i.d. uniform in [-1/4, 1/4]; windows take consecutive,
    disjoint feature blocks; l_w ~ U(0.05, 0.3); sigma_w = 1; m = 4.  The
    bandwidth n is left at 32 here and chosen per window by the caller.
    """
    rng = np.random.default_rng(seed)
    # draw order: sizes and window shapes first fix D, then X, then V, then params
    sizes = np.round(np.exp(rng.uniform(math.log(n_min), math.log(n_max), size=n_problems))).astype(int)
    shapes = []
    for _ in range(n_problems):
        W = int(rng.integers(1, 6))
        shapes.append([int(d) for d in rng.integers(1, 4, size=W)])
    probs = []
    Xs = []
    for p in range(n_problems):
        D = sum(shapes[p])
        Xs.append(rng.uniform(-0.25, 0.25, size=(sizes[p], D)))
    Vs = [rng.standard_normal(size=(sizes[p], R)) for p in range(n_problems)]
    for p in range(n_problems):
        wins, s = [], 0
        for d in shapes[p]:
            wins.append(list(range(s, s + d)))
            s += d
        ell = rng.uniform(0.05, 0.3, size=len(wins))
        probs.append(Problem("batch%02d_N%d" % (p, sizes[p]), Xs[p], Vs[p], wins, ell,
                             np.ones(len(wins)), GAUSSIAN, n=32, m=4))
    return probs


def small_problem(N: int, D: int, windows: List[List[int]], seed: int, R: int = 1,
                  ell: Optional[List[float]] = None, sigma: Optional[List[float]] = None,
                  kernel: int = GAUSSIAN, n: int = 32, m: int = 6,
                  dist: str = "uniform") -> Problem:
    """Small seeded problem for parity and edge-case tests."""
    rng = np.random.default_rng(seed)
    if dist == "uniform":
        X = rng.uniform(-0.25, 0.25, size=(N, D))
    else:
        X = minmax_quarter(rng.standard_normal(size=(N, D))) if N > 1 else np.zeros((N, D))
    V = rng.standard_normal(size=(N, R))
    P = len(windows)
    ell_a = np.asarray(ell if ell is not None else rng.uniform(0.08, 0.3, size=P), dtype=np.float64)
    sig_a = np.asarray(sigma if sigma is not None else rng.uniform(0.5, 1.5, size=P), dtype=np.float64)
    return Problem("small_N%d_D%d_s%d" % (N, D, seed), X, V, windows, ell_a, sig_a, kernel, n=n, m=m)


def derivative_c3_rhs(N: int = 100000, R: int = 8, seed: int = 17346) -> np.ndarray:
    """R right-hand sides for the derivative workload: column 0 is that
    workload's own v (seed 17343), the others N(0,1) from ``seed``."""
    v0 = derivative_c3(N=N).V
    if R == 1:
        return v0.copy()
    rng = np.random.default_rng(seed)
    return np.concatenate([v0, rng.standard_normal(size=(N, R - 1))], axis=1)


def large_d1(N: int = 1000000, seed: int = 17347, R: int = 16, D: int = 15) -> Problem:
    """The large workload's points with every feature its own d = 1 window:
    N(0,1) features min-max scaled, l = 0.1, sigma_w = 1, n = 64, m = 6 (12 taps
    per point and window: the spread and interpolation move more bytes than
    they compute on)."""
    rng = np.random.default_rng(seed)
    X = minmax_quarter(rng.standard_normal(size=(N, D)))
    V = rng.standard_normal(size=(N, R))
    return Problem("large_%dxd1_N%d_R%d" % (D, N, R), X, V, consecutive_windows(D, 1),
                   np.full(D, 0.1), np.ones(D), GAUSSIAN, n=64, m=6)
