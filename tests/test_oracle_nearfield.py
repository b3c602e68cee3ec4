"""Pins of the near-field corrected Matern-1/2 oracle against facts that do not
come from the oracle itself: the direct O(N^2) sum, the kernel it must
reproduce pair by pair, the order of the Taylor joint, and the properties of
the folded square that make the periodic kernel image-free."""
import numpy as np
import pytest

from oracle import fourier as F
from oracle import nearfield as NF
from oracle.direct import oracle_direct


def test_fold_square_properties():
    L, T = 0.5, NF.near_period(0.5, 0.1)
    x = np.linspace(-L, L, 1001)
    assert np.max(np.abs(NF.fold_sq(x, L, T) - x * x)) < 1e-15                      # x^2 on [-L, L]
    y = np.random.default_rng(0).uniform(-3 * T, 3 * T, 2000)
    s = NF.fold_sq(y, L, T)
    np.testing.assert_allclose(NF.fold_sq(y + T, L, T), s, rtol=1e-13, atol=1e-13)   # periodic
    np.testing.assert_allclose(NF.fold_sq(-y, L, T), s, rtol=1e-13, atol=1e-13)      # even
    g = np.linspace(L, T - L, 999)
    assert np.all(NF.fold_sq(g, L, T) >= L * L * (1 - 1e-12))                       # no shorter distance
    # smooth at the joints: one-sided difference quotients agree up to O(h)
    for x0 in (L, T - L):
        h = 1e-5
        left = (NF.fold_sq(x0, L, T) - NF.fold_sq(x0 - h, L, T)) / h
        right = (NF.fold_sq(x0 + h, L, T) - NF.fold_sq(x0, L, T)) / h
        assert abs(left - right) < 1e-3
    t = np.linspace(0, 1, 101)
    np.testing.assert_allclose(NF.smoothstep7(t) + NF.smoothstep7(1 - t), 1.0, atol=1e-14)


@pytest.mark.parametrize("der", [False, True])
@pytest.mark.parametrize("ell", [0.05, 0.2])
def test_taylor_joint_order(der, ell):
    """p - kappa vanishes to order q + 1 at eps: halving the distance to eps
    divides the gap by about 2^(q+1).  A wrong derivative (sign, factor) at any
    order s <= q leaves a term of order s and fails the ratio."""
    eps = NF.near_radius(NF.near_period(0.5, ell), 64)
    a = NF.taylor_even_poly(ell, eps, der)
    kap = (lambda r: r / ell * np.exp(-r / ell)) if der else (lambda r: np.exp(-r / ell))
    gap = lambda dl: abs(NF.even_poly(a, 1 - dl) - kap(eps * (1 - dl)))  # noqa: E731
    g1, g2 = gap(0.04), gap(0.02)
    ratio = g1 / g2
    assert 0.6 * 2 ** (NF.NEAR_Q + 1) < ratio < 1.5 * 2 ** (NF.NEAR_Q + 1), ratio
    assert NF.near_kernel(np.array([eps, 2 * eps]), ell, eps, a, der).tolist() == [0.0, 0.0]


@pytest.mark.parametrize("d,ell", [(1, 0.05), (2, 0.1), (3, 0.2)])
def test_regularised_series_reproduces_kernel(d, ell):
    """Pairwise: the regularised Fourier series plus the near-field kernel
    reproduces kappa(|x|) for differences x in [-L, L]^d (every pair of a
    window), to within 2e-5 of kappa(0); the plain truncated series of the
    periodised kernel does not (error > 1e-3)."""
    n, L = 64, 0.5
    T = NF.near_period(L, ell)
    eps = NF.near_radius(T, n)
    c = NF.coeffs_regularised(ell, T, L, n, d)
    a = NF.taylor_even_poly(ell, eps, False)
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.uniform(-L, L, (300, d)), rng.uniform(-2 * eps, 2 * eps, (300, d))])
    k = F.modes(n)
    K = np.meshgrid(*([k] * d), indexing="ij")
    ph = sum(np.multiply.outer(x[:, i], Ki) for i, Ki in enumerate(K)) * (2 * np.pi / T)
    series = (np.cos(ph) * c).reshape(len(x), -1).sum(1)
    r = np.sqrt((x * x).sum(1))
    approx = series + NF.near_kernel(r, ell, eps, a, False)
    assert np.max(np.abs(approx - np.exp(-r / ell))) < 2e-5
    Ta = F.torus_period_auto(F.MATERN12, L, ell, n)
    ca = F.coeffs_analytic(F.MATERN12, ell, Ta, n, d)
    ph = sum(np.multiply.outer(x[:, i], Ki) for i, Ki in enumerate(K)) * (2 * np.pi / Ta)
    plain = (np.cos(ph) * ca).reshape(len(x), -1).sum(1)
    assert np.max(np.abs(plain - np.exp(-r / ell))) > 1e-3


@pytest.mark.parametrize("wins,ell", [([[0], [1, 2]], 0.05), ([[0, 1, 2]], 0.2)])
def test_nearfield_fast_sum_matches_direct(wins, ell):
    """The whole corrected product against the direct sum (FP64, all rows):
    K V, (dK/dl) V and (dK/dsigma) V within 2e-5."""
    rng = np.random.default_rng(5)
    N = 300
    X = rng.uniform(-0.25, 0.25, (N, 3))
    V = rng.standard_normal((N, 2))
    P = len(wins)
    sig = [1.0, 0.7][:P]
    Y, dl, ds = NF.nearfield_fast_sum_oracle(X, wins, [ell] * P, sig, V, 64, want_derivs=True)
    Yd, dld, dsd = oracle_direct(X, wins, F.MATERN12, [ell] * P, sig, V, want_derivs=True)

    def rel(a, b):
        return np.linalg.norm(a - b) / np.linalg.norm(b)
    assert rel(Y, Yd) < 2e-5
    for w in range(P):
        assert rel(dl[w], dld[w]) < 2e-5
        assert rel(ds[w], dsd[w]) < 2e-5
    # and the plain scheme is far off on the same problem
    Yp = F.fast_sum_oracle(X, wins, F.MATERN12, [ell] * P, sig, V, 64)
    assert rel(Yp, Yd) > 1e-3


@pytest.mark.parametrize("d", [1, 3])
def test_coincident_points(d):
    """All points equal (L = 0): every kernel value is kappa(0) = 1, so
    K v = (sum_j v_j) for every row and the derivative kernel (r/l) e^{-r/l}
    vanishes, up to the method's error at n = 64 (measured 3e-7 and 8e-7 of
    sum |v| for d = 1, 3; 5e-6 for the derivative kernel)."""
    X = np.tile(np.array([[0.1, -0.05, 0.2]])[:, :d], (4, 1))
    V = np.array([[1.0], [-0.5], [2.0], [0.25]])
    Y, dl, _ = NF.nearfield_fast_sum_oracle(X, [list(range(d))], [0.1], [1.0], V, 64, want_derivs=True)
    np.testing.assert_allclose(Y, np.full((4, 1), V.sum()), rtol=0, atol=2e-6 * abs(V).sum())
    assert np.abs(dl).max() < 1e-5 * abs(V).sum()
