"""Pins of the Matern-3/2 parts of the oracle ((1 + a r) e^{-a r}, a = sqrt(3)/l,
the further kernel that the kernel-extension subsection names).

Independent of the formulas under test: numerical quadrature of the Fourier
integrals in d = 1, 2, 3, the Matern spectral density with smoothness 3/2
written through Gamma functions, finite differences in l, the direct sum, and
the order of the Taylor joint of the near-field polynomial."""
import math

import numpy as np
import pytest
from scipy import integrate, special

from oracle import fourier as F
from oracle import nearfield as NF
from oracle.direct import oracle_direct

M3 = F.MATERN32


def _kappa(r, ell):
    """The kernel value through the direct-sum oracle (pinned against the
    Bessel-function form of the Matern family in test_oracle_pins)."""
    X = np.array([[0.0], [r]])
    return float(oracle_direct(X, [[0]], M3, ell, 1.0, np.array([[0.0], [1.0]]))[0, 0])


def _radial_ft(f, xi, d, rmax):
    """int_{R^d} f(|x|) e^{-2 pi i xi.x} dx for a radial f by 1-D quadrature."""
    if d == 1:
        if xi == 0:
            return 2 * integrate.quad(f, 0, rmax, limit=400, epsabs=1e-16)[0]
        return 2 * integrate.quad(f, 0, rmax, weight="cos", wvar=2 * math.pi * xi, limit=400)[0]
    if d == 2:
        return integrate.quad(lambda r: 2 * math.pi * r * special.j0(2 * math.pi * xi * r) * f(r), 0, rmax,
                              limit=4000, epsabs=1e-15)[0]
    if xi == 0:
        return integrate.quad(lambda r: 4 * math.pi * r * r * f(r), 0, rmax, limit=400, epsabs=1e-16)[0]
    return 2.0 / xi * integrate.quad(lambda r: r * f(r), 0, rmax, weight="sin", wvar=2 * math.pi * xi,
                                     limit=400)[0]


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("ell,xi", [(0.1, 0.0), (0.1, 2.0), (0.05, 9.0), (0.3, 1.3)])
def test_ft_matches_quadrature(d, ell, xi):
    a = math.sqrt(3.0) / ell
    v = _radial_ft(lambda r: (1 + a * r) * math.exp(-a * r), xi, d, 80 * ell)
    assert F.kernel_ft(M3, xi * xi, ell, d) == pytest.approx(v, rel=2e-7)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_ft_is_the_matern_spectral_density(d):
    """Matern family, smoothness nu: S(xi) = 2^d pi^(d/2) Gamma(nu + d/2) (2 nu)^nu
    / (Gamma(nu) l^(2 nu)) (2 nu / l^2 + 4 pi^2 |xi|^2)^-(nu + d/2), at nu = 3/2."""
    nu, ell = 1.5, 0.13
    xi = np.linspace(0.0, 20.0, 41)
    S = (2 ** d * math.pi ** (d / 2) * special.gamma(nu + d / 2) * (2 * nu) ** nu / (special.gamma(nu) * ell ** (2 * nu))
         * (2 * nu / ell ** 2 + 4 * math.pi ** 2 * xi ** 2) ** (-(nu + d / 2)))
    np.testing.assert_allclose(F.kernel_ft(M3, xi * xi, ell, d), S, rtol=1e-13)


def test_value_at_zero_matches_the_ft_integral():
    """kappa(0) = 1 = int S(xi) dxi (inverse transform at the origin, d = 1, 3)."""
    ell = 0.1
    for d in (1, 3):
        if d == 1:
            v = 2 * integrate.quad(lambda x: F.kernel_ft(M3, x * x, ell, 1), 0, np.inf, limit=400)[0]
        else:
            v = integrate.quad(lambda x: 4 * math.pi * x * x * F.kernel_ft(M3, x * x, ell, 3), 0, np.inf,
                               limit=400)[0]
        assert v == pytest.approx(1.0, rel=1e-9)


@pytest.mark.parametrize("d", [1, 3])
@pytest.mark.parametrize("xi", [0.0, 2.5, 7.0])
def test_derivative_ft_matches_quadrature(d, xi):
    """The derivative kernel (a r)^2 e^{-a r}: transform by quadrature."""
    ell = 0.08
    a = math.sqrt(3.0) / ell
    v = _radial_ft(lambda r: (a * r) ** 2 * math.exp(-a * r), xi, d, 80 * ell)
    assert F.kernel_der_ft(M3, xi * xi, ell, d) == pytest.approx(v, rel=2e-7, abs=1e-14)


def test_derivative_kernel_is_l_times_the_l_derivative():
    """K_der = l dK/dl: direct sums against central differences in l, and the
    analytic coefficients of the derivative kernel against l d/dl of the kernel's."""
    rng = np.random.default_rng(50)
    X = rng.uniform(-0.25, 0.25, (120, 3))
    v = rng.standard_normal((120, 1))
    ell, h = 0.12, 1e-6
    _, dl, _ = oracle_direct(X, [[0, 1, 2]], M3, ell, 1.0, v, want_derivs=True)
    fd = (oracle_direct(X, [[0, 1, 2]], M3, ell + h, 1.0, v) - oracle_direct(X, [[0, 1, 2]], M3, ell - h, 1.0, v)) / (2 * h)
    assert np.linalg.norm(fd - dl[0]) <= 1e-7 * np.linalg.norm(dl[0])
    T, n = 1.4, 32
    for d in (1, 2, 3):
        def cd(hl):
            return (F.coeffs_analytic(M3, ell + hl, T, n, d) - F.coeffs_analytic(M3, ell - hl, T, n, d)) / (2 * hl)
        cfd = (4.0 * cd(5e-5) - cd(1e-4)) / 3.0  # Richardson: O(h^4)
        np.testing.assert_allclose(F.coeffs_analytic(M3, ell, T, n, d, der=True), ell * cfd, rtol=1e-8,
                                   atol=1e-12 * np.abs(cfd).max())


def test_sampled_coefficients_satisfy_aliasing_formula():
    """Lemma 1 (d = 1): the discrete coefficients from n kernel samples equal
    the sum of the analytic coefficients over all aliases k + n r.  The aliases
    decay like |k + n r|^-4, so 4000 of them leave a tail below 1e-12; the
    kernel's value at the torus edge (T = 2, l = 0.05) is 3e-14."""
    ell, T, n = 0.05, 2.0, 64
    cs = F.coeffs_sampled(M3, ell, T, n, 1)
    k = F.modes(n).astype(np.float64)
    r = np.arange(-2000, 2001, dtype=np.float64)
    alias = F.kernel_ft(M3, ((k[:, None] + n * r[None, :]) / T) ** 2, ell, 1).sum(axis=1) / T
    np.testing.assert_allclose(cs, alias, rtol=0, atol=1e-12 * cs.max())
    assert np.max(np.abs(cs - F.coeffs_analytic(M3, ell, T, n, 1))) > 1e-3 * cs.max()  # aliases matter here


def test_trig_sum_converges_to_the_direct_sum():
    """The truncated series of the Matern-3/2 kernel converges algebraically:
    doubling n cuts the error by about 2^3."""
    rng = np.random.default_rng(51)
    X = rng.uniform(-0.25, 0.25, (300, 3))
    v = rng.standard_normal((300, 1))
    y = oracle_direct(X, [[0, 1, 2]], M3, 0.1, 1.0, v)
    err = []
    for n in (16, 32):
        T = F.torus_period_auto(M3, 0.5, 0.1, n)
        yt = F.fast_sum_oracle(X, [[0, 1, 2]], M3, 0.1, 1.0, v, n, periods=[T])
        err.append(np.linalg.norm(yt - y) / np.linalg.norm(y))
    assert err[1] < err[0] / 4 and err[1] < 2e-2, err


# ------------------------------------------------------------------ near field


@pytest.mark.parametrize("der", [False, True])
@pytest.mark.parametrize("ell", [0.05, 0.2])
def test_taylor_joint_order(der, ell):
    """p - kappa vanishes to order q + 1 at eps (ratio test as for Matern-1/2),
    with the kernel evaluated through the direct-sum oracle."""
    eps = NF.near_radius(NF.near_period(0.5, ell), 64)
    a = NF.taylor_even_poly(ell, eps, der, kernel=M3)

    def kap(r):
        if der:  # l dkappa/dl from the oracle's analytic l-derivative
            X = np.array([[0.0], [r]])
            _, dl, _ = oracle_direct(X, [[0]], M3, ell, 1.0, np.array([[0.0], [1.0]]), want_derivs=True)
            return ell * float(dl[0, 0, 0])
        return _kappa(r, ell)
    gap = lambda dl: abs(NF.even_poly(a, 1 - dl) - kap(eps * (1 - dl)))  # noqa: E731
    ratio = gap(0.08) / gap(0.04)
    assert 0.5 * 2 ** (NF.NEAR_Q + 1) < ratio < 1.6 * 2 ** (NF.NEAR_Q + 1), ratio


@pytest.mark.parametrize("d,ell", [(1, 0.05), (2, 0.1), (3, 0.2)])
def test_regularised_series_reproduces_kernel(d, ell):
    """Pairwise: the regularised series plus the near-field kernel reproduces
    kappa(|x|) on every difference of a window within 1e-5 of kappa(0); the
    plain truncated series of the periodised kernel misses by more."""
    n, L = 64, 0.5
    T = NF.near_period(L, ell)
    eps = NF.near_radius(T, n)
    c = NF.coeffs_regularised(ell, T, L, n, d, kernel=M3)
    a = NF.taylor_even_poly(ell, eps, False, kernel=M3)
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.uniform(-L, L, (300, d)), rng.uniform(-2 * eps, 2 * eps, (300, d))])
    k = F.modes(n)
    K = np.meshgrid(*([k] * d), indexing="ij")
    ph = sum(np.multiply.outer(x[:, i], Ki) for i, Ki in enumerate(K)) * (2 * np.pi / T)
    series = (np.cos(ph) * c).reshape(len(x), -1).sum(1)
    r = np.sqrt((x * x).sum(1))
    exact = F.kernel_value(M3, r * r, ell)
    approx = series + NF.near_kernel(r, ell, eps, a, False, kernel=M3)
    assert np.max(np.abs(approx - exact)) < 1e-5
    Ta = F.torus_period_auto(M3, L, ell, n)
    ca = F.coeffs_analytic(M3, ell, Ta, n, d)
    ph = sum(np.multiply.outer(x[:, i], Ki) for i, Ki in enumerate(K)) * (2 * np.pi / Ta)
    plain = (np.cos(ph) * ca).reshape(len(x), -1).sum(1)
    assert np.max(np.abs(plain - exact)) > 10 * np.max(np.abs(approx - exact))


@pytest.mark.parametrize("wins,ell", [([[0], [1, 2]], 0.05), ([[0, 1, 2]], 0.2)])
def test_nearfield_fast_sum_matches_direct(wins, ell):
    """The corrected product against the direct sum (FP64, all rows): K V,
    (dK/dl) V and (dK/dsigma) V within 1e-5; the plain series is far off."""
    rng = np.random.default_rng(5)
    N = 300
    X = rng.uniform(-0.25, 0.25, (N, 3))
    V = rng.standard_normal((N, 2))
    P = len(wins)
    sig = [1.0, 0.7][:P]
    Y, dl, ds = NF.nearfield_fast_sum_oracle(X, wins, [ell] * P, sig, V, 64, want_derivs=True, kernel=M3)
    Yd, dld, dsd = oracle_direct(X, wins, M3, [ell] * P, sig, V, want_derivs=True)

    def rel(a, b):
        return np.linalg.norm(a - b) / np.linalg.norm(b)
    assert rel(Y, Yd) < 1e-5
    for w in range(P):
        assert rel(dl[w], dld[w]) < 1e-5
        assert rel(ds[w], dsd[w]) < 1e-5
    Yp = F.fast_sum_oracle(X, wins, M3, [ell] * P, sig, V, 64)
    assert rel(Yp, Yd) > 10 * rel(Y, Yd)
