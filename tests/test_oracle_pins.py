"""Pins of the CPU oracle against facts the paper and the mathematics fix.

None of these re-types an oracle formula and compares it with itself: each
check is an invariant (diagonal, symmetry, linearity, permutation and
rotation invariance, separability), an independent library routine
(quadrature, Faddeeva function, exactly rounded summation), a closed-form
structural property (the Markov property of the 1-D Matern-1/2 kernel),
finite differences, or an inequality the paper proves (Theorems 1-2).
"""
import math

import numpy as np
import pytest
from scipy import integrate, special

from oracle import fourier as F
from oracle.direct import oracle_direct, oracle_vjp

G, M, M3 = F.GAUSSIAN, F.MATERN12, F.MATERN32


def _pts(N, D, seed):
    return np.random.default_rng(seed).uniform(-0.25, 0.25, size=(N, D))


def _kmat(X, windows, kernel, ell, sigma):
    """Full kernel matrix assembled column by column from oracle matvecs with unit vectors."""
    N = X.shape[0]
    return oracle_direct(X, windows, kernel, ell, sigma, np.eye(N))


# ---------------------------------------------------------------- direct sums


@pytest.mark.parametrize("kernel", [G, M, M3])
def test_diagonal_is_sum_of_sigma_squared(kernel):
    X = _pts(40, 7, 1)
    wins = [[0, 1, 2], [3, 4], [5], [6, 0]]
    sig = [0.7, 1.3, 0.4, 2.0]
    K = _kmat(X, wins, kernel, [0.1, 0.2, 0.05, 0.3], sig)
    np.testing.assert_allclose(np.diag(K), sum(s * s for s in sig), rtol=1e-15)


@pytest.mark.parametrize("kernel", [G, M, M3])
def test_symmetry_and_linearity(kernel):
    X = _pts(200, 6, 2)
    wins = [[0, 1, 2], [3, 4, 5]]
    rng = np.random.default_rng(3)
    u, v = rng.standard_normal((200, 1)), rng.standard_normal((200, 1))
    Ku = oracle_direct(X, wins, kernel, [0.08, 0.15], [1.0, 0.5], u)
    Kv = oracle_direct(X, wins, kernel, [0.08, 0.15], [1.0, 0.5], v)
    a, b = float((u.T @ Kv)[0, 0]), float((v.T @ Ku)[0, 0])
    assert abs(a - b) < 1e-12 * abs(a)
    Kuv = oracle_direct(X, wins, kernel, [0.08, 0.15], [1.0, 0.5], 2.0 * u - 3.0 * v)
    np.testing.assert_allclose(Kuv, 2.0 * Ku - 3.0 * Kv, rtol=1e-12, atol=1e-12)


def test_permutation_equivariance():
    X = _pts(150, 3, 4)
    v = np.random.default_rng(5).standard_normal((150, 2))
    p = np.random.default_rng(6).permutation(150)
    y = oracle_direct(X, [[0, 1, 2]], G, 0.1, 1.0, v)
    yp = oracle_direct(X[p], [[0, 1, 2]], G, 0.1, 1.0, v[p])
    np.testing.assert_allclose(yp, y[p], rtol=1e-13, atol=1e-13)


def test_additive_split_over_windows():
    X = _pts(120, 5, 7)
    v = np.random.default_rng(8).standard_normal((120, 3))
    wins, ell, sig = [[0, 1], [2, 3, 4], [1, 3]], [0.1, 0.2, 0.05], [0.3, 1.1, 0.9]
    y = oracle_direct(X, wins, G, ell, sig, v)
    parts = sum(oracle_direct(X, [w], G, [l], [s], v) for w, l, s in zip(wins, ell, sig))
    np.testing.assert_allclose(y, parts, rtol=1e-13, atol=1e-13)


def test_gaussian_is_product_of_1d_kernels():
    """The d-th order ANOVA kernel with Gaussian bases is the SE kernel (Sec. 2)."""
    X = _pts(50, 3, 9)
    K3 = _kmat(X, [[0, 1, 2]], G, [0.12], [1.0])
    K1 = [_kmat(X, [[a]], G, [0.12], [1.0]) for a in range(3)]
    np.testing.assert_allclose(K3, K1[0] * K1[1] * K1[2], rtol=1e-13, atol=1e-300)


def test_two_point_special_values():
    ell = 0.1
    X = np.array([[0.0, 0.0, 0.0], [3 * ell, 4 * ell, 0.0]])  # distance 5 l
    Kg = _kmat(X, [[0, 1, 2]], G, [ell], [1.0])
    Km = _kmat(X, [[0, 1, 2]], M, [ell], [1.0])
    assert Kg[0, 1] == pytest.approx(math.exp(-12.5), rel=1e-14)
    assert Km[0, 1] == pytest.approx(math.exp(-5.0), rel=1e-14)


@pytest.mark.parametrize("kernel", [G, M, M3])
def test_rotation_invariance(kernel):
    """The kernels depend on the Euclidean distance only."""
    X = _pts(80, 3, 10)
    Q, _ = np.linalg.qr(np.random.default_rng(11).standard_normal((3, 3)))
    v = np.random.default_rng(12).standard_normal((80, 1))
    y = oracle_direct(X, [[0, 1, 2]], kernel, 0.07, 1.0, v)
    yr = oracle_direct(X @ Q.T, [[0, 1, 2]], kernel, 0.07, 1.0, v)
    np.testing.assert_allclose(yr, y, rtol=1e-12, atol=1e-13)


def test_matern_1d_has_tridiagonal_inverse():
    """exp(-|x-y|/l) is the Ornstein-Uhlenbeck covariance: for sorted 1-D points its
    inverse is tridiagonal (Markov property).  A Gaussian fails this."""
    x = np.sort(np.random.default_rng(13).uniform(-0.25, 0.25, 25))[:, None]
    Ki = np.linalg.inv(_kmat(x, [[0]], M, [0.05], [1.0]))
    off = Ki - np.triu(np.tril(Ki, 1), -1)
    assert np.max(np.abs(off)) < 1e-8 * np.max(np.abs(Ki))
    Kgi = np.linalg.inv(_kmat(x, [[0]], G, [0.05], [1.0]) + 1e-3 * np.eye(25))
    offg = Kgi - np.triu(np.tril(Kgi, 1), -1)
    assert np.max(np.abs(offg)) > 1e-3 * np.max(np.abs(Kgi))


@pytest.mark.parametrize("kernel", [G, M, M3])
def test_derivatives_match_central_differences(kernel):
    X = _pts(300, 6, 14)
    wins = [[0, 1, 2], [3, 4, 5]]
    ell, sig = np.array([0.09, 0.2]), np.array([1.2, 0.8])
    v = np.random.default_rng(15).standard_normal((300, 2))
    _, dl, ds = oracle_direct(X, wins, kernel, ell, sig, v, want_derivs=True)
    h = 1e-6
    for w in range(2):
        e = np.zeros(2)
        e[w] = h
        fd_l = (oracle_direct(X, wins, kernel, ell + e, sig, v) - oracle_direct(X, wins, kernel, ell - e, sig, v)) / (2 * h)
        fd_s = (oracle_direct(X, wins, kernel, ell, sig + e, v) - oracle_direct(X, wins, kernel, ell, sig - e, v)) / (2 * h)
        assert np.linalg.norm(fd_l - dl[w]) <= 1e-7 * np.linalg.norm(dl[w])
        assert np.linalg.norm(fd_s - ds[w]) <= 1e-8 * np.linalg.norm(ds[w])


def test_sigma_derivative_identity():
    """dK/dsigma_f v = (2/sigma_f) K v for one shared sigma_f ("Implementing the NFFT approach")."""
    X = _pts(100, 6, 16)
    v = np.random.default_rng(17).standard_normal((100, 1))
    y, _, ds = oracle_direct(X, [[0, 1, 2], [3, 4, 5]], G, [0.1, 0.1], [0.7, 0.7], v, want_derivs=True)
    np.testing.assert_allclose(ds.sum(axis=0), 2.0 / 0.7 * y, rtol=1e-13)


def test_vjp_matches_finite_differences():
    X = _pts(150, 3, 18)
    rng = np.random.default_rng(19)
    v, g = rng.standard_normal((150, 2)), rng.standard_normal((150, 2))
    ell, sig = np.array([0.11]), np.array([0.9])
    gV, gl, gs = oracle_vjp(X, [[0, 1, 2]], G, ell, sig, v, g)

    def loss(l, s, vv):
        return float(np.sum(g * oracle_direct(X, [[0, 1, 2]], G, l, s, vv)))

    h = 1e-6
    assert (loss(ell + h, sig, v) - loss(ell - h, sig, v)) / (2 * h) == pytest.approx(gl[0], rel=1e-7)
    assert (loss(ell, sig + h, v) - loss(ell, sig - h, v)) / (2 * h) == pytest.approx(gs[0], rel=1e-8)
    dv = rng.standard_normal((150, 2))
    fd = (loss(ell, sig, v + h * dv) - loss(ell, sig, v - h * dv)) / (2 * h)
    assert fd == pytest.approx(float(np.sum(gV * dv)), rel=1e-7)


def test_compensated_sum_matches_exactly_rounded_sum():
    """Long sums agree with math.fsum (exactly rounded) to ~1e-15 relative."""
    N = 40000
    X = np.zeros((N, 1))  # all points coincide: every kernel value is exactly 1
    rng = np.random.default_rng(20)
    v = rng.standard_normal((N, 1)) * 10.0 ** rng.uniform(-4, 4, size=(N, 1))
    y = oracle_direct(X, [[0]], G, 0.1, 1.0, v, rows=np.array([0]))
    exact = math.fsum(v[:, 0])
    assert abs(y[0, 0] - exact) <= 4e-16 * np.sum(np.abs(v))


def test_row_subset_matches_full():
    X = _pts(500, 3, 21)
    v = np.random.default_rng(22).standard_normal((500, 3))
    rows = np.array([0, 17, 499, 250])
    y = oracle_direct(X, [[0, 1, 2]], M, 0.1, 1.3, v)
    ys = oracle_direct(X, [[0, 1, 2]], M, 0.1, 1.3, v, rows=rows)
    np.testing.assert_array_equal(ys, y[rows])


def test_rejects_bad_arguments():
    X = _pts(10, 3, 23)
    with pytest.raises(ValueError):
        oracle_direct(X, [[0, 1, 5]], G, 0.1, 1.0, np.ones((10, 1)))
    with pytest.raises(ValueError):
        oracle_direct(X, [[0]], G, -0.1, 1.0, np.ones((10, 1)))


def _matern_bessel(r, ell, nu):
    """The Matern kernel of smoothness nu in its general form
    2^(1-nu)/Gamma(nu) z^nu K_nu(z), z = sqrt(2 nu) r / l (SciPy's modified
    Bessel function of the second kind), with the limit 1 at r = 0."""
    r = np.asarray(r, dtype=np.float64)
    z = math.sqrt(2.0 * nu) * r / ell
    out = np.ones_like(z)
    nz = z > 0
    out[nz] = 2.0 ** (1.0 - nu) / special.gamma(nu) * z[nz] ** nu * special.kv(nu, z[nz])
    return out


def _explicit_matrix(Xw, kernel, ell):
    """N x N kernel matrix of one window assembled with NumPy from pairwise distances."""
    D = Xw[:, None, :] - Xw[None, :, :]
    r = np.sqrt((D * D).sum(-1))
    if kernel == G:
        return np.exp(-r * r / (2.0 * ell * ell))
    return _matern_bessel(r, ell, 0.5 if kernel == M else 1.5)


@pytest.mark.parametrize("kernel", [G, M, M3])
def test_direct_sums_equal_explicit_numpy_matrices(kernel):
    """N = 48: the direct sums equal products with kernel matrices built
    explicitly in NumPy (Matern kernels from the Bessel-function form of the
    Matern family, smoothness 1/2 and 3/2); the l-derivative matrices are
    Richardson-extrapolated central differences of those matrices."""
    X = _pts(48, 6, 40)
    wins = [[0, 1, 2], [3, 4], [5]]
    ell, sig = np.array([0.09, 0.17, 0.3]), np.array([1.1, 0.6, 0.8])
    V = np.random.default_rng(41).standard_normal((48, 3))
    Y, dl, ds = oracle_direct(X, wins, kernel, ell, sig, V, want_derivs=True)
    Ye = np.zeros_like(V)
    for w, feats in enumerate(wins):
        Kw = _explicit_matrix(X[:, feats], kernel, ell[w])
        Ye += sig[w] ** 2 * Kw @ V
        np.testing.assert_allclose(ds[w], 2.0 * sig[w] * Kw @ V, rtol=1e-12, atol=1e-13)
        h = 1e-3 * ell[w]

        def cd(step):
            return (_explicit_matrix(X[:, feats], kernel, ell[w] + step)
                    - _explicit_matrix(X[:, feats], kernel, ell[w] - step)) / (2 * step)
        dK = (4.0 * cd(h / 2) - cd(h)) / 3.0
        np.testing.assert_allclose(dl[w], sig[w] ** 2 * dK @ V, rtol=1e-8, atol=1e-9 * np.abs(dl[w]).max())
    np.testing.assert_allclose(Y, Ye, rtol=1e-12, atol=1e-13)


def test_matern32_two_point_values():
    """(1 + sqrt3 r/l) e^{-sqrt3 r/l} at r = 0 (1) and at r = l / sqrt3 (2/e),
    and its l-derivative vanishing at r = 0."""
    ell = 0.2
    X = np.array([[0.0, 0.0], [ell / math.sqrt(3.0), 0.0]])
    v = np.array([[0.0], [1.0]])
    y, dl, _ = oracle_direct(X, [[0, 1]], M3, ell, 1.0, v, want_derivs=True)
    assert y[0, 0] == pytest.approx(2.0 / math.e, rel=1e-15)
    assert y[1, 0] == pytest.approx(1.0, rel=1e-15)
    assert dl[0, 1, 0] == 0.0


# ---------------------------------------------------------------- Fourier side


@pytest.mark.parametrize("ell,xi", [(0.1, 0.0), (0.1, 3.0), (0.05, 7.5), (0.3, 1.2)])
def test_gaussian_ft_matches_quadrature(ell, xi):
    val, _ = integrate.quad(lambda x: math.exp(-x * x / (2 * ell * ell)) * math.cos(2 * math.pi * xi * x),
                            -40 * ell, 40 * ell, limit=400, epsabs=1e-15)
    assert F.kernel_ft(G, xi * xi, ell, 1) == pytest.approx(val, rel=1e-10, abs=1e-15)
    # tensor product in three dimensions
    assert F.kernel_ft(G, 3 * xi * xi, ell, 3) == pytest.approx(val ** 3, rel=1e-9, abs=1e-30)


@pytest.mark.parametrize("ell,xi", [(0.1, 0.0), (0.1, 2.0), (0.05, 9.0)])
def test_matern_ft_matches_quadrature(ell, xi):
    # d = 1: int e^{-|x|/l} cos(2 pi xi x) dx
    v1, _ = integrate.quad(lambda x: 2 * math.exp(-x / ell), 0, np.inf, weight="cos", wvar=2 * math.pi * xi) \
        if xi > 0 else integrate.quad(lambda x: 2 * math.exp(-x / ell), 0, np.inf)
    assert F.kernel_ft(M, xi * xi, ell, 1) == pytest.approx(v1, rel=1e-8)
    # d = 3: radial transform (2/rho) int_0^inf r sin(2 pi rho r) kappa(r) dr
    if xi > 0:
        v3, _ = integrate.quad(lambda r: r * math.exp(-r / ell), 0, np.inf, weight="sin", wvar=2 * math.pi * xi)
        v3 *= 2.0 / xi
    else:
        v3, _ = integrate.quad(lambda r: 4 * math.pi * r * r * math.exp(-r / ell), 0, np.inf)
    assert F.kernel_ft(M, xi * xi, ell, 3) == pytest.approx(v3, rel=1e-8)
    # d = 2: Hankel transform 2 pi int_0^inf r J0(2 pi rho r) kappa(r) dr
    v2, _ = integrate.quad(lambda r: 2 * math.pi * r * special.j0(2 * math.pi * xi * r) * math.exp(-r / ell),
                           0, 60 * ell, limit=2000, epsabs=1e-14)
    assert F.kernel_ft(M, xi * xi, ell, 2) == pytest.approx(v2, rel=1e-7)


@pytest.mark.parametrize("kernel", [G, M, M3])
@pytest.mark.parametrize("xi", [0.0, 2.5, 6.0])
def test_derivative_kernel_ft_matches_quadrature(kernel, xi):
    ell = 0.08
    f = (lambda x: F.kernel_der_value(kernel, x * x, ell) * math.cos(2 * math.pi * xi * x))
    v, _ = integrate.quad(f, -50 * ell, 50 * ell, limit=2000, epsabs=1e-15, points=[0.0])
    assert F.kernel_der_ft(kernel, xi * xi, ell, 1) == pytest.approx(v, rel=1e-7, abs=1e-13)
    if kernel == G:
        # d = 3 via the radial transform of r^2/(2l^2) e^{-r^2/(2l^2)}
        if xi > 0:
            v3, _ = integrate.quad(lambda r: r * F.kernel_der_value(G, r * r, ell) * math.sin(2 * math.pi * xi * r),
                                   0, 50 * ell, limit=2000, epsabs=1e-16)
            v3 *= 2.0 / xi
        else:
            v3, _ = integrate.quad(lambda r: 4 * math.pi * r * r * F.kernel_der_value(G, r * r, ell), 0, 50 * ell)
        assert F.kernel_der_ft(G, 3 * (xi / math.sqrt(3)) ** 2, ell, 3) == pytest.approx(v3, rel=1e-7, abs=1e-14)


@pytest.mark.parametrize("ell", [0.05, 0.1, 0.3])
def test_truncated_gauss_erf_form_matches_quadrature(ell):
    for k in [0, 1, 5, 16, 40]:
        v, _ = integrate.quad(lambda r: math.exp(-r * r / (2 * ell * ell)) * math.cos(2 * math.pi * k * r),
                              -0.5, 0.5, limit=400, epsabs=1e-16)
        assert F.truncated_gauss_coeff_1d(k, ell) == pytest.approx(v, rel=1e-9, abs=1e-15)


@pytest.mark.parametrize("ell,n", [(0.1, 16), (0.2, 32), (0.05, 64)])
def test_sampled_coefficients_satisfy_aliasing_formula(ell, n):
    """Lemma 1: c^_k = sum_r c_{k + n r} with c_k the coefficients of the
    simple periodic continuation (closed erf form)."""
    ch = F.coeffs_sampled(G, ell, 1.0, n, 1)
    ks = F.modes(n)
    Rr = 400
    rr = np.arange(-Rr, Rr + 1)
    # The continuation has a kink at +-1/2, so c_k ~ C (-1)^{k+1} / k^2 with
    # C = e^{-1/(8 l^2)} / (4 l^2 pi^2) (first integration by parts in the proof
    # of Theorem 1).  The aliases beyond |r| > Rr are summed with that leading
    # term through the trigamma function; the remainder is O((n Rr)^-3).
    C = math.exp(-1.0 / (8 * ell * ell)) / (4 * ell * ell * math.pi ** 2)
    alias = []
    for k in ks:
        s = np.sum(F.truncated_gauss_coeff_1d(k + n * rr, ell))
        tail = (special.polygamma(1, Rr + 1 + k / n) + special.polygamma(1, Rr + 1 - k / n)) / n ** 2
        alias.append(s + (-1.0) ** (k + 1) * C * tail)
    np.testing.assert_allclose(ch, np.array(alias), rtol=0, atol=5e-14)


def test_sampled_equals_aliased_analytic_for_long_period():
    """With T large the kernel is negligible at the torus faces; the sampled
    coefficients are then the aliased Poisson coefficients (Lemma 1)."""
    ell, T, n = 0.1, 1.8, 64
    for d in (1, 2, 3):
        ch = F.coeffs_sampled(G, ell, T, n, d)
        ks = F.modes(n).astype(float)
        acc = np.zeros((n,) * d)
        for shift in range(-3, 4):
            kk = ks + n * shift
            g1 = F.kernel_ft(G, kk * kk / (T * T), ell, 1) / T
            if d == 1:
                acc += g1 if shift == 0 else 0.0
        # separable aliasing: product over dimensions of the 1-D aliased sums
        one = sum(F.kernel_ft(G, (ks + n * s) ** 2 / (T * T), ell, 1) / T for s in range(-3, 4))
        full = one
        for _ in range(d - 1):
            full = np.multiply.outer(full, one)
        np.testing.assert_allclose(ch, full, rtol=0, atol=1e-15)
        ca = F.coeffs_analytic(G, ell, T, n, d)
        assert np.max(np.abs(ca - full)) < 1e-15


def test_derivative_coefficient_relation():
    """c_k(kappa_der) = (1/2)(1 - 4 pi^2 k^2 l^2) c_k(kappa) (1-D, unit torus) and its
    d-dimensional form (d/2 - 2 pi^2 l^2 |k|^2) c_k(kappa)."""
    ell, T, n = 0.1, 1.7, 32
    for d in (1, 3):
        k2 = F._k2_grid(n, d) / (T * T)
        ratio = F.coeffs_analytic(G, ell, T, n, d, der=True) / F.coeffs_analytic(G, ell, T, n, d)
        np.testing.assert_allclose(ratio, d / 2.0 - 2 * math.pi ** 2 * ell ** 2 * k2, rtol=1e-12)
    # the same relation holds (up to aliasing of tiny tails) for sampled coefficients
    # with n = 64 the aliases of the sampled coefficients are below 1e-30
    cs = F.coeffs_sampled(G, ell, T, 64, 1, der=True)
    cg = F.coeffs_sampled(G, ell, T, 64, 1)
    k2 = (F.modes(64) / T) ** 2
    np.testing.assert_allclose(cs, (0.5 - 2 * math.pi ** 2 * ell ** 2 * k2) * cg, atol=1e-14)


def test_trig_sum_single_point_and_plane_wave():
    rng = np.random.default_rng(24)
    c = rng.uniform(0.1, 1.0, size=(8, 8))
    c = 0.5 * (c + np.flip(c, (0, 1)))  # coefficients need not be even for this identity
    x = rng.uniform(-0.5, 0.5, size=(1, 2))
    # one point: sum_k c_k e^{-2pi i k x} e^{2pi i k x} = sum_k c_k
    assert F.trig_sum(c, x, np.array([2.0]))[0] == pytest.approx(2.0 * c.sum(), rel=1e-13)


@pytest.mark.parametrize("kernel", [G])
@pytest.mark.parametrize("d,n", [(1, 32), (2, 32), (3, 32)])
def test_trig_sum_reproduces_direct_sum(kernel, d, n):
    """With the automatic torus period the trigonometric sum of eq. (6) equals the
    direct kernel sum to ~1e-12 (Gaussian, l well resolved)."""
    X = _pts(250, d, 25 + d)
    v = np.random.default_rng(26).standard_normal((250, 1))
    wins = [list(range(d))]
    y = oracle_direct(X, wins, kernel, 0.1, 1.0, v)
    yt = F.fast_sum_oracle(X, wins, kernel, 0.1, 1.0, v, n)
    assert np.linalg.norm(yt - y) / np.linalg.norm(y) < 1e-11


def test_trig_sum_derivatives_reproduce_direct_sums():
    X = _pts(200, 6, 27)
    v = np.random.default_rng(28).standard_normal((200, 1))
    wins = [[0, 1, 2], [3, 4, 5]]
    ell, sig = [0.1, 0.15], [1.0, 0.6]
    y, dl, ds = oracle_direct(X, wins, G, ell, sig, v, want_derivs=True)
    yt, dlt, dst = F.fast_sum_oracle(X, wins, G, ell, sig, v, 32, want_derivs=True)
    assert np.linalg.norm(yt - y) / np.linalg.norm(y) < 1e-11
    for w in range(2):
        assert np.linalg.norm(dlt[w] - dl[w]) / np.linalg.norm(dl[w]) < 1e-10
        assert np.linalg.norm(dst[w] - ds[w]) / np.linalg.norm(ds[w]) < 1e-11


def test_matern_trig_sum_is_approximate_but_consistent():
    """Matern-1/2 has algebraically decaying coefficients; the Fourier error is
    ~1e-3..1e-2 (no bound in the paper), and shrinks as n grows."""
    X = _pts(300, 3, 29)
    v = np.random.default_rng(30).standard_normal((300, 1))
    y = oracle_direct(X, [[0, 1, 2]], M, 0.1, 1.0, v)
    e16 = np.linalg.norm(F.fast_sum_oracle(X, [[0, 1, 2]], M, 0.1, 1.0, v, 16) - y) / np.linalg.norm(y)
    e32 = np.linalg.norm(F.fast_sum_oracle(X, [[0, 1, 2]], M, 0.1, 1.0, v, 32) - y) / np.linalg.norm(y)
    assert e32 < e16 < 0.2


def test_auto_period_balances_the_two_error_terms():
    L, ell, n = 0.5, 0.1, 64
    T = F.torus_period_auto(G, L, ell, n)
    img = (T - L) ** 2 / (2 * ell ** 2)
    trunc = 2 * math.pi ** 2 * ell ** 2 * (n / 2) ** 2 / T ** 2
    assert img == pytest.approx(trunc, rel=1e-12)
    assert F.torus_period_paper(0.5, 3) == pytest.approx(math.sqrt(3.0))


# ---------------------------------------------------------------- error bounds


@pytest.mark.parametrize("n", [16, 32])
@pytest.mark.parametrize("ell", [0.1, 0.2, 0.35, 0.6, 1.5])
def test_measured_errors_below_theorem_bounds(n, ell):
    """The comparison of measured and estimated errors (d = 3, uniform r in
    [-1/2, 1/2]^3, sampled coefficients): measured <= Theorem 1 / Theorem 2."""
    if F.eta(ell, n) < 1:
        pytest.skip("bounds need eta >= 1")
    eg = F.measured_fourier_error(False, ell, n, 3, 1500, 31)
    ed = F.measured_fourier_error(True, ell, n, 3, 1500, 32)
    # the bounds hold in exact arithmetic; allow for FP64 rounding of the sums
    assert eg <= F.theorem1_bound(ell, n) + 1e-14
    assert ed <= F.theorem2_bound(ell, n) + 1e-14


@pytest.mark.parametrize("n", [16, 32, 64])
@pytest.mark.parametrize("ell", [0.05, 0.1, 0.3, 0.8])
def test_measured_errors_below_1d_remarks(n, ell):
    if F.eta(ell, n) < 1:
        pytest.skip("bounds need eta >= 1")
    assert F.measured_fourier_error(False, ell, n, 1, 4000, 33) <= F.remark1_bound(ell, n) + 1e-14
    assert F.measured_fourier_error(True, ell, n, 1, 4000, 34) <= F.remark2_bound(ell, n) + 1e-14


def test_bounds_need_eta_at_least_one():
    with pytest.raises(ValueError):
        F.theorem1_bound(0.01, 16)


# ------------------------------------------------------- global sensitivity


def _anova_variances(c: np.ndarray) -> dict:
    """Variances of the ANOVA terms of f(x) = sum_k c_k e^{2 pi i k.x} on the
    torus, computed from the definition of the decomposition: f is sampled on
    a uniform grid (inverse FFT), each term f_u is the average of f over the
    features outside u minus the terms of the proper subsets of u, and its
    variance is the grid mean of |f_u|^2 (exact for trigonometric polynomials
    on a grid with more points than the bandwidth)."""
    d = c.ndim
    n = c.shape[0]
    G = n + 2
    full = np.zeros((G,) * d, dtype=np.complex128)
    idx = np.ix_(*([(np.arange(n) - n // 2) % G] * d))
    full[idx] = c
    f = np.fft.ifftn(full) * G ** d  # f at x = j / G
    terms = {}
    for u in range(1 << d):
        axes = tuple(i for i in range(d) if not (u >> i & 1))
        g = f.mean(axis=axes, keepdims=True) if axes else f
        for v in terms:
            if v & u == v and v != u:
                g = g - terms[v]
        terms[u] = g
    return {u: float(np.mean(np.abs(np.broadcast_to(t, f.shape)) ** 2)) for u, t in terms.items()}


@pytest.mark.parametrize("d", [1, 2, 3])
def test_gsi_theta_matches_anova_of_the_trigonometric_polynomial(d):
    """theta of Algorithm 1 equals the variances of the ANOVA terms of the
    window's trigonometric polynomial, obtained independently by averaging the
    polynomial over the other features on a grid."""
    rng = np.random.default_rng(70 + d)
    N, n, ell = 300, 12, 0.15
    X = rng.uniform(-0.25, 0.25, size=(N, d))
    v = rng.standard_normal(N)
    theta = F.gsi_theta_oracle(X, [list(range(d))], F.GAUSSIAN, [ell], v, n)[0]
    c, L = F.window_geometry(X)
    T = F.torus_period_auto(F.GAUSSIAN, L, ell, n)
    xt = (X - c) / T
    coef = F.coeffs_analytic(F.GAUSSIAN, ell, T, n, d) * np.conj(F._adjoint_ndft(xt, v, n))
    var = _anova_variances(coef)
    for u in range(1 << d):
        assert theta[u] == pytest.approx(var[u], rel=1e-9, abs=1e-12 * sum(var.values()))


def test_gsi_indices_sum_to_one_and_follow_the_data():
    """The indices of all nonempty subsets sum to one; a target that varies only
    with feature 0 puts (almost) all weight on the subsets holding feature 0."""
    rng = np.random.default_rng(75)
    N = 400
    X = rng.uniform(-0.25, 0.25, size=(N, 4))
    v = np.sin(12 * X[:, 0]) * 0.1
    rho = F.gsi_oracle(X, [[0, 1], [2, 3]], F.GAUSSIAN, [0.2, 0.2], v, 16)
    assert sum(rho.values()) == pytest.approx(1.0, rel=1e-12)
    assert set(rho) == {(0,), (1,), (0, 1), (2,), (3,), (2, 3)}
    assert all(r >= 0 for r in rho.values())


# ------------------------------------------- the bound components, one by one
#
# Each component of the Theorem 1/2 bounds bounds a specific quantity of the
# one-dimensional truncated functions f(x) = e^{-x^2/2l^2} and
# g(x) = x^2/(2 l^2) f(x) on [-1/2, 1/2] (Theorem 1 and 2 proofs):
#   gamma >= |c_{m/2}(f)|,  A >= sum_{k > m/2} |c_k(f)|,
#   xi    >= |c_{m/2}(g)|,  S >= sum_{k > m/2} |c_k(g)|.
# The coefficients here come from adaptive quadrature of their defining
# integrals (independent of every formula in the oracle).  Where e^{-1/8l^2}
# is negligible the coefficients are the sampled continuous transforms, so
# gamma and xi are then tight: their leading terms must equal the quadrature
# value up to the one-sided term of xi, (eta^2 + 1/2) / (eta^2 - 1/2).  A
# wrong constant in a leading term fails the tightness check; one in a tail
# term fails the bound check in the regime where that term dominates.


def _quad_coeff(fun, k):
    """int_{-1/2}^{1/2} fun(x) cos(2 pi k x) dx (fun even), by QUADPACK's
    oscillatory rule."""
    if k == 0:
        return integrate.quad(fun, -0.5, 0.5, limit=400, epsabs=1e-17, epsrel=1e-13)[0]
    return integrate.quad(fun, -0.5, 0.5, weight="cos", wvar=2 * math.pi * k, limit=400, epsabs=1e-18)[0]


def _fg(ell):
    f = lambda x: math.exp(-x * x / (2 * ell * ell))  # noqa: E731
    g = lambda x: x * x / (2 * ell * ell) * math.exp(-x * x / (2 * ell * ell))  # noqa: E731
    return f, g


@pytest.mark.parametrize("ell,n", [(0.05, 10), (0.05, 16), (0.08, 12), (0.2, 8), (0.3, 16), (0.45, 8),
                                   (0.6, 6), (1.0, 8), (2.0, 4)])
def test_bound_components_bound_their_quantities(ell, n):
    et = F.eta(ell, n)
    if et < 1:
        pytest.skip("eta < 1")
    f, g = _fg(ell)
    cf = abs(_quad_coeff(f, n // 2))
    cg = abs(_quad_coeff(g, n // 2))
    kmax = n // 2 + 400
    tf = sum(abs(_quad_coeff(f, k)) for k in range(n // 2 + 1, kmax))
    tg = sum(abs(_quad_coeff(g, k)) for k in range(n // 2 + 1, kmax))
    assert cf <= F.gamma_bound(et, ell) * (1 + 1e-9)
    assert tf <= F.A_bound(et, ell) * (1 + 1e-9)
    assert cg <= F.xi_bound(et, ell) * (1 + 1e-9)
    assert tg <= F.S_bound(et, ell) * (1 + 1e-9)


@pytest.mark.parametrize("ell,n", [(0.05, 10), (0.05, 14), (0.06, 12), (0.04, 16)])
def test_bound_components_tight_where_the_gaussian_term_dominates(ell, n):
    et = F.eta(ell, n)
    lead = ell * math.sqrt(2 * math.pi) * math.exp(-et ** 2)
    assert et >= 1 and math.exp(-1 / (8 * ell * ell)) < 1e-12 * lead
    f, g = _fg(ell)
    cf = abs(_quad_coeff(f, n // 2))
    cg = abs(_quad_coeff(g, n // 2))
    assert F.gamma_bound(et, ell) / cf == pytest.approx(1.0, abs=1e-8)
    assert F.xi_bound(et, ell) / cg == pytest.approx((et ** 2 + 0.5) / (et ** 2 - 0.5), rel=1e-8)
    # the tails: within the integral comparison's slack (a few terms' worth)
    tf = sum(abs(_quad_coeff(f, k)) for k in range(n // 2 + 1, n // 2 + 60))
    tg = sum(abs(_quad_coeff(g, k)) for k in range(n // 2 + 1, n // 2 + 60))
    assert 1.0 <= F.A_bound(et, ell) / tf < 4.0
    assert 1.0 <= F.S_bound(et, ell) / tg < 8.0
