"""GPU parity: the HIP path against the CPU oracle, element by element.

Tolerances (relative 2-norm per RHS, worst RHS):
  * FP64 path vs the direct sum, Gaussian, m = 6:  1e-10
  * FP64 path vs the brute-force trigonometric sum of eq. (6) with the
    plan's own torus period (any kernel, any coefficient mode): 1e-10 --
    this isolates the NFFT window error from the Fourier truncation error
  * FP32 path vs the direct sum: 1e-5
  * c1 configuration (m = 4): 1e-6 (window-limited, about 7e-8 expected)
"""
import sys

import numpy as np
import pytest

import workloads as WL
from _parity import relerr
from oracle import fourier as F
from oracle.direct import oracle_direct

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print("[gpu-case] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def A():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2404_17344_amd as A
    return A


def make_plan(A, p, precision="fp64", **kw):
    return A.Plan(p.X, p.windows, p.ell, p.sigma, kernel=p.kernel, n=p.n, m=p.m, oversampling=p.oversampling,
                  precision=precision, **kw)


def gpu_matvec(plan, V):
    return plan.matvec(torch.from_numpy(np.ascontiguousarray(V)).cuda()).cpu().numpy()


MIXED = [[0, 1, 2], [3, 4], [5]]


@pytest.mark.parametrize("wins", [[[0]], [[0, 1]], [[0, 1, 2]], MIXED])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_small_gaussian_vs_direct(A, wins, prec, tol):
    p = WL.small_problem(700, 6, wins, seed=101, R=3, n=32, m=6)
    _say("small gaussian %s %s" % (wins, prec))
    Y = gpu_matvec(make_plan(A, p, prec), p.V)
    Yo = oracle_direct(p.X, p.windows, p.kernel, p.ell, p.sigma, p.V)
    assert relerr(Y, Yo) < tol


@pytest.mark.parametrize("kernel", [WL.GAUSSIAN, WL.MATERN12])
@pytest.mark.parametrize("coef", ["analytic", "sampled"])
@pytest.mark.parametrize("wins", [[[0]], [[0, 1]], [[0, 1, 2]]])
def test_fp64_vs_trigonometric_sum(A, kernel, coef, wins):
    """Same torus, same coefficients: the GPU result equals the brute-force sum
    of eq. (6) up to the NFFT window error."""
    p = WL.small_problem(400, 3, wins, seed=102, R=2, n=32, m=6, kernel=kernel, ell=[0.12], sigma=[0.9])
    _say("trig-sum kernel=%d coef=%s wins=%s" % (kernel, coef, wins))
    plan = make_plan(A, p, "fp64", coef=coef)
    T = plan.query()["T"]
    Y = gpu_matvec(plan, p.V)
    Yt = F.fast_sum_oracle(p.X, p.windows, kernel, p.ell, p.sigma, p.V, p.n, periods=T, mode=coef)
    assert relerr(Y, Yt) < 1e-10


def test_plan_period_matches_oracle_rule(A):
    p = WL.small_problem(300, 6, MIXED, seed=103, R=1, n=32, m=6)
    _say("period")
    q = make_plan(A, p).query()
    for w, feats in enumerate(p.windows):
        _, L = F.window_geometry(p.X[:, feats])
        assert q["T"][w] == pytest.approx(F.torus_period_auto(p.kernel, L, p.ell[w], p.n), rel=1e-13)
        assert q["d"][w] == len(feats)


def test_c1_single_window(A):
    """Plain FP64 single window (N=2000, n=32, m=4): window-limited to ~7e-8;
    the m = 6 variant reaches the 1e-10 bar."""
    p = WL.single_window_c1()
    _say("c1 m=4")
    Yo = oracle_direct(p.X, p.windows, p.kernel, p.ell, p.sigma, p.V)
    e4 = relerr(gpu_matvec(make_plan(A, p), p.V), Yo)
    p6 = WL.single_window_c1(m=6)
    _say("c1 m=6")
    e6 = relerr(gpu_matvec(make_plan(A, p6), p6.V), Yo)
    print("c1 errors: m=4 %.3e  m=6 %.3e" % (e4, e6))
    assert e4 < 1e-6
    assert e6 < 1e-10


def _outer_rows(p, per_window):
    """The rows farthest from the centre of each window's points (sorted, unique)."""
    out = []
    for feats in p.windows:
        Z = p.X[:, feats]
        r = np.linalg.norm(Z - 0.5 * (Z.min(axis=0) + Z.max(axis=0)), axis=1)
        out.append(np.argsort(r)[-per_window:])
    return np.unique(np.concatenate(out))


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_c2_full_size_sampled_rows(A, prec, tol):
    """Additive 3 x d=3 windows, N = 1e5, n = 64, m = 6, at full size; rows sampled."""
    p = WL.additive_c2()
    _say("c2 %s" % prec)
    Y = gpu_matvec(make_plan(A, p, prec), p.V)
    rows = np.unique(np.concatenate([np.random.default_rng(7).choice(p.N, 384, replace=False), _outer_rows(p, 8)]))
    Yo = oracle_direct(p.X, p.windows, p.kernel, p.ell, p.sigma, p.V, rows=rows)
    err = relerr(Y[rows], Yo)
    print("c2 %s rel err %.3e" % (prec, err))
    assert err < tol


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("fp64", 1e-10)])
def test_c5_full_size_dmatvec_sampled_rows(A, prec, tol):
    """The large workload in the timed launch configuration (N = 1e6, 5 windows
    d = 3, R = 16 column-major, n = 64, m = 6): K V and dK/dl_w V on sampled
    rows against the direct sums."""
    p = WL.large_c5()
    _say("c5 full size %s" % prec)
    V = torch.from_numpy(np.ascontiguousarray(p.V.T)).cuda().t()
    plan = make_plan(A, p, prec)
    Y, dl, _ = plan.dmatvec(V, want_y=True, want_dell=True, want_dsigma=False)
    Y, dl = Y.cpu().numpy(), dl.cpu().numpy()
    plan.close()
    rows = np.random.default_rng(11).choice(p.N, 96, replace=False)
    outer = _outer_rows(p, 8)
    rows = np.unique(np.concatenate([rows, outer]))
    Yo, dlo, _ = oracle_direct(p.X, p.windows, p.kernel, p.ell, p.sigma, p.V, rows=rows, want_derivs=True)
    errs = [relerr(Y[rows], Yo)] + [relerr(dl[w][rows], dlo[w]) for w in range(p.P)]
    print("c5 %s rel errs %s" % (prec, " ".join("%.2e" % e for e in errs)))
    assert max(errs) < tol
    # the outermost points of every window lie in sparsely populated tiles (tile
    # kernels); relerr's element-wise measure covers them among the sampled rows
    io = np.searchsorted(rows, outer)
    errs_o = [np.abs(Y[outer] - Yo[io]).max() / np.abs(Yo).max()] + \
        [np.abs(dl[w][outer] - dlo[w][io]).max() / np.abs(dlo[w]).max() for w in range(p.P)]
    print("c5 %s outer rows: max error / max |y| %s" % (prec, " ".join("%.2e" % e for e in errs_o)))


def test_many_rhs_and_ragged_blocks(A):
    """R = 19 spans several RHS blocks and an odd last complex grid."""
    p = WL.small_problem(900, 6, MIXED, seed=104, R=19, n=32, m=6)
    _say("R=19")
    for prec, tol in [("fp64", 1e-10), ("fp32", 1e-5)]:
        Y = gpu_matvec(make_plan(A, p, prec), p.V)
        Yo = oracle_direct(p.X, p.windows, p.kernel, p.ell, p.sigma, p.V)
        assert relerr(Y, Yo) < tol


def test_chunked_dense_tile(A):
    """Many points in one tile (more than one chunk of 1024) and a ragged tail."""
    rng = np.random.default_rng(105)
    X = np.concatenate([rng.normal(0, 0.002, size=(5000, 3)), rng.uniform(-0.25, 0.25, size=(37, 3))])
    V = rng.standard_normal((X.shape[0], 2))
    _say("dense tile")
    plan = A.Plan(X, [[0, 1, 2]], [0.1], [1.0], n=32, m=6)
    Y = gpu_matvec(plan, V)
    Yo = oracle_direct(X, [[0, 1, 2]], WL.GAUSSIAN, [0.1], [1.0], V)
    assert relerr(Y, Yo) < 1e-10


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 2e-6)])
def test_dense_cell_kernels_match_tile_kernels(A, prec, tol):
    """Dense-cell kernels and tile kernels compute the same sums (different order)."""
    p = WL.small_problem(20000, 6, [[0, 1, 2], [3, 4], [5]], seed=109, R=5, n=32, m=6, dist="normal")
    _say("dense vs tile %s" % prec)
    Yd = gpu_matvec(make_plan(A, p, prec), p.V)
    Yt = gpu_matvec(make_plan(A, p, prec, dense_kernels=False), p.V)
    assert relerr(Yd, Yt) < tol
    Yo = oracle_direct(p.X, p.windows, p.kernel, p.ell, p.sigma, p.V, rows=np.arange(0, 20000, 97))
    assert relerr(Yd[::97], Yo) < (1e-10 if prec == "fp64" else 1e-5)


@pytest.mark.parametrize("m", [4, 6])
@pytest.mark.parametrize("R", [1, 3, 8, 16, 21])
def test_matrix_core_kernels_match_vector_kernels(A, m, R):
    """FP32 dense-cell kernels on the matrix cores agree with the vector-ALU ones,
    the tile kernels and the oracle (RHS counts that fill, underfill and spill a
    16-wide block; one RHS takes the spread with the z-slabs as columns)."""
    rng = np.random.default_rng(111)
    X = np.concatenate([rng.normal(0, 0.02, size=(30000, 3)), rng.uniform(-0.25, 0.25, size=(700, 3))])
    V = rng.standard_normal((X.shape[0], R))
    _say("mfma vs valu m=%d R=%d" % (m, R))
    mk = lambda **kw: A.Plan(X, [[0, 1, 2]], [0.1], [1.0], n=32, m=m, precision="fp32", **kw)  # noqa: E731
    pm = mk()
    Ym, dlm, _ = pm.dmatvec(torch.from_numpy(V).cuda())
    Yv, dlv, _ = mk(matrix_cores=False).dmatvec(torch.from_numpy(V).cuda())
    Yt, dlt, _ = mk(dense_kernels=False).dmatvec(torch.from_numpy(V).cuda())
    Y64, dl64, _ = A.Plan(X, [[0, 1, 2]], [0.1], [1.0], n=32, m=m, precision="fp64").dmatvec(
        torch.from_numpy(V).cuda())
    assert pm.query()["dense_points"] > 20000
    # Each FP32 variant carries its own rounding error.  This data set is a tight
    # cluster (up to ~2e3 points per grid cell, random-sign RHS), where FP32 sums
    # of n terms lose about eps32 * sqrt(n) ~ 1e-5 relative: every variant is held
    # to 2e-5 against the FP64 path and any two of them to 60% of that.  The
    # workload-shaped cases are held to 1e-5 elsewhere.
    tol = 2e-5
    for a in [Ym, Yv, Yt]:
        assert relerr(a.cpu().numpy(), Y64.cpu().numpy()) < tol
    for a in [dlm, dlv, dlt]:
        assert relerr(a[0].cpu().numpy(), dl64[0].cpu().numpy()) < tol
    for a, b in [(Ym, Yv), (Ym, Yt), (dlm[0], dlv[0]), (dlm[0], dlt[0])]:
        assert relerr(a.cpu().numpy(), b.cpu().numpy()) < 0.6 * tol
    # K V alone runs the one-output variants of the same kernels
    Yk = pm.matvec(torch.from_numpy(V).cuda())
    assert relerr(Yk.cpu().numpy(), Y64.cpu().numpy()) < tol
    assert relerr(Yk.cpu().numpy(), Ym.cpu().numpy()) < 0.6 * tol
    rows = np.arange(0, X.shape[0], 61)
    Yo = oracle_direct(X, [[0, 1, 2]], WL.GAUSSIAN, [0.1], [1.0], V, rows=rows)
    assert relerr(Ym.cpu().numpy()[rows], Yo) < (1e-5 if m == 6 else 2e-5)


@pytest.mark.parametrize("m", [4, 6])
@pytest.mark.parametrize("R", [8, 16, 21])
def test_fp64_matrix_core_interp(A, m, R):
    """FP64 dense-cell and sparse-tile interpolation (the 700 uniform points) on
    the matrix cores (v_mfma_f64_16x16x4f64) against the vector-ALU kernels
    (same FP64 products, other summation order) and the direct sum, for K V
    alone and with the derivative products."""
    rng = np.random.default_rng(112)
    X = np.concatenate([rng.normal(0, 0.02, size=(30000, 3)), rng.uniform(-0.25, 0.25, size=(700, 3))])
    V = rng.standard_normal((X.shape[0], R))
    _say("fp64 mfma interp m=%d R=%d" % (m, R))
    mk = lambda **kw: A.Plan(X, [[0, 1, 2]], [0.1], [1.0], n=32, m=m, precision="fp64", **kw)  # noqa: E731
    pm, pv = mk(), mk(matrix_cores=False)
    assert pm.query()["dense_points"] > 20000
    Vc = torch.from_numpy(V).cuda()
    Ym, dlm, _ = pm.dmatvec(Vc)
    Yv, dlv, _ = pv.dmatvec(Vc)
    Yk = pm.matvec(Vc)
    assert relerr(Ym.cpu().numpy(), Yv.cpu().numpy()) < 1e-12
    assert relerr(dlm[0].cpu().numpy(), dlv[0].cpu().numpy()) < 1e-12
    assert relerr(Yk.cpu().numpy(), Yv.cpu().numpy()) < 1e-12
    rows = np.arange(0, X.shape[0], 61)
    Yo, dlo, _ = oracle_direct(X, [[0, 1, 2]], WL.GAUSSIAN, [0.1], [1.0], V, rows=rows, want_derivs=True)
    # m = 4 is window-limited: on this tight cluster its element-wise error
    # reaches 1.5e-6 of max |y| (both FP64 kernels alike)
    tol = 1e-10 if m == 6 else 5e-6
    assert relerr(Ym.cpu().numpy()[rows], Yo) < tol
    assert relerr(dlm[0].cpu().numpy()[rows], dlo[0]) < tol


@pytest.mark.parametrize("m", [4, 6])
def test_dense_kernels_all_dims(A, m):
    """Clustered points in d = 1, 2, 3 windows so that every dense kernel runs."""
    rng = np.random.default_rng(110)
    X = np.concatenate([rng.normal(0, 0.01, size=(6000, 6)), rng.uniform(-0.25, 0.25, size=(500, 6))])
    V = rng.standard_normal((X.shape[0], 7))
    wins = [[0], [1, 2], [3, 4, 5]]
    _say("dense all dims m=%d" % m)
    plan = A.Plan(X, wins, [0.1, 0.12, 0.15], [1.0, 0.8, 1.2], n=32, m=m)
    Y = gpu_matvec(plan, V)
    Yo = oracle_direct(X, wins, WL.GAUSSIAN, [0.1, 0.12, 0.15], [1.0, 0.8, 1.2], V, rows=np.arange(0, 6500, 13))
    assert relerr(Y[::13], Yo) < (1e-10 if m == 6 else 1e-6)


def test_single_point_and_identical_points(A):
    _say("degenerate")
    X1 = np.array([[0.1, -0.2, 0.05]])
    plan = A.Plan(X1, [[0, 1, 2], [1]], [0.1, 0.2], [0.7, 1.1], n=32, m=6)
    v = np.array([[2.5]])
    assert gpu_matvec(plan, v)[0, 0] == pytest.approx((0.49 + 1.21) * 2.5, rel=1e-10)
    Xs = np.tile(np.array([[0.05, 0.0, -0.1]]), (50, 1))  # zero extent: L = 0
    vs = np.random.default_rng(106).standard_normal((50, 1))
    Ys = gpu_matvec(A.Plan(Xs, [[0, 1, 2]], [0.1], [1.0], n=32, m=6), vs)
    np.testing.assert_allclose(Ys[:, 0], vs.sum(), rtol=1e-10)


def test_empty_plan(A):
    _say("empty")
    plan = A.Plan(np.zeros((0, 3)), [[0, 1, 2]], [0.1], [1.0], n=32, m=6)
    Y = plan.matvec(torch.zeros((0, 2), dtype=torch.float64, device="cuda"))
    assert tuple(Y.shape) == (0, 2)


def test_raw_abi_leading_dimensions(A):
    """Padded leading dimensions through the C ABI directly."""
    import ctypes
    from paper_2404_17344_amd import _lib as L
    p = WL.small_problem(300, 3, [[0, 1, 2]], seed=107, R=2, n=32, m=6)
    _say("raw abi ld")
    plan = make_plan(A, p)
    ld = p.N + 5
    Vp = torch.zeros((2, ld), dtype=torch.float64, device="cuda")
    Vp[:, :p.N] = torch.from_numpy(p.V.T.copy())
    Yp = torch.full((2, ld + 3), 7.0, dtype=torch.float64, device="cuda")
    L.check(L.load().addk_matvec(plan.handle, 2, Vp.data_ptr(), ld, Yp.data_ptr(), ld + 3, ctypes.c_void_p(0)),
            "addk_matvec")
    torch.cuda.synchronize()
    Y = Yp[:, :p.N].cpu().numpy().T
    Yo = oracle_direct(p.X, p.windows, p.kernel, p.ell, p.sigma, p.V)
    assert relerr(Y, Yo) < 1e-10
    assert torch.all(Yp[:, p.N:ld + 3] == 7.0)  # padding untouched


def test_argument_errors(A):
    _say("errors")
    X = np.random.default_rng(108).uniform(-0.25, 0.25, (50, 4))
    with pytest.raises(A.AddkError, match="unsupported"):
        A.Plan(X, [[0, 1, 2, 3]], [0.1], [1.0], n=32, m=6)
    with pytest.raises(A.AddkError, match="invalid"):
        A.Plan(X, [[0]], [0.1], [1.0], n=31, m=6)
    with pytest.raises(A.AddkError, match="accuracy"):
        A.Plan(X, [[0]], [0.005], [1.0], n=16, m=4)
    with pytest.raises(A.AddkError, match="unsupported"):
        A.Plan(X, [[0]], [0.1], [1.0], n=128, m=6, oversampling=4.0)  # n_os = 512
    plan = A.Plan(X, [[0, 1]], [0.1], [1.0], n=32, m=6)
    import ctypes
    from paper_2404_17344_amd import _lib as L
    host = np.zeros((50, 1))
    st = L.load().addk_matvec(plan.handle, 1, host.ctypes.data, 50, host.ctypes.data, 50, ctypes.c_void_p(0))
    assert st == L.ADDK_ERR_INVALID_ARG
    st = L.load().addk_matvec(plan.handle, 0, host.ctypes.data, 50, host.ctypes.data, 50, ctypes.c_void_p(0))
    assert st == L.ADDK_ERR_INVALID_ARG
