"""GPU parity of the near-field corrected Matern-1/2 products (ADDK_NEAR_FIELD):
against the oracle of the same corrected method (FP64, tight), against the
direct sum at the size of the derivative workload (N = 1e5, three d = 3
windows, FP64 and FP32), for the vjp, for target points, inside a batch, for
the symmetric one-right-hand-side kernel against the one-sided one, and on
degenerate inputs."""
import sys

import numpy as np
import pytest

import workloads as WL
from _parity import relerr
from oracle import nearfield as NF
from oracle.direct import oracle_direct, oracle_vjp

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


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _plan(A, p, prec, **kw):
    return A.Plan(p.X, p.windows, p.ell, p.sigma, kernel="matern12", n=p.n, m=p.m, precision=prec,
                  near_field=True, **kw)


@pytest.mark.parametrize("R", [3, 1])
@pytest.mark.parametrize("N", [1500, 37])
def test_matches_the_corrected_method_oracle(A, N, R):
    """Same method, independent implementations: spread / FFT / interp plus the
    close-pair kernel against exact NDFTs plus a dense pair sum.  d = 1, 2, 3
    windows with their own l; n = 32 (more than one tile per axis, ragged
    tiles); FP64 agreement to 1e-8 (the window's own error is far below).
    R = 1 takes the symmetric close-pair kernel (each pair evaluated once)."""
    p = WL.small_problem(N, 6, [[0], [1, 2], [3, 4, 5]], seed=301, R=R, ell=[0.05, 0.1, 0.2],
                         sigma=[1.0, 0.8, 0.6], kernel=WL.MATERN12, n=32, m=6)
    _say("near field vs corrected oracle N=%d R=%d" % (N, R))
    plan = _plan(A, p, "fp64")
    Y, dl, ds = plan.dmatvec(cuda(p.V))
    Yo, dlo, dso = NF.nearfield_fast_sum_oracle(p.X, p.windows, p.ell, p.sigma, p.V, p.n, want_derivs=True)
    assert relerr(Y.cpu().numpy(), Yo) < 1e-8
    for w in range(3):
        assert relerr(dl[w].cpu().numpy(), dlo[w]) < 1e-8
        assert relerr(ds[w].cpu().numpy(), dso[w]) < 1e-8


@pytest.fixture(scope="module")
def c3m():
    return WL.derivative_c3(N=100000, kernel=WL.MATERN12)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_derivative_workload_against_direct_sum(A, c3m, prec):
    """N = 1e5 Gaussian-distributed points, three d = 3 windows with l = 0.05,
    0.1, 0.2, n = 64, m = 6: K v, (dK/dl_w) v and (dK/dsigma_w) v within 1e-5
    of the direct FP64 sums on 96 sampled rows (rows sampled, all columns)."""
    p = c3m
    _say("near field c3 matern %s" % prec)
    plan = _plan(A, p, prec)
    Y, dl, ds = plan.dmatvec(cuda(p.V))
    rows = np.sort(np.random.default_rng(7).choice(p.N, 96, replace=False))
    Yo, dlo, dso = oracle_direct(p.X, p.windows, WL.MATERN12, p.ell, p.sigma, p.V, rows=rows, want_derivs=True)
    assert relerr(Y.cpu().numpy()[rows], Yo) < 1e-5
    for w in range(3):
        assert relerr(dl[w].cpu().numpy()[rows], dlo[w]) < 1e-5
        assert relerr(ds[w].cpu().numpy()[rows], dso[w]) < 1e-5
    # the same plan without the correction is far off (the cusp and the images)
    plain = A.Plan(p.X, p.windows, p.ell, p.sigma, kernel="matern12", n=p.n, m=p.m, precision=prec)
    assert relerr(plain.matvec(cuda(p.V)).cpu().numpy()[rows], Yo) > 1e-3


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-5), ("fp32", 2e-5)])
def test_vjp_against_direct_gradients(A, prec, tol):
    """Gradients of <G, K V>: K G and the l / sigma gradients, which include the
    close-pair inner products, against the direct sums."""
    p = WL.small_problem(4000, 6, [[0, 1, 2], [3, 4], [5]], seed=302, R=2, ell=[0.1, 0.07, 0.15],
                         sigma=[1.0, 0.9, 1.2], kernel=WL.MATERN12, n=64, m=6, dist="gauss")
    G = np.random.default_rng(303).standard_normal(p.V.shape)
    _say("near field vjp %s" % prec)
    plan = _plan(A, p, prec)
    gV, gl, gs = plan.vjp(cuda(p.V), cuda(G))
    gVo, glo, gso = oracle_vjp(p.X, p.windows, WL.MATERN12, p.ell, p.sigma, p.V, G)
    assert relerr(gV.cpu().numpy(), gVo) < tol
    np.testing.assert_allclose(gl.cpu().numpy(), glo, rtol=tol, atol=tol * np.abs(glo).max())
    np.testing.assert_allclose(gs.cpu().numpy(), gso, rtol=tol, atol=tol * np.abs(gso).max())


def test_targets_and_batch(A):
    """Separate target points (their rows of the stacked direct sum), and the
    corrected plans inside a captured batch next to a Gaussian plan: graph
    replays agree with each plan's own product."""
    rng = np.random.default_rng(304)
    wins = [[0, 1, 2], [3]]
    Xs = WL.minmax_quarter(rng.standard_normal((6000, 4)))
    Xt = rng.uniform(-0.2, 0.2, (900, 4))
    V = rng.standard_normal((6000, 2))
    ell, sig = [0.08, 0.12], [1.0, 0.5]
    _say("near field targets")
    pt = A.Plan(Xs, wins, ell, sig, kernel="matern12", n=64, m=6, near_field=True, targets=Xt)
    Y = pt.matvec(cuda(V)).cpu().numpy()
    X = np.concatenate([Xs, Xt])
    Vz = np.concatenate([V, np.zeros((Xt.shape[0], 2))])
    Yo = oracle_direct(X, wins, WL.MATERN12, ell, sig, Vz, rows=np.arange(6000, 6900))
    assert relerr(Y, Yo) < 1e-5
    _say("near field batch")
    q1 = WL.small_problem(5000, 4, wins, seed=305, R=2, ell=ell, sigma=sig, kernel=WL.MATERN12, n=64, m=6)
    q2 = WL.small_problem(3000, 3, [[0, 1], [2]], seed=306, R=2, ell=[0.1, 0.2], sigma=[1.0, 1.0],
                          kernel=WL.MATERN12, n=64, m=6)
    q3 = WL.small_problem(4000, 3, [[0, 1, 2]], seed=307, R=2, n=32, m=6)
    plans = [_plan(A, q1, "fp64"), _plan(A, q2, "fp64"),
             A.Plan(q3.X, q3.windows, q3.ell, q3.sigma, n=32, m=6)]
    own = [pl.matvec(cuda(q.V)).cpu().numpy() for pl, q in zip(plans, [q1, q2, q3])]
    B = A.Batch(plans, R=2)
    B.set_inputs([cuda(q.V) for q in [q1, q2, q3]])
    for _ in range(2):
        B.launch()
        torch.cuda.synchronize()
        for y, y0 in zip(B.outputs(), own):
            assert relerr(y.cpu().numpy(), y0) < 1e-12
    B.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_symmetric_pairs_equal_one_sided(A, prec, tol):
    """One right-hand side (each close pair evaluated once, for both points)
    against the same vector as both columns of an R = 2 product (each pair
    from both ends): equal up to rounding, also on a second call (the sums
    by sorted position are cleared after each use).  Gaussian points, so
    that tiles hold full and partial 64-point batches."""
    p = WL.small_problem(20000, 6, [[0, 1, 2], [3, 4], [5]], seed=308, R=1, ell=[0.1, 0.05, 0.2],
                         sigma=[1.0, 0.7, 0.9], kernel=WL.MATERN12, n=64, m=6, dist="gauss")
    _say("near field symmetric vs one-sided %s" % prec)
    plan = _plan(A, p, prec)
    v = cuda(p.V[:, :1])
    two = cuda(np.concatenate([p.V[:, :1], p.V[:, :1]], axis=1))
    Y2, dl2, ds2 = plan.dmatvec(two)
    for _ in range(2):
        Y1, dl1, ds1 = plan.dmatvec(v)
        assert relerr(Y1.cpu().numpy(), Y2.cpu().numpy()[:, :1]) < tol
        for w in range(3):
            assert relerr(dl1[w].cpu().numpy(), dl2[w].cpu().numpy()[:, :1]) < tol
            assert relerr(ds1[w].cpu().numpy(), ds2[w].cpu().numpy()[:, :1]) < tol
    _say("near field symmetric batch replays")
    q = WL.small_problem(3000, 3, [[0, 1], [2]], seed=309, R=1, ell=[0.1, 0.2], sigma=[1.0, 1.0],
                         kernel=WL.MATERN12, n=64, m=6)
    plans = [plan, _plan(A, q, prec)]
    own = [pl.matvec(cuda(x)).cpu().numpy() for pl, x in zip(plans, (p.V[:, :1], q.V))]
    B = A.Batch(plans, R=1)
    B.set_inputs([v, cuda(q.V)])
    for _ in range(3):
        B.launch()
        torch.cuda.synchronize()
        for y, y0 in zip(B.outputs(), own):
            assert relerr(y.cpu().numpy(), y0) < tol
    B.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-5), ("fp32", 1e-5)])
def test_targets_one_rhs(A, prec, tol):
    """Separate target points with one right-hand side (the one-sided
    close-pair kernel, since targets and sources differ): the targets' rows of
    the stacked direct sum, for K v and the derivative products."""
    rng = np.random.default_rng(310)
    wins = [[0, 1, 2], [3, 4]]
    Xs = WL.minmax_quarter(rng.standard_normal((5000, 5)))
    Xt = rng.uniform(-0.2, 0.2, (700, 5))
    V = rng.standard_normal((5000, 1))
    ell, sig = [0.1, 0.06], [1.0, 0.7]
    _say("near field targets R=1 %s" % prec)
    pt = A.Plan(Xs, wins, ell, sig, kernel="matern12", n=64, m=6, precision=prec, near_field=True, targets=Xt)
    Y, dl, ds = pt.dmatvec(cuda(V))
    X = np.concatenate([Xs, Xt])
    Vz = np.concatenate([V, np.zeros((Xt.shape[0], 1))])
    rows = np.arange(5000, 5700)
    Yo, dlo, dso = oracle_direct(X, wins, WL.MATERN12, ell, sig, Vz, rows=rows, want_derivs=True)
    assert relerr(Y.cpu().numpy(), Yo) < tol
    for w in range(2):
        assert relerr(dl[w].cpu().numpy(), dlo[w]) < 2 * tol
        assert relerr(ds[w].cpu().numpy(), dso[w]) < tol


def test_degenerate_inputs_and_refusals(A):
    """One point (L = 0, where the result is sigma^2 v up to the method's
    error at n = 64), two far-apart points (no close pairs but the diagonal),
    and the configurations the correction refuses."""
    X1 = np.array([[0.1, -0.2, 0.05]])
    V1 = np.array([[1.5]])
    _say("near field degenerate")
    Y1 = A.Plan(X1, [[0, 1, 2]], [0.1], [0.7], kernel="matern12", n=64, m=6, near_field=True).matvec(cuda(V1))
    assert abs(Y1.cpu().numpy()[0, 0] - 0.49 * 1.5) < 1e-5 * 0.49 * 1.5
    X2 = np.array([[-0.25, 0.0], [0.25, 0.1]])
    V2 = np.array([[1.0], [-2.0]])
    Y2 = A.Plan(X2, [[0, 1]], [0.05], [1.0], kernel="matern12", n=64, m=6, near_field=True).matvec(cuda(V2))
    Yo = oracle_direct(X2, [[0, 1]], WL.MATERN12, [0.05], [1.0], V2)
    assert relerr(Y2.cpu().numpy(), Yo) < 1e-5
    with pytest.raises(A.AddkError):
        A.Plan(X2, [[0, 1]], [0.1], [1.0], kernel="gaussian", n=32, near_field=True)
    with pytest.raises(A.AddkError):
        A.Plan(X2, [[0, 1]], [0.1], [1.0], kernel="matern12", n=32, near_field=True, coef="sampled")
    with pytest.raises(A.AddkError):
        A.Plan(X2, [[0, 1]], [0.1], [1.0], kernel="matern12", n=8, m=2, near_field=True)
    pl = A.Plan(X2, [[0, 1]], [0.1], [1.0], kernel="matern12", n=32, near_field=True)
    with pytest.raises(A.AddkError):
        pl.gsi(cuda(V2[:, 0]))
