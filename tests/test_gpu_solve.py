"""GPU parity of products at separate target points (eq. (4) with x' != x) and
of the conjugate-gradient solve of the kernel ridge regression system (eq. (9))."""
import sys

import numpy as np
import pytest

import workloads as WL
from _parity import relerr
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


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


WINS = [[0, 1, 2], [3, 4], [5]]


def _rect_case(seed, Ns=3000, Nt=1700, R=3):
    rng = np.random.default_rng(seed)
    Xs = rng.uniform(-0.25, 0.25, size=(Ns, 6))
    Xt = rng.uniform(-0.2, 0.25, size=(Nt, 6))
    V = rng.standard_normal((Ns, R))
    ell = np.array([0.12, 0.2, 0.1])
    sig = np.array([1.0, 0.7, 1.3])
    return Xs, Xt, V, ell, sig


def _oracle_targets(Xs, Xt, V, ell, sig, want_derivs=False):
    """y_i = sum_j K(x'_i, x_j) v_j: the direct sum over the sources, evaluated at
    the target rows of the stacked point set (the targets carry no weight)."""
    X = np.concatenate([Xs, Xt])
    Vz = np.concatenate([V, np.zeros((Xt.shape[0], V.shape[1]))])
    rows = np.arange(Xs.shape[0], X.shape[0])
    return oracle_direct(X, WINS, WL.GAUSSIAN, ell, sig, Vz, rows=rows, want_derivs=want_derivs)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_targets_match_direct_sum(A, prec, tol):
    Xs, Xt, V, ell, sig = _rect_case(91)
    _say("targets %s" % prec)
    plan = A.Plan(Xs, WINS, ell, sig, n=32, m=6, precision=prec, targets=Xt)
    q = plan.query()
    assert q["n_sources"] == Xs.shape[0] and q["n_targets"] == Xt.shape[0]
    Y = plan.matvec(cuda(V)).cpu().numpy()
    assert Y.shape == (Xt.shape[0], V.shape[1])
    Yo, dlo, dso = _oracle_targets(Xs, Xt, V, ell, sig, want_derivs=True)
    assert relerr(Y, Yo) < tol
    Y2, dl, ds = plan.dmatvec(cuda(V))
    assert relerr(Y2.cpu().numpy(), Yo) < tol
    for w in range(len(WINS)):
        assert relerr(dl[w].cpu().numpy(), dlo[w]) < (1e-10 if prec == "fp64" else 1e-5)
        assert relerr(ds[w].cpu().numpy(), dso[w]) < tol


def test_targets_equal_to_sources_give_the_square_product(A):
    Xs, _, V, ell, sig = _rect_case(92, Ns=2500)
    _say("targets = sources")
    sq = A.Plan(Xs, WINS, ell, sig, n=32, m=6).matvec(cuda(V)).cpu().numpy()
    rc = A.Plan(Xs, WINS, ell, sig, n=32, m=6, targets=Xs).matvec(cuda(V)).cpu().numpy()
    assert relerr(rc, sq) < 1e-12


def test_square_only_entry_points_refuse_target_plans(A):
    Xs, Xt, V, ell, sig = _rect_case(93, Ns=500, Nt=300, R=1)
    plan = A.Plan(Xs, WINS, ell, sig, n=32, m=6, targets=Xt)
    with pytest.raises(A.AddkError):
        plan.vjp(cuda(V), cuda(V))
    with pytest.raises(A.AddkError):
        plan.cg(cuda(V), beta=1.0)
    with pytest.raises(A.AddkError):
        A.Batch([plan], R=1)


def test_cg_solves_the_regularised_system(A):
    """FP64 plan, tight tolerance: the solution satisfies (K + beta I) x = y for
    the exact kernel matrix (built column by column by the oracle) up to the
    product's approximation error."""
    rng = np.random.default_rng(94)
    N = 1200
    X = rng.uniform(-0.25, 0.25, size=(N, 6))
    ell = [0.15, 0.2, 0.12]
    sig = [1.0, 0.8, 0.6]
    y = rng.standard_normal((N, 2))
    beta = 0.05
    _say("cg fp64")
    plan = A.Plan(X, WINS, ell, sig, n=32, m=6)
    x, it, rel = plan.cg(cuda(y), beta=beta, tol=1e-10, maxit=2000)
    assert 0 < it < 2000 and np.all(rel <= 1e-10)
    K = oracle_direct(X, WINS, WL.GAUSSIAN, ell, sig, np.eye(N))
    xs = np.linalg.solve(K + beta * np.eye(N), y)
    assert relerr(x.cpu().numpy(), xs) < 1e-6
    res = (K + beta * np.eye(N)) @ x.cpu().numpy() - y
    assert np.max(np.linalg.norm(res, axis=0) / np.linalg.norm(y, axis=0)) < 1e-8


def test_cg_near_field_matern_one_rhs(A):
    """CG on a near-field corrected Matern-1/2 plan with one right-hand side
    (its products evaluate each close pair once, for both points): the residual
    recomputed through the two-column product (each pair from both ends) meets
    the tolerance, and the residual with the direct kernel matrix is the
    product's error, (K - K_fast) x, about 1e-5 of |K x| <= 2 |y|."""
    rng = np.random.default_rng(95)
    N = 1200
    X = WL.minmax_quarter(rng.standard_normal((N, 6)))
    ell = [0.1, 0.07, 0.15]
    sig = [1.0, 0.8, 0.6]
    y = rng.standard_normal((N, 1))
    beta = 0.05
    _say("cg near field matern fp64")
    plan = A.Plan(X, WINS, ell, sig, kernel="matern12", n=64, m=6, near_field=True)
    x, it, rel = plan.cg(cuda(y), beta=beta, tol=1e-10, maxit=2000)
    assert 0 < it < 2000 and rel[0] <= 1e-10
    xn = x.cpu().numpy()
    both = plan.matvec(cuda(np.concatenate([xn, xn], axis=1))).cpu().numpy()
    for c in range(2):
        r = both[:, c:c + 1] + beta * xn - y
        assert np.linalg.norm(r) / np.linalg.norm(y) < 1e-9
    K = oracle_direct(X, WINS, WL.MATERN12, ell, sig, np.eye(N))
    r = K @ xn + beta * xn - y
    assert np.linalg.norm(r) / np.linalg.norm(y) < 1e-4


def test_cg_krr_additive_workload(A):
    """Kernel ridge regression on the additive 1e5-point workload (FP32 products,
    tolerance 1e-3 as in the paper's solver runs); the residual recomputed with
    the FP64 product meets the tolerance."""
    p = WL.additive_c2(N=100000, R=1)
    y = (np.sin(8 * p.X[:, 0]) + 0.5 * p.X[:, 4] * p.X[:, 7] + 0.1 * p.V[:, 0])[:, None]
    assert y.shape == (p.N, 1)
    _say("cg krr N=1e5")
    beta = 1.0
    p32 = A.Plan(p.X, p.windows, p.ell, p.sigma, n=64, m=6, precision="fp32")
    x, it, rel = p32.cg(cuda(y), beta=beta, tol=1e-3, maxit=1000)
    _say("cg krr: %d iterations, relres %.2e" % (it, rel[0]))
    assert it < 1000 and rel[0] <= 1e-3
    p64 = A.Plan(p.X, p.windows, p.ell, p.sigma, n=64, m=6, precision="fp64")
    r = p64.matvec(x).cpu().numpy() + beta * x.cpu().numpy() - y
    assert np.linalg.norm(r) / np.linalg.norm(y) < 1.2e-3


@pytest.mark.parametrize("case", ["outside", "one_target", "one_source"])
def test_target_edge_cases(A, case):
    """Targets partly outside the sources' box (the torus covers both sets), a
    single target and a single source: FP64 against the direct sum."""
    rng = np.random.default_rng(95)
    Ns, Nt = {"outside": (2000, 800), "one_target": (2500, 1), "one_source": (1, 600)}[case]
    Xs = rng.uniform(-0.25, 0.25, size=(Ns, 6))
    Xt = rng.uniform(0.1, 0.4, size=(Nt, 6)) if case == "outside" else rng.uniform(-0.25, 0.25, size=(Nt, 6))
    V = rng.standard_normal((Ns, 2))
    ell, sig = np.array([0.12, 0.2, 0.1]), np.array([1.0, 0.7, 1.3])
    _say("targets edge case %s" % case)
    plan = A.Plan(Xs, WINS, ell, sig, n=32, m=6, targets=Xt)
    Y = plan.matvec(cuda(V)).cpu().numpy()
    Yo = _oracle_targets(Xs, Xt, V, ell, sig)
    assert relerr(Y, Yo) < 1e-10
