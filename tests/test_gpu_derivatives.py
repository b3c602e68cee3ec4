"""GPU parity of the derivative products, the vjp, autograd and batching."""
import sys

import numpy as np
import pytest

import workloads as WL
from _parity import relerr
from oracle import fourier as F
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


def make_plan(A, p, precision="fp64", **kw):
    return A.Plan(p.X, p.windows, p.ell, p.sigma, kernel=p.kernel, n=p.n, m=p.m, oversampling=p.oversampling,
                  precision=precision, **kw)


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


MIXED = [[0, 1, 2], [3, 4], [5]]


@pytest.mark.parametrize("R", [1, 3, 4, 5])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_dmatvec_gaussian_vs_direct(A, prec, tol, R):
    """R <= 4 combines row by row, R = 5 through the 16-RHS tiles."""
    p = WL.small_problem(800, 6, MIXED, seed=201, R=R, n=32, m=6)
    _say("dmatvec gaussian %s R=%d" % (prec, R))
    Y, dl, ds = make_plan(A, p, prec).dmatvec(cuda(p.V))
    Yo, dlo, dso = oracle_direct(p.X, p.windows, p.kernel, p.ell, p.sigma, p.V, want_derivs=True)
    assert relerr(Y.cpu().numpy(), Yo) < tol
    for w in range(p.P):
        assert relerr(dl[w].cpu().numpy(), dlo[w]) < tol
        assert relerr(ds[w].cpu().numpy(), dso[w]) < tol


@pytest.mark.parametrize("coef", ["analytic", "sampled"])
def test_dmatvec_matern_vs_trigonometric_sum(A, coef):
    p = WL.small_problem(500, 6, MIXED, seed=202, R=2, n=32, m=6, kernel=WL.MATERN12)
    _say("dmatvec matern %s" % coef)
    plan = make_plan(A, p, "fp64", coef=coef)
    T = plan.query()["T"]
    Y, dl, ds = plan.dmatvec(cuda(p.V))
    Yt, dlt, dst = F.fast_sum_oracle(p.X, p.windows, p.kernel, p.ell, p.sigma, p.V, p.n, periods=T, mode=coef,
                                     want_derivs=True)
    assert relerr(Y.cpu().numpy(), Yt) < 1e-10
    for w in range(p.P):
        assert relerr(dl[w].cpu().numpy(), dlt[w]) < 1e-10
        assert relerr(ds[w].cpu().numpy(), dst[w]) < 1e-10


def test_matern_vs_direct_at_stated_estimate(A):
    """Matern-1/2 has no near-field correction: the error against the direct sum
    is at the level of the plan's own a-priori estimate (~1e-2 at n = 64)."""
    p = WL.derivative_c3(N=20000, kernel=WL.MATERN12)
    _say("matern vs direct")
    plan = make_plan(A, p)
    Y = plan.matvec(cuda(p.V)).cpu().numpy()
    rows = np.random.default_rng(3).choice(p.N, 256, replace=False)
    Yo = oracle_direct(p.X, p.windows, p.kernel, p.ell, p.sigma, p.V, rows=rows)
    err = relerr(Y[rows], Yo)
    print("matern rel err vs direct %.3e, estimate %.3e" % (err, plan.query()["err_estimate"]))
    assert err < 5e-2


def test_derivative_is_fd_of_fast_operator(A):
    """Central differences (h = 1e-6) of the FP64 fast product in l_w and sigma_w,
    with the torus frozen, equal the derivative products."""
    p = WL.small_problem(600, 6, MIXED, seed=203, R=2, n=32, m=6)
    _say("fd of fast operator")
    plan = make_plan(A, p)
    V = cuda(p.V)
    _, dl, ds = plan.dmatvec(V)
    h = 1e-6
    for w in range(p.P):
        for which, ref in (("ell", dl), ("sigma", ds)):
            ep, em = p.ell.copy(), p.ell.copy()
            sp, sm = p.sigma.copy(), p.sigma.copy()
            if which == "ell":
                ep[w] += h
                em[w] -= h
            else:
                sp[w] += h
                sm[w] -= h
            plan.update_params(ep, sp)
            yp = plan.matvec(V).cpu().numpy()
            plan.update_params(em, sm)
            ym = plan.matvec(V).cpu().numpy()
            fd = (yp - ym) / (2 * h)
            assert relerr(fd, ref[w].cpu().numpy()) < 1e-7, (which, w)
    plan.update_params(p.ell, p.sigma)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_vjp_vs_oracle(A, prec, tol):
    p = WL.small_problem(700, 6, MIXED, seed=204, R=3, n=32, m=6)
    G = np.random.default_rng(205).standard_normal(p.V.shape)
    _say("vjp %s" % prec)
    gV, gl, gs = make_plan(A, p, prec).vjp(cuda(p.V), cuda(G))
    gVo, glo, gso = oracle_vjp(p.X, p.windows, p.kernel, p.ell, p.sigma, p.V, G)
    assert relerr(gV.cpu().numpy(), gVo) < tol
    print("vjp %s: grad_ell rel %s grad_sigma rel %s" % (prec, np.abs(gl.cpu().numpy() / glo - 1),
                                                        np.abs(gs.cpu().numpy() / gso - 1)))
    np.testing.assert_allclose(gl.cpu().numpy(), glo, rtol=tol)
    np.testing.assert_allclose(gs.cpu().numpy(), gso, rtol=tol)


def test_vjp_scalars_equal_interpolation_inner_products(A):
    """<G, dY/dl_w> from dmatvec equals the Fourier-domain vjp scalar (same operator)."""
    p = WL.small_problem(500, 6, MIXED, seed=206, R=2, n=32, m=6)
    G = np.random.default_rng(207).standard_normal(p.V.shape)
    _say("vjp consistency")
    plan = make_plan(A, p)
    _, dl, ds = plan.dmatvec(cuda(p.V))
    _, gl, gs = plan.vjp(cuda(p.V), cuda(G))
    for w in range(p.P):
        assert gl[w].item() == pytest.approx(float(np.sum(G * dl[w].cpu().numpy())), rel=1e-11)
        assert gs[w].item() == pytest.approx(float(np.sum(G * ds[w].cpu().numpy())), rel=1e-11)


def test_autograd_loss_vKv(A):
    """Backward of L = v^T K v: dL/dv = 2 K v, dL/dl_w = v^T dK/dl_w v; central FD in FP64."""
    p = WL.small_problem(500, 6, MIXED, seed=208, R=1, n=32, m=6)
    _say("autograd")
    plan = make_plan(A, p)
    v = cuda(p.V[:, 0]).requires_grad_(True)
    ell = torch.tensor(p.ell, dtype=torch.float64, device="cuda", requires_grad=True)
    sig = torch.tensor(p.sigma, dtype=torch.float64, device="cuda", requires_grad=True)
    y = A.KernelMatvec.apply(v, ell, sig, plan)
    loss = torch.dot(v, y)
    loss.backward()
    Ko = oracle_direct(p.X, p.windows, p.kernel, p.ell, p.sigma, p.V)[:, 0]
    np.testing.assert_allclose(v.grad.cpu().numpy(), 2 * Ko, rtol=1e-8, atol=1e-8 * np.abs(Ko).max())
    _, dlo, dso = oracle_direct(p.X, p.windows, p.kernel, p.ell, p.sigma, p.V, want_derivs=True)
    np.testing.assert_allclose(ell.grad.cpu().numpy(), [p.V[:, 0] @ dlo[w][:, 0] for w in range(p.P)], rtol=1e-8)
    np.testing.assert_allclose(sig.grad.cpu().numpy(), [p.V[:, 0] @ dso[w][:, 0] for w in range(p.P)], rtol=1e-8)
    # central differences of the fast operator itself
    h = 1e-6
    with torch.no_grad():
        for w in range(p.P):
            e = torch.zeros_like(ell)
            e[w] = h
            lp = torch.dot(v, A.KernelMatvec.apply(v, ell + e, sig, plan)).item()
            lm = torch.dot(v, A.KernelMatvec.apply(v, ell - e, sig, plan)).item()
            assert (lp - lm) / (2 * h) == pytest.approx(ell.grad[w].item(), rel=1e-6)


def _batch_problems(seed=301, count=6):
    rng = np.random.default_rng(seed)
    probs = []
    for i in range(count):
        N = int(rng.integers(300, 3000))
        dims = [int(d) for d in rng.integers(1, 4, size=int(rng.integers(1, 4)))]
        D = sum(dims)
        wins, s = [], 0
        for d in dims:
            wins.append(list(range(s, s + d)))
            s += d
        X = rng.uniform(-0.25, 0.25, size=(N, D))
        V = rng.standard_normal((N, 4))
        probs.append(WL.Problem("b%d" % i, X, V, wins, rng.uniform(0.08, 0.3, len(wins)), np.ones(len(wins)),
                                WL.GAUSSIAN, n=32, m=4))
    return probs


@pytest.mark.parametrize("R", [1, 4])
@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("fp64", 1e-6)])
def test_batch_graph_matches_plans_and_oracle(A, prec, tol, R):
    probs = _batch_problems()
    for p in probs:
        p.V = np.ascontiguousarray(p.V[:, :R])
    _say("batch %s R=%d" % (prec, R))
    plans = [make_plan(A, p, prec) for p in probs]
    B = A.Batch(plans, R=R)
    B.set_inputs([cuda(p.V) for p in probs])
    B.launch()
    torch.cuda.synchronize()
    first = [y.cpu().numpy().copy() for y in B.outputs()]
    for rep in range(3):
        B.launch()
        torch.cuda.synchronize()
        for y0, y in zip(first, B.outputs()):
            assert relerr(y.cpu().numpy(), y0) < 1e-6
    B.run_eager()
    torch.cuda.synchronize()
    for p, pl, y in zip(probs, plans, B.outputs()):
        yi = pl.matvec(cuda(p.V)).cpu().numpy()
        assert relerr(y.cpu().numpy(), yi) < 1e-6
        Yo = oracle_direct(p.X, p.windows, p.kernel, p.ell, p.sigma, p.V)
        assert relerr(y.cpu().numpy(), Yo) < tol
    B.close()
