"""GPU parity of the Matern-3/2 kernel (1 + a r) e^{-a r}, a = sqrt(3)/l, the
further kernel of the kernel-extension subsection (ADDK_MATERN32).

* Plain Fourier method: against the brute-force trigonometric sum of eq. (6)
  with the plan's own torus and coefficients (analytic and sampled), FP64 to
  1e-10; against the direct sum at the level of the truncated series.
* Near-field corrected (ADDK_NEAR_FIELD): against the oracle of the same
  corrected method (FP64, 1e-8), and against the direct sums at the size of
  the derivative workload (N = 1e5, three d = 3 windows, n = 64): K v,
  dK/dl_w v and dK/dsigma_w v within 1e-5 in FP64 and FP32; the vjp against
  the oracle's.
"""
import sys

import numpy as np
import pytest

import workloads as WL
from _parity import inner_err, relerr
from oracle import fourier as F
from oracle import nearfield as NF
from oracle.direct import oracle_direct

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

M32 = WL.MATERN32
MIXED = [[0, 1, 2], [3, 4], [5]]


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


def _plan(A, p, prec="fp64", **kw):
    return A.Plan(p.X, p.windows, p.ell, p.sigma, kernel="matern32", n=p.n, m=p.m, precision=prec, **kw)


@pytest.mark.parametrize("coef", ["analytic", "sampled"])
def test_matern32_vs_trigonometric_sum(A, coef):
    p = WL.small_problem(500, 6, MIXED, seed=601, R=2, n=32, m=6, kernel=M32)
    _say("matern32 trig sum %s" % coef)
    plan = _plan(A, p, coef=coef)
    q = plan.query()
    for w, feats in enumerate(p.windows):
        _, L = F.window_geometry(p.X[:, feats])
        assert q["T"][w] == pytest.approx(F.torus_period_auto(M32, L, p.ell[w], p.n), rel=1e-13)
    Y, dl, ds = plan.dmatvec(cuda(p.V))
    Yt, dlt, dst = F.fast_sum_oracle(p.X, p.windows, M32, p.ell, p.sigma, p.V, p.n, periods=q["T"], mode=coef,
                                     want_derivs=True)
    assert relerr(Y.cpu().numpy(), Yt) < 1e-10
    for w in range(p.P):
        assert relerr(dl[w].cpu().numpy(), dlt[w]) < 1e-10
        assert relerr(ds[w].cpu().numpy(), dst[w]) < 1e-10


def test_matern32_plain_vs_direct(A):
    """Without the near field the truncated series of the r^3-smooth kernel
    stays near 1e-3 of the direct sum at n = 64."""
    p = WL.derivative_c3(N=20000, kernel=M32)
    _say("matern32 plain vs direct")
    plan = _plan(A, p)
    Y = plan.matvec(cuda(p.V)).cpu().numpy()
    rows = np.random.default_rng(5).choice(p.N, 256, replace=False)
    Yo = oracle_direct(p.X, p.windows, M32, p.ell, p.sigma, p.V, rows=rows)
    err = relerr(Y[rows], Yo)
    print("matern32 plain rel err vs direct %.3e, estimate %.3e" % (err, plan.query()["err_estimate"]))
    assert err < 2e-2


@pytest.mark.parametrize("R", [3, 1])
def test_matern32_near_field_vs_corrected_oracle(A, R):
    p = WL.small_problem(1500, 6, [[0], [1, 2], [3, 4, 5]], seed=602, R=R, ell=[0.05, 0.1, 0.2],
                         sigma=[1.0, 0.8, 0.6], kernel=M32, n=32, m=6)
    _say("matern32 near field vs corrected oracle R=%d" % R)
    plan = _plan(A, p, near_field=True)
    Y, dl, ds = plan.dmatvec(cuda(p.V))
    Yo, dlo, dso = NF.nearfield_fast_sum_oracle(p.X, p.windows, p.ell, p.sigma, p.V, p.n, want_derivs=True,
                                                kernel=M32)
    errs = [relerr(Y.cpu().numpy(), Yo)] + [relerr(dl[w].cpu().numpy(), dlo[w]) for w in range(3)] + \
        [relerr(ds[w].cpu().numpy(), dso[w]) for w in range(3)]
    print("matern32 near field vs corrected oracle R=%d: %s" % (R, " ".join("%.2e" % e for e in errs)))
    assert max(errs) < 1e-8


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_matern32_near_field_derivative_workload(A, prec):
    """N = 1e5, three d = 3 windows, l = (0.05, 0.1, 0.2), n = 64, m = 6: the
    corrected products within 1e-5 of the direct sums on sampled rows."""
    p = WL.derivative_c3(kernel=M32)
    _say("matern32 near field c3 %s" % prec)
    plan = _plan(A, p, prec, near_field=True)
    Y, dl, ds = plan.dmatvec(cuda(p.V))
    rows = np.sort(np.random.default_rng(9).choice(p.N, 128, replace=False))
    Yo, dlo, dso = oracle_direct(p.X, p.windows, M32, p.ell, p.sigma, p.V, rows=rows, want_derivs=True)
    errs = [relerr(Y.cpu().numpy()[rows], Yo)] + [relerr(dl[w].cpu().numpy()[rows], dlo[w]) for w in range(3)] + \
        [relerr(ds[w].cpu().numpy()[rows], dso[w]) for w in range(3)]
    print("matern32 near field c3 %s: %s" % (prec, " ".join("%.2e" % e for e in errs)))
    assert max(errs) < 1e-5


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_matern32_near_field_vjp(A, prec):
    """Gradients of <G, K V> against the direct sums; the scalar gradients
    <G, dK/dl_w V> are held on the scale ||G|| ||dK/dl_w V|| (they may cancel)."""
    p = WL.small_problem(4000, 6, MIXED, seed=603, R=3, ell=[0.06, 0.1, 0.15], sigma=[1.0, 0.7, 1.2],
                         kernel=M32, n=64, m=6, dist="normal")
    G = np.random.default_rng(604).standard_normal(p.V.shape)
    _say("matern32 near field vjp %s" % prec)
    gV, gl, gs = _plan(A, p, prec, near_field=True).vjp(cuda(p.V), cuda(G))
    gVo = oracle_direct(p.X, p.windows, M32, p.ell, p.sigma, G)
    _, dlo, dso = oracle_direct(p.X, p.windows, M32, p.ell, p.sigma, p.V, want_derivs=True)
    e = relerr(gV.cpu().numpy(), gVo)
    nG = np.linalg.norm(G)
    el = [inner_err(gl[w].item(), np.sum(G * dlo[w]), nG, np.linalg.norm(dlo[w])) for w in range(3)]
    es = [inner_err(gs[w].item(), np.sum(G * dso[w]), nG, np.linalg.norm(dso[w])) for w in range(3)]
    print("matern32 vjp %s: grad_V %.2e grad_l %s grad_sigma %s" % (prec, e, el, es))
    assert e < 1e-5
    assert max(el) < 1e-5
    assert max(es) < 1e-5
