"""GPU parity of plans whose windows are all d = 1, where the interpolation runs
fused with the window sum in the caller's point order (no per-window product
buffer): against the FP64 direct sum, for K V, dK/dl_w V, dK/dsigma_w V, the
vjp's K G and the allocation-free entry point."""
import sys

import numpy as np
import pytest

import workloads as WL
from _parity import relerr
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


D1 = [[0], [1], [2], [3], [4], [5]]


@pytest.mark.parametrize("R", [1, 5, 16, 21])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
@pytest.mark.parametrize("m", [4, 6])
def test_all_d1_dmatvec_vs_direct(A, prec, tol, R, m):
    """Clustered and uniform points (dense cells and sparse tiles alike go through
    the fused kernel), six d = 1 windows."""
    rng = np.random.default_rng(120 + R)
    X = np.concatenate([rng.normal(0, 0.03, size=(4000, 6)), rng.uniform(-0.25, 0.25, size=(1500, 6))])
    V = rng.standard_normal((X.shape[0], R))
    ell = np.linspace(0.05, 0.3, 6)
    sig = np.linspace(0.5, 1.5, 6)
    _say("all-d1 %s R=%d m=%d" % (prec, R, m))
    pl = A.Plan(X, D1, ell, sig, n=64, m=m, precision=prec)
    Y, dl, ds = pl.dmatvec(cuda(V))
    rows = np.arange(0, X.shape[0], 7)
    Yo, dlo, dso = oracle_direct(X, D1, WL.GAUSSIAN, ell, sig, V, rows=rows, want_derivs=True)
    # m = 4 is window-limited: up to ~1e-6 of max |y| here (the smallest l = 0.05)
    t = tol if m == 6 else max(tol, 5e-6)
    assert relerr(Y.cpu().numpy()[rows], Yo) < t
    for w in range(6):
        assert relerr(dl[w].cpu().numpy()[rows], dlo[w]) < t
        assert relerr(ds[w].cpu().numpy()[rows], dso[w]) < t
    Yk = pl.matvec(cuda(V)).cpu().numpy()
    assert relerr(Yk, Y.cpu().numpy()) < (1e-14 if prec == "fp64" else 1e-6)


def test_all_d1_vjp_and_noalloc(A):
    rng = np.random.default_rng(130)
    X = rng.uniform(-0.25, 0.25, size=(3000, 6))
    V = rng.standard_normal((3000, 3))
    G = rng.standard_normal((3000, 3))
    ell = np.full(6, 0.1)
    sig = np.ones(6)
    _say("all-d1 vjp + noalloc")
    pl = A.Plan(X, D1, ell, sig, n=64, m=6, precision="fp64")
    gV, gl, gs = pl.vjp(cuda(V), cuda(G))
    gVo, glo, gso = oracle_vjp(X, D1, WL.GAUSSIAN, ell, sig, V, G)
    assert relerr(gV.cpu().numpy(), gVo) < 1e-10
    np.testing.assert_allclose(gl.cpu().numpy(), glo, rtol=1e-9)
    out = torch.empty((3, 3000), dtype=torch.float64, device="cuda")
    Yn = pl.matvec_noalloc(cuda(V), out).cpu().numpy()
    assert relerr(Yn, oracle_direct(X, D1, WL.GAUSSIAN, ell, sig, V)) < 1e-10
