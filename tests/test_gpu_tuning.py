"""GPU tests of the tuning knobs and the tuning cache (addk_plan_set_knobs,
addk_plan_autotune, addk_tune_cache_lookup / _clear)."""
import sys

import numpy as np
import pytest

import workloads as WL
from _parity import relerr

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


@pytest.mark.parametrize("m", [4, 6])
def test_spread_split_same_products(A, m):
    """The split dense-spread shape (M tiles over several blocks per item) sums the
    same points in the same order per accumulator tile, so the FP32 products
    agree with the one-block shape to rounding (the two are compiled apart and
    may contract multiply-adds differently; measured: identical at m = 4,
    ~1e-8 at m = 6), K V and dK/dl V."""
    p = WL.additive_c2(N=100000, R=16)
    _say("spread split m=%d" % m)
    mk = lambda: A.Plan(p.X, p.windows, p.ell, p.sigma, n=64, m=m, precision="fp32")  # noqa: E731
    p1, p2 = mk(), mk()
    assert p1.query()["dense_points"] > 50000
    p1.set_knobs(A.ADDK_KNOB_ALL_MFMA)
    p2.set_knobs(A.ADDK_KNOB_ALL_MFMA | A.ADDK_KNOB_SPREAD_SPLIT)
    assert p2.query()["knobs"] == A.ADDK_KNOB_ALL
    V = cuda(p.V)
    Y1, d1, _ = p1.dmatvec(V, want_dsigma=False)
    Y2, d2, _ = p2.dmatvec(V, want_dsigma=False)
    assert relerr(Y2.cpu().numpy(), Y1.cpu().numpy()) < 1e-6
    for w in range(p.P):
        assert relerr(d2[w].cpu().numpy(), d1[w].cpu().numpy()) < 1e-6


def test_tune_cache(A):
    """An autotune records its choice under the plan's shape; an untuned plan of the
    same shape finds it (and runs with it: same bits as the tuned plan), other R
    do not; clearing forgets it."""
    p = WL.additive_c2(N=60000, seed=11, R=8)
    _say("tune cache")
    A.tune_cache_clear()
    mk = lambda: A.Plan(p.X, p.windows, p.ell, p.sigma, n=64, m=6, precision="fp32")  # noqa: E731
    pa, pb = mk(), mk()
    assert pb.cached_knobs(8, 2) is None
    k = pa.autotune(R=8, nout=2, reps=1)
    assert 0 <= k <= A.ADDK_KNOB_ALL
    assert pb.cached_knobs(8, 2) == k
    assert pb.cached_knobs(4, 2) is None and pb.cached_knobs(8, 1) is None
    assert not pb.query()["tuned"]
    V = cuda(p.V)
    Ya, da, _ = pa.dmatvec(V, want_dsigma=False)
    Yb, db, _ = pb.dmatvec(V, want_dsigma=False)
    assert np.array_equal(Ya.cpu().numpy(), Yb.cpu().numpy())
    assert np.array_equal(da.cpu().numpy(), db.cpu().numpy())
    A.tune_cache_clear()
    assert pb.cached_knobs(8, 2) is None


def test_set_knobs_rejects(A):
    p = WL.small_problem(300, 3, [[0, 1, 2]], seed=5, R=1, n=16, m=4)
    pl = A.Plan(p.X, p.windows, p.ell, p.sigma, n=16, m=4)
    with pytest.raises(A.AddkError):
        pl.set_knobs((A.ADDK_KNOB_ALL | A.ADDK_KNOB_SPARSE_ATOMIC) + 1)


@pytest.mark.parametrize("prec,tol", [("fp32", 5e-6), ("fp64", 1e-12)])
def test_sparse_atomic_spread_same_products(A, prec, tol):
    """The atomic per-tile sparse spread (ADDK_KNOB_SPARSE_ATOMIC) against the
    output-tile spread: the same sums in another order (FP32: the two orders
    round apart by ~1.4e-6 of max |y|, both within the FP32 bound of the exact
    product)."""
    p = WL.additive_c2(N=30000, seed=21, R=5)
    _say("sparse atomic %s" % prec)
    mk = lambda: A.Plan(p.X, p.windows, p.ell, p.sigma, n=64, m=6, precision=prec)  # noqa: E731
    p1, p2 = mk(), mk()
    assert p1.query()["tile_points"] > 1000
    p2.set_knobs(A.ADDK_KNOB_ALL_MFMA | A.ADDK_KNOB_SPARSE_ATOMIC)
    V = cuda(p.V)
    Y1, d1, _ = p1.dmatvec(V, want_dsigma=False)
    Y2, d2, _ = p2.dmatvec(V, want_dsigma=False)
    assert relerr(Y2.cpu().numpy(), Y1.cpu().numpy()) < tol
    for w in range(p.P):
        assert relerr(d2[w].cpu().numpy(), d1[w].cpu().numpy()) < tol
