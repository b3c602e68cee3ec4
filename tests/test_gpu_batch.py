"""GPU parity of the batched products at the full size of the uneven-batch
workload, and of the autotuner (kernel-variant choice by measurement)."""
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


def test_uneven_batch_full_size_graph_autotuned(A):
    """64 problems (N from 5e3 to 2e5, 1-5 windows of d in {1, 2, 3}, 3e6 points in
    all), 8 RHS each, FP32, bandwidth per problem from the error model at 1e-5,
    m = 4.  The autotuned graph replays agree with each other and with eager
    launches, and every problem agrees with the FP64 direct sum on sampled rows."""
    probs = WL.batched_c4()
    _say("uneven batch: %d problems, %d points" % (len(probs), sum(p.N for p in probs)))
    plans = []
    for p in probs:
        n = A.choose_n_for(p.X, p.windows, p.ell, m=4, oversampling=2.0, tol=1e-5)
        plans.append(A.Plan(p.X, p.windows, p.ell, p.sigma, n=n, m=4, precision="fp32"))
    B = A.Batch(plans, R=8)
    B.set_inputs([cuda(p.V) for p in probs])
    _say("uneven batch: autotune")
    knobs = B.autotune(reps=2)
    assert 0 <= knobs <= A.ADDK_KNOB_ALL
    # Replays and eager runs agree to FP32 rounding (within the FP32 tolerance):
    # the d = 1, 2 spreads sum with atomics, so the FP32 summation order of
    # those windows varies run to run (d = 3 windows are bitwise reproducible).  A graph that reused stale
    # buffers would be off by O(1).
    B.launch()
    torch.cuda.synchronize()
    first = [y.cpu().numpy().copy() for y in B.outputs()]
    for _ in range(2):
        B.launch()
        torch.cuda.synchronize()
        for y0, y in zip(first, B.outputs()):
            assert relerr(y.cpu().numpy(), y0) < 1e-5
    B.run_eager()
    torch.cuda.synchronize()
    outs = [y.cpu().numpy() for y in B.outputs()]
    for y0, y in zip(first, outs):
        assert relerr(y, y0) < 1e-5
    _say("uneven batch: oracle rows")
    rng = np.random.default_rng(44)
    for p, y in zip(probs, outs):
        rows = np.sort(rng.choice(p.N, 48, replace=False))
        Yo = oracle_direct(p.X, p.windows, p.kernel, p.ell, p.sigma, p.V, rows=rows)
        assert relerr(y[rows], Yo) < 1e-5, p.name
    B.close()


@pytest.mark.parametrize("R,nout", [(16, 2), (4, 1)])
def test_plan_autotune_keeps_results(A, R, nout):
    """Whatever kernel variants the tuner picks, the products stay within the FP32
    tolerance of the FP64 path."""
    p = WL.additive_c2(N=40000, seed=9, R=R)
    _say("plan autotune R=%d nout=%d" % (R, nout))
    mk = lambda prec: A.Plan(p.X, p.windows, p.ell, p.sigma, n=64, m=6, precision=prec)  # noqa: E731
    p32, p64 = mk("fp32"), mk("fp64")
    k = p32.autotune(R=R, nout=nout, reps=2)
    q = p32.query()
    assert q["tuned"] and q["knobs"] == k and 0 <= k <= A.ADDK_KNOB_ALL
    assert 0 <= p64.autotune(R=R, nout=nout, reps=1) <= A.ADDK_KNOB_ALL
    V = cuda(p.V)
    Y32, dl32, _ = p32.dmatvec(V, want_dsigma=False)
    Y64, dl64, _ = p64.dmatvec(V, want_dsigma=False)
    assert relerr(Y32.cpu().numpy(), Y64.cpu().numpy()) < 1e-5
    for w in range(p.P):
        assert relerr(dl32[w].cpu().numpy(), dl64[w].cpu().numpy()) < 1e-5
    A.tune_cache_clear()  # the choices above stay with these plans only
