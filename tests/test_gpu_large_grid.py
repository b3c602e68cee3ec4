"""GPU parity on 256-point oversampled grids (n up to 128): the line FFTs then
run half as many lines per block.  Against the brute-force trigonometric sum
of eq. (6) (FP64, same torus and coefficients), against the direct sum (FP64
and FP32), in a batch that mixes grid sizes, and for the near-field corrected
Matern-1/2 workload, whose close-pair radius shrinks with 1/n."""
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


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("kernel", [WL.GAUSSIAN, WL.MATERN12])
@pytest.mark.parametrize("wins", [[[0]], [[0, 1]]])
def test_fp64_vs_trigonometric_sum_n128(A, kernel, wins):
    """n = 128, n_os = 256: equal to the brute-force sum of eq. (6) up to the
    window error (1e-10), for one- and two-dimensional windows."""
    p = WL.small_problem(500, 2, wins, seed=401, R=2, n=128, m=6, kernel=kernel, ell=[0.03], sigma=[0.9])
    _say("n128 trig-sum kernel=%d wins=%s" % (kernel, wins))
    plan = A.Plan(p.X, p.windows, p.ell, p.sigma, kernel=p.kernel, n=128, m=6, precision="fp64")
    assert plan.query()["n_os"] == 256
    T = plan.query()["T"]
    Y = plan.matvec(cuda(p.V)).cpu().numpy()
    Yt = F.fast_sum_oracle(p.X, p.windows, kernel, p.ell, p.sigma, p.V, 128, periods=T)
    assert relerr(Y, Yt) < 1e-10


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_d3_small_length_scale_vs_direct(A, prec, tol):
    """A d = 3 window with l = 0.02 (too small for n = 64: eta < 1 there) and a
    d = 2 window, N = 20000 N(0,1) points: K V and dK/dl V against the direct sum."""
    p = WL.small_problem(20000, 5, [[0, 1, 2], [3, 4]], seed=402, R=3, n=128, m=6, ell=[0.02, 0.03],
                         sigma=[1.0, 0.7], dist="gauss")
    _say("n128 d3 small l %s" % prec)
    plan = A.Plan(p.X, p.windows, p.ell, p.sigma, n=128, m=6, precision=prec)
    Y, dl, _ = plan.dmatvec(cuda(p.V), want_dsigma=False)
    rows = np.sort(np.random.default_rng(4).choice(p.N, 200, replace=False))
    Yo, dlo, _ = oracle_direct(p.X, p.windows, p.kernel, p.ell, p.sigma, p.V, rows=rows, want_derivs=True)
    assert relerr(Y.cpu().numpy()[rows], Yo) < tol
    for w in range(2):
        assert relerr(dl[w].cpu().numpy()[rows], dlo[w]) < tol


def test_batch_mixing_grid_sizes(A):
    """One batch holding plans on 64- and 256-point grids: the graph replays
    equal each plan's own product (the batch runs every window with the
    smaller line groups)."""
    q1 = WL.small_problem(3000, 3, [[0, 1, 2]], seed=403, R=2, n=32, m=6)
    q2 = WL.small_problem(4000, 3, [[0, 1], [2]], seed=404, R=2, n=128, m=6, ell=[0.03, 0.05], sigma=[1.0, 1.0])
    plans = [A.Plan(q.X, q.windows, q.ell, q.sigma, n=q.n, m=6, precision="fp64") for q in (q1, q2)]
    own = [pl.matvec(cuda(q.V)).cpu().numpy() for pl, q in zip(plans, (q1, q2))]
    _say("batch mixing grid sizes")
    B = A.Batch(plans, R=2)
    B.set_inputs([cuda(q.V) for q in (q1, q2)])
    for _ in range(2):
        B.launch()
        torch.cuda.synchronize()
        for y, y0 in zip(B.outputs(), own):
            assert relerr(y.cpu().numpy(), y0) < 1e-12
    B.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_near_field_matern_n128(A, prec):
    """The derivative workload (N = 1e5, three d = 3 windows) with the
    near-field correction at n = 128: within 1e-5 of the direct sums."""
    p = WL.derivative_c3(N=100000, kernel=WL.MATERN12)
    _say("near field n128 %s" % prec)
    plan = A.Plan(p.X, p.windows, p.ell, p.sigma, kernel="matern12", n=128, m=6, precision=prec, near_field=True)
    Y, dl, ds = plan.dmatvec(cuda(p.V))
    rows = np.sort(np.random.default_rng(8).choice(p.N, 96, replace=False))
    Yo, dlo, dso = oracle_direct(p.X, p.windows, WL.MATERN12, p.ell, p.sigma, p.V, rows=rows, want_derivs=True)
    assert relerr(Y.cpu().numpy()[rows], Yo) < 1e-5
    for w in range(3):
        assert relerr(dl[w].cpu().numpy()[rows], dlo[w]) < 1e-5
        assert relerr(ds[w].cpu().numpy()[rows], dso[w]) < 1e-5
