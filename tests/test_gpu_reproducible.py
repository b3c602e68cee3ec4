"""Bitwise reproducible FP32 products (no atomics on the d = 3 path).

The points are placed by a stable sort, the dense cells' spread blocks are
summed by a fixed-order gather, the sparse cells are spread by output tiles
(each grid value written once), and the FFTs, interpolations and window sums
have no atomics: two plans built from the same points, repeated products and
graph replays give identical bits.  Workload: the additive case (N = 1e5,
three d = 3 windows of N(0,1) features min-max scaled, n = 64, m = 6)."""
import sys

import numpy as np
import pytest

import workloads as WL

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


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("R", [1, 4, 16])
def test_products_bitwise_reproducible(A, R, prec):
    p = WL.additive_c2(N=100000, R=R)
    _say("reproducible %s R=%d" % (prec, R))
    mk = lambda: A.Plan(p.X, p.windows, p.ell, p.sigma, n=p.n, m=p.m, precision=prec)  # noqa: E731
    p1, p2 = mk(), mk()
    V = torch.from_numpy(np.ascontiguousarray(p.V)).cuda()
    outs = []
    for pl in (p1, p2, p1):
        Y, dl, _ = pl.dmatvec(V, want_dsigma=False)
        outs.append((Y.cpu().numpy(), dl.cpu().numpy()))
    for Y, dl in outs[1:]:
        assert np.array_equal(Y, outs[0][0])
        assert np.array_equal(dl, outs[0][1])
    K1 = p1.matvec(V).cpu().numpy()
    assert np.array_equal(p2.matvec(V).cpu().numpy(), K1)
    # graph replays of a batch holding the plan
    B = A.Batch([p1], R=R)
    B.set_inputs([V])
    reps = []
    for _ in range(3):
        B.launch()
        torch.cuda.synchronize()
        reps.append(B.outputs()[0].cpu().numpy().copy())
    for y in reps[1:]:
        assert np.array_equal(y, reps[0])
    assert np.array_equal(reps[0], K1)
    B.close()
