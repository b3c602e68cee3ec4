"""GPU parity of the dense-cell spread on hand-placed clusters of points.

The matrix-core spread treats some item shapes specially: an item of two
z-adjacent dense cells runs the rounds before its first upper-cell point
without the extra z-slab, a partial last round runs only the K steps it fills,
and an item holds at most 1024 points (a longer two-cell run is split, and the
second part may start in the upper cell).  Clusters with point counts on and
around the 32-point rounds put every such case into one window; the products
are compared with the FP64 direct sums of the oracle on every row.
"""
import sys

import numpy as np
import pytest

import workloads as WL
from _parity import relerr
from oracle.direct import oracle_direct

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N_OVERSAMPLED_HALF = 32  # bandwidth n; the grid has 2n points per dimension
M = 6                    # 2m = 12 taps: the matrix-core width
ELL = 0.3

# (lower-cell points, upper-cell points) of two-cell items, and single-cell counts
TWO_CELL = [(16, 16), (31, 17), (32, 40), (33, 31), (64, 16), (100, 64), (700, 600)]
ONE_CELL = [16, 32, 47, 64, 96]


def _say(msg):
    print("[gpu-case] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def A():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2404_17344_amd as A
    return A


def _anchors():
    return np.array([[0.0, 0.0, 0.0], [1.0, 1.0, 1.0]])


def _cluster_points(rng, T, nos, lo, cell, count):
    """count points whose grid coordinates lie inside base cell `cell` (per
    dimension, away from the cell faces).  The grid coordinate of x is
    ((x - 0.5) / T + 0.5) nos - lo for points centred on the unit cube, and a
    point's base cell is floor(u) - m + 1."""
    u = np.asarray(cell, dtype=np.float64)[None, :] + (M - 1) + rng.uniform(0.1, 0.9, size=(count, 3))
    return ((u + lo) / nos - 0.5) * T + 0.5


def _problem(A, R, seed=4711):
    rng = np.random.default_rng(seed)
    # the torus period and grid depend only on the extent (the anchors) and l
    probe = A.Plan(np.concatenate([_anchors(), rng.uniform(0, 1, size=(64, 3))]), [[0, 1, 2]], np.array([ELL]),
                   np.array([1.0]), n=N_OVERSAMPLED_HALF, m=M, precision="fp64")
    q = probe.query()
    T, nos = q["T"][0], q["n_os"]
    lo = int(np.floor((-0.5 / T + 0.5) * nos)) - M
    umax = (0.5 / T + 0.5) * nos
    nbase = (int(np.floor(umax)) + M + 1 - lo + 1) - 2 * M + 1
    assert nbase >= 16, nbase
    # z base cell 4k pairs with 4k + 1 inside one 4-cell tile; 4k + 3 has no partner
    bz2, bz1 = 4 * (nbase // 8), 4 * (nbase // 8) + 3
    xy = [(bx, by) for bx in range(2, nbase - 2, 2) for by in range(2, nbase - 2, 2)]
    pts, k = [_anchors(), rng.uniform(0.05, 0.95, size=(80, 3))], 0  # sparse points too
    for nlo, nhi in TWO_CELL:
        bx, by = xy[k]
        k += 1
        pts.append(_cluster_points(rng, T, nos, lo, (bx, by, bz2), nlo))
        pts.append(_cluster_points(rng, T, nos, lo, (bx, by, bz2 + 1), nhi))
    for cnt in ONE_CELL:
        bx, by = xy[k]
        k += 1
        pts.append(_cluster_points(rng, T, nos, lo, (bx, by, bz1), cnt))
    X = np.concatenate(pts)
    V = rng.standard_normal(size=(len(X), R))
    return X, V


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("R", [16, 5])
@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("fp64", 1e-10)])
def test_dense_spread_items_vs_direct(A, prec, tol, R):
    X, V = _problem(A, R)
    _say("spread items %s R=%d N=%d" % (prec, R, len(X)))
    ell, sig = np.array([ELL]), np.array([1.3])
    plan = A.Plan(X, [[0, 1, 2]], ell, sig, n=N_OVERSAMPLED_HALF, m=M, precision=prec)
    clustered = sum(a + b for a, b in TWO_CELL) + sum(ONE_CELL)
    assert plan.query()["dense_points"] >= clustered
    Y, dl, _ = plan.dmatvec(_cuda(V), want_dsigma=False)
    Yo, dlo, _ = oracle_direct(X, [[0, 1, 2]], WL.GAUSSIAN, ell, sig, V, want_derivs=True)
    assert relerr(Y.cpu().numpy(), Yo) < tol
    assert relerr(dl[0].cpu().numpy(), dlo[0]) < tol
