"""GPU parity of the global sensitivity indices (Algorithm 1) against the oracle."""
import sys

import numpy as np
import pytest

import workloads as WL
from oracle import fourier as F

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


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-8), ("fp32", 1e-5)])
def test_gsi_matches_oracle(A, prec, tol):
    """Per-window variance contributions and the normalised indices of mixed
    d = 3, 2, 1 windows, against brute-force S(k, W) on the same torus."""
    wins = [[0, 1, 2], [3, 4], [5]]
    p = WL.small_problem(3000, 6, wins, seed=81, R=1, ell=[0.12, 0.2, 0.1], sigma=[1.0, 0.7, 1.3], n=32, m=6)
    _say("gsi %s" % prec)
    plan = A.Plan(p.X, p.windows, p.ell, p.sigma, n=p.n, m=p.m, precision=prec)
    T = plan.query()["T"]
    v = torch.from_numpy(p.V[:, 0].copy()).cuda()
    th = plan.gsi_theta(v)
    tho = F.gsi_theta_oracle(p.X, p.windows, F.GAUSSIAN, p.ell, p.V[:, 0], p.n, periods=T)
    for w in range(len(wins)):
        scale = tho[w].sum()
        assert np.max(np.abs(th[w] - tho[w])) <= tol * scale, (w, th[w], tho[w])
    rho = plan.gsi(v)
    rho_o = F.gsi_oracle(p.X, p.windows, F.GAUSSIAN, p.ell, p.V[:, 0], p.n, periods=T)
    assert set(rho) == set(rho_o)
    for k in rho:
        assert abs(rho[k] - rho_o[k]) <= tol
    assert sum(rho.values()) == pytest.approx(1.0, rel=1e-12)


def test_gsi_full_size_additive(A):
    """The additive 1e5-point, three d = 3 window workload (FP32): indices sum
    to one, are nonnegative and cover every nonempty subset of every window;
    the per-window totals agree with the FP64 path."""
    p = WL.additive_c2(N=100000)
    _say("gsi additive N=1e5")
    v = torch.from_numpy(p.V[:, 0].copy()).cuda()
    r32 = A.Plan(p.X, p.windows, p.ell, p.sigma, n=64, m=6, precision="fp32").gsi_theta(v)
    r64 = A.Plan(p.X, p.windows, p.ell, p.sigma, n=64, m=6, precision="fp64").gsi_theta(v)
    for w in range(p.P):
        assert np.max(np.abs(r32[w] - r64[w])) <= 1e-5 * r64[w].sum()
    rho = A.Plan(p.X, p.windows, p.ell, p.sigma, n=64, m=6, precision="fp64").gsi(v)
    assert len(rho) == 3 * 7
    assert all(r >= 0 for r in rho.values())
    assert sum(rho.values()) == pytest.approx(1.0, rel=1e-12)
