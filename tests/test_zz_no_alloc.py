"""The allocation-free product (addk_matvec_noalloc) against addk_matvec.

Both entry points run the same stage kernels; the allocation-free one takes
its workspace from the library's fixed per-GPU array.  Consecutive calls reuse
that array with different layouts, so the second call of each pair uses a
smaller input (another plan, fewer right-hand sides) on what the first left.
Tolerances: the relative 2-norm per column and the largest element error
relative to the largest |y|, 1e-6 in FP32 (atomic sums of the tile spread
may round in another order) and 1e-12 in FP64.
"""
import ctypes
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


def _noalloc(A, plan, Vt):
    """Call the C ABI directly: Vt is a column-major (R, N) device tensor."""
    lib = A._lib.load()
    R, N = Vt.shape
    out = torch.full((R, plan.N_out), float("nan"), dtype=torch.float64, device="cuda")
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    s = lib.addk_matvec_noalloc(plan.handle, R, Vt.data_ptr(), N, out.data_ptr(), plan.N_out, st)
    return s, out


def _check(y, ref, tol):
    y = y.cpu().numpy()
    ref = ref.cpu().numpy()
    assert np.all(np.isfinite(y))
    for r in range(ref.shape[0]):
        assert np.linalg.norm(y[r] - ref[r]) / np.linalg.norm(ref[r]) <= tol
    assert np.max(np.abs(y - ref)) / np.max(np.abs(ref)) <= tol


def _ref(plan, Vt):
    return plan.matvec(Vt.t()).t().contiguous()


def test_noalloc_matches_matvec(A):
    # plan A: FP32, dense centre (matrix-core spread with per-item blocks), mixed d
    pa = WL.small_problem(100000, 6, [[0, 1, 2], [3, 4], [5]], seed=501, R=5, n=16, m=6, dist="normal")
    plan_a = A.Plan(pa.X, pa.windows, pa.ell, pa.sigma, n=pa.n, m=pa.m, precision="fp32")
    assert plan_a.query()["dense_points"] > 0
    Va = torch.from_numpy(np.ascontiguousarray(pa.V.T)).cuda()
    _say("noalloc plan A fp32 N=1e5 R=5 (first call)")
    s, ya = _noalloc(A, plan_a, Va)
    assert s == 0, A._lib.load().addk_last_error().decode()
    _check(ya, _ref(plan_a, Va), 1e-6)

    # second call, smaller input: plan B, FP64 Matern-1/2 near field, one RHS
    pb = WL.small_problem(5000, 3, [[0, 1, 2]], seed=502, R=1, kernel=WL.MATERN12, n=32, m=6, dist="normal")
    plan_b = A.Plan(pb.X, pb.windows, pb.ell, pb.sigma, kernel="matern12", n=pb.n, m=pb.m, precision="fp64",
                    near_field=True)
    Vb = torch.from_numpy(np.ascontiguousarray(pb.V.T)).cuda()
    _say("noalloc plan B fp64 matern near field N=5000 R=1 (second call)")
    s, yb = _noalloc(A, plan_b, Vb)
    assert s == 0, A._lib.load().addk_last_error().decode()
    _check(yb, _ref(plan_b, Vb), 1e-12)

    # plan A again with fewer RHS, then its own (allocating) product still agrees
    Va2 = Va[:2].contiguous()
    _say("noalloc plan A fp32 R=2 (third call)")
    s, ya2 = _noalloc(A, plan_a, Va2)
    assert s == 0, A._lib.load().addk_last_error().decode()
    ref2 = _ref(plan_a, Va2)
    _check(ya2, ref2, 1e-6)
    _check(ya2, _ref(plan_a, Va2), 1e-6)
    # the same call twice in a row gives the same product
    s, ya3 = _noalloc(A, plan_a, Va2)
    assert s == 0
    _check(ya3, ref2, 1e-6)


def test_noalloc_two_calls_same_plan_fp64(A):
    p = WL.small_problem(30000, 5, [[0, 1, 2], [3, 4]], seed=503, R=4, n=32, m=6, dist="normal")
    plan = A.Plan(p.X, p.windows, p.ell, p.sigma, n=p.n, m=p.m, precision="fp64")
    V = torch.from_numpy(np.ascontiguousarray(p.V.T)).cuda()
    _say("noalloc fp64 N=30000 R=4 then R=1")
    s, y = _noalloc(A, plan, V)
    assert s == 0, A._lib.load().addk_last_error().decode()
    _check(y, _ref(plan, V), 1e-12)
    V1 = V[3:4].contiguous()
    s, y1 = _noalloc(A, plan, V1)
    assert s == 0, A._lib.load().addk_last_error().decode()
    _check(y1, _ref(plan, V1), 1e-12)


def test_noalloc_rejects_oversize(A):
    # 64 RHS on 1e5 points and 3 windows: the FP64 per-window products alone
    # take 2 * 64 * 1e5 * 3 * 8 bytes = 307 MB, beyond the fixed array
    p = WL.small_problem(100000, 6, [[0, 1, 2], [3, 4], [5]], seed=504, R=1, n=16, m=6)
    plan = A.Plan(p.X, p.windows, p.ell, p.sigma, n=p.n, m=p.m, precision="fp32")
    V = torch.zeros((64, p.N), dtype=torch.float64, device="cuda")
    _say("noalloc oversize request")
    s, y = _noalloc(A, plan, V)
    assert s == A._lib.ADDK_ERR_INVALID_ARG
    assert "workspace" in A._lib.load().addk_last_error().decode()
    assert torch.isnan(y).all()  # nothing was written
