"""The derivative workload at its configured size: N = 1e5 points with nine
N(0,1) features min-max scaled, three d = 3 windows, l = (0.05, 0.1, 0.2),
sigma_w = 1, n = 64, m = 6 (seed 17343).

* Gaussian, FP64: K v, dK/dl_w v and dK/dsigma_w v against the direct sums on
  sampled rows (1e-10), and central differences (h = 1e-6) of the GPU product
  in every l_w and sigma_w against the derivative products.
* The backward of L = v^T K v through KernelMatvec (Gaussian FP64, and the
  near-field corrected Matern-1/2 and Matern-3/2 kernels): dL/dv = 2 K v
  against the direct sums on sampled rows; L, dL/dl_w and dL/dsigma_w against
  v^T K v, v^T dK/dl_w v and v^T dK/dsigma_w v over all N^2 pairs
  (tests/golden/c3_quadratic_forms.json, written by the oracle alone);
  central differences of L in l_w, sigma_w (h = 1e-6) and in entries of v.
* The FP32 vjp with one and eight right-hand sides, where the dense-cell
  matrix-core spread, gather and interpolation carry the centre of the data.
"""
import json
import os
import sys

import numpy as np
import pytest

import workloads as WL
from _parity import inner_err, relerr
from oracle.direct import oracle_direct

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "c3_quadratic_forms.json")))
KNAME = {WL.GAUSSIAN: "gaussian", WL.MATERN12: "matern12", WL.MATERN32: "matern32"}


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


def _rows(p, count=128, seed=31):
    """Random rows plus the outermost points of every window (sparse tiles)."""
    out = [np.random.default_rng(seed).choice(p.N, count, replace=False)]
    for feats in p.windows:
        Z = p.X[:, feats]
        r = np.linalg.norm(Z - 0.5 * (Z.min(axis=0) + Z.max(axis=0)), axis=1)
        out.append(np.argsort(r)[-6:])
    return np.unique(np.concatenate(out))


def _plan(A, p, kernel, precision):
    if kernel == WL.GAUSSIAN:
        return A.Plan(p.X, p.windows, p.ell, p.sigma, n=p.n, m=p.m, precision=precision)
    return A.Plan(p.X, p.windows, p.ell, p.sigma, kernel=KNAME[kernel], n=p.n, m=p.m, precision=precision,
                  near_field=True)


def test_c3_gaussian_fp64_products_and_finite_differences(A):
    p = WL.derivative_c3()
    _say("c3 gaussian fp64 dmatvec + FD")
    plan = _plan(A, p, WL.GAUSSIAN, "fp64")
    V = cuda(p.V)
    Y, dl, ds = plan.dmatvec(V)
    Y, dl, ds = Y.cpu().numpy(), dl.cpu().numpy(), ds.cpu().numpy()
    rows = _rows(p)
    Yo, dlo, dso = oracle_direct(p.X, p.windows, p.kernel, p.ell, p.sigma, p.V, rows=rows, want_derivs=True)
    errs = [relerr(Y[rows], Yo)] + [relerr(dl[w][rows], dlo[w]) for w in range(3)] + \
        [relerr(ds[w][rows], dso[w]) for w in range(3)]
    print("c3 fp64 errors Y, dY/dl_w, dY/dsigma_w: %s" % " ".join("%.2e" % e for e in errs))
    assert max(errs) < 1e-10
    h = 1e-6
    for w in range(3):
        for which, ref in (("ell", dl), ("sigma", ds)):
            ep, em, sp, sm = p.ell.copy(), p.ell.copy(), p.sigma.copy(), p.sigma.copy()
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
            e = relerr((yp - ym) / (2 * h), ref[w])
            print("c3 FD %s_%d rel err %.2e" % (which, w, e))
            assert e < 1e-7, (which, w)
    plan.update_params(p.ell, p.sigma)


@pytest.mark.parametrize("kernel,tol", [(WL.GAUSSIAN, 1e-10), (WL.MATERN12, 1e-5), (WL.MATERN32, 1e-5)])
def test_c3_autograd_quadratic_loss(A, kernel, tol):
    p = WL.derivative_c3(kernel=kernel)
    _say("c3 autograd v^T K v kernel=%d" % kernel)
    plan = _plan(A, p, kernel, "fp64")
    gold = GOLD[KNAME[kernel]]["R1"]
    v = cuda(p.V[:, 0]).requires_grad_(True)
    ell = torch.tensor(p.ell, dtype=torch.float64, device="cuda", requires_grad=True)
    sig = torch.tensor(p.sigma, dtype=torch.float64, device="cuda", requires_grad=True)
    loss = torch.dot(v, A.KernelMatvec.apply(v, ell, sig, plan))
    loss.backward()
    gl, gs, gv = ell.grad.cpu().numpy(), sig.grad.cpu().numpy(), v.grad.cpu().numpy()
    rows = _rows(p)
    Ko, dlo, dso = oracle_direct(p.X, p.windows, kernel, p.ell, p.sigma, p.V, rows=rows, want_derivs=True)
    assert relerr(gv[rows], 2 * Ko[:, 0]) < tol
    # the scalars are inner products v^T y: their errors are measured against
    # ||v|| ||y|| (y = K v, dK/dl_w v, dK/dsigma_w v; norms estimated from the
    # oracle's sampled rows), since v^T dK/dl_w v may cancel
    nv = np.linalg.norm(p.V[:, 0])
    scale = np.sqrt(p.N / len(rows))
    nK = scale * np.linalg.norm(Ko)
    nl = [scale * np.linalg.norm(dlo[w]) for w in range(3)]
    ns = [scale * np.linalg.norm(dso[w]) for w in range(3)]
    eL = inner_err(loss.item(), gold["vKv"], nv, nK)
    el = [inner_err(gl[w], gold["vdKdl"][w], nv, nl[w]) for w in range(3)]
    es = [inner_err(gs[w], gold["vdKds"][w], nv, ns[w]) for w in range(3)]
    print("c3 autograd kernel=%d: L %.2e, dL/dl %s, dL/dsigma %s (relative: dL/dl %s)" % (
        kernel, eL, ["%.2e" % e for e in el], ["%.2e" % e for e in es],
        ["%.2e" % (abs(gl[w] / gold["vdKdl"][w] - 1)) for w in range(3)]))
    assert eL < tol
    assert max(el) < tol
    assert max(es) < tol
    h = 1e-6
    rel = lambda a, b: abs(a - b) / abs(b)  # noqa: E731
    with torch.no_grad():
        def L(e, s, vv=v):
            return torch.dot(vv, A.KernelMatvec.apply(vv, e, s, plan)).item()
        for w in range(3):
            e = torch.zeros_like(ell)
            e[w] = h
            fd_l = (L(ell + e, sig) - L(ell - e, sig)) / (2 * h)
            fd_s = (L(ell, sig + e) - L(ell, sig - e)) / (2 * h)
            print("c3 FD of L kernel=%d w=%d: l %.2e sigma %.2e" % (kernel, w, rel(fd_l, gl[w]), rel(fd_s, gs[w])))
            assert fd_l == pytest.approx(gl[w], rel=1e-6)
            assert fd_s == pytest.approx(gs[w], rel=1e-6)
        # L is exactly quadratic in v for the fast operator: central differences
        # of any step are exact up to rounding
        hv = 1e-2
        for i in np.random.default_rng(32).choice(p.N, 4, replace=False):
            ei = torch.zeros_like(v)
            ei[i] = hv
            fd_v = (L(ell, sig, v + ei) - L(ell, sig, v - ei)) / (2 * hv)
            assert fd_v == pytest.approx(gv[i], rel=1e-6, abs=1e-6 * np.abs(gv).max())


@pytest.mark.parametrize("R", [1, 8])
def test_c3_vjp_fp32_dense_kernels(A, R):
    p = WL.derivative_c3()
    V = WL.derivative_c3_rhs(R=R)
    _say("c3 fp32 vjp R=%d" % R)
    plan = _plan(A, p, WL.GAUSSIAN, "fp32")
    q = plan.query()
    assert q["dense_points"] > 0.2 * (q["dense_points"] + q["tile_points"])
    gold = GOLD["gaussian"]["R%d" % R]
    Vc = cuda(V)
    gV, gl, gs = plan.vjp(Vc, Vc)
    gV, gl, gs = gV.cpu().numpy(), gl.cpu().numpy(), gs.cpu().numpy()
    rows = _rows(p)
    Ko, dlo, dso = oracle_direct(p.X, p.windows, p.kernel, p.ell, p.sigma, V, rows=rows, want_derivs=True)
    e = relerr(gV[rows], Ko)
    print("c3 fp32 vjp R=%d grad_V rel err %.2e" % (R, e))
    assert e < 1e-5
    nv = np.linalg.norm(V)
    scale = np.sqrt(p.N / len(rows))
    el = [inner_err(gl[w], gold["vdKdl"][w], nv, scale * np.linalg.norm(dlo[w])) for w in range(3)]
    es = [inner_err(gs[w], gold["vdKds"][w], nv, scale * np.linalg.norm(dso[w])) for w in range(3)]
    print("c3 fp32 vjp R=%d dense share %.2f: dL/dl %s dL/dsigma %s" % (
        R, q["dense_points"] / (q["dense_points"] + q["tile_points"]), ["%.2e" % x for x in el],
        ["%.2e" % x for x in es]))
    assert max(el) < 1e-5
    assert max(es) < 1e-5


def test_autograd_backward_after_a_forward_at_other_parameters(A):
    """Two forwards at different l, then the first one's backward: the graph
    keeps its own parameters (the plan is shared)."""
    p = WL.small_problem(3000, 6, [[0, 1, 2], [3, 4], [5]], seed=209, R=1, n=32, m=6)
    _say("autograd two forwards")
    plan = _plan(A, p, WL.GAUSSIAN, "fp64")

    def grads(ell_vals, other=None):
        v = cuda(p.V[:, 0]).requires_grad_(True)
        ell = torch.tensor(ell_vals, dtype=torch.float64, device="cuda", requires_grad=True)
        sig = torch.tensor(p.sigma, dtype=torch.float64, device="cuda", requires_grad=True)
        loss = torch.dot(v, A.KernelMatvec.apply(v, ell, sig, plan))
        if other is not None:  # a second graph at other parameters, built before the first backward
            v2 = cuda(p.V[:, 0]).requires_grad_(True)
            e2 = torch.tensor(other, dtype=torch.float64, device="cuda", requires_grad=True)
            torch.dot(v2, A.KernelMatvec.apply(v2, e2, sig, plan)).item()
        loss.backward()
        return v.grad.cpu().numpy(), ell.grad.cpu().numpy(), sig.grad.cpu().numpy()

    ref = grads(p.ell)
    mixed = grads(p.ell, other=1.3 * p.ell)
    for a, b in zip(ref, mixed):
        np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-12 * np.abs(b).max())
    np.testing.assert_array_equal(plan.ell, 1.3 * p.ell)  # the plan is back at the last forward's values


def test_batch_follows_update_params(A):
    """A batch holds copies of its plans' descriptors: after update_params on a
    plan, the next launch uses the new l and sigma (and, with the near field,
    the new polynomials)."""
    q1 = WL.small_problem(4000, 5, [[0, 1, 2], [3, 4]], seed=210, R=2, n=32, m=6)
    q2 = WL.small_problem(3000, 3, [[0, 1, 2]], seed=211, R=2, n=32, m=6, kernel=WL.MATERN12, dist="normal")
    p1 = A.Plan(q1.X, q1.windows, q1.ell, q1.sigma, n=32, m=6, precision="fp64")
    p2 = A.Plan(q2.X, q2.windows, q2.ell, q2.sigma, kernel="matern12", n=32, m=6, precision="fp64", near_field=True)
    _say("batch after update_params")
    B = A.Batch([p1, p2], R=2)
    B.set_inputs([cuda(q1.V), cuda(q2.V)])
    B.launch()
    torch.cuda.synchronize()
    p1.update_params(1.2 * q1.ell, 0.7 * q1.sigma)
    p2.update_params(0.8 * q2.ell, 1.5 * q2.sigma)
    for run in (B.launch, B.run_eager):
        run()
        torch.cuda.synchronize()
        own = [p1.matvec(cuda(q1.V)).cpu().numpy(), p2.matvec(cuda(q2.V)).cpu().numpy()]
        for y, y0 in zip(B.outputs(), own):
            assert relerr(y.cpu().numpy(), y0) < 1e-12
    Y1 = oracle_direct(q1.X, q1.windows, WL.GAUSSIAN, 1.2 * q1.ell, 0.7 * q1.sigma, q1.V)
    assert relerr(B.outputs()[0].cpu().numpy(), Y1) < 1e-10
    B.close()
