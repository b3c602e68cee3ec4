"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function declared in include/addk.h, and its host-only helpers agree
with the independent oracle / quadrature."""
import math
import os
import re

import numpy as np
import pytest
from scipy import integrate

from oracle import fourier as F

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2404_17344_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libaddk.so not built")
    return L


def test_every_declared_function_is_exported():
    L = _lib()
    lib = L.load()
    header = open(os.path.join(ROOT, "include", "addk.h")).read()
    names = set(re.findall(r"\b(addk_[a-z_]+)\s*\(", header))
    assert len(names) >= 15
    for name in sorted(names):
        assert hasattr(lib, name), name
    assert set(L._SIGS) == names


def test_status_strings_and_version():
    L = _lib()
    lib = L.load()
    for s in range(6):
        assert len(lib.addk_status_string(s)) > 0
    assert b"gfx950" in lib.addk_version()


@pytest.mark.parametrize("kernel", [F.GAUSSIAN, F.MATERN12])
@pytest.mark.parametrize("L,ell,n", [(0.5, 0.1, 64), (0.5, 0.05, 32), (0.3, 0.2, 16), (0.0, 0.1, 64)])
def test_torus_period_matches_oracle_rule(kernel, L, ell, n):
    import paper_2404_17344_amd as A
    _lib()
    assert A.torus_period(kernel, L, ell, n) == pytest.approx(F.torus_period_auto(kernel, L, ell, n), rel=1e-14)
    if L > 0:
        assert A.torus_period(kernel, L, ell, n, paper_rule=True, dmax=3) == pytest.approx(
            F.torus_period_paper(L, 3), rel=1e-14)


def _kb(z, m, b):
    s = np.sqrt(np.maximum(m * m - z * z, 0.0))
    return np.where(s > 1e-12, np.sinh(b * s) / np.where(s > 1e-12, s, 1.0), b) * m / np.sinh(b * m)


@pytest.mark.parametrize("m,nos", [(4, 64), (6, 128), (6, 64)])
def test_window_transform_matches_adaptive_quadrature(m, nos):
    """Psi(k) = int psi(z) cos(2 pi z k / n_os) dz for the normalised Kaiser-Bessel window."""
    import paper_2404_17344_amd as A
    _lib()
    b = math.pi * (2.0 - 0.5)
    for k in [0, 1, 7, nos // 4, nos // 4 - 1]:
        ref, _ = integrate.quad(lambda z: _kb(z, m, b) * math.cos(2 * math.pi * z * k / nos), -m, m, limit=400,
                                epsabs=1e-14, epsrel=1e-14)
        assert A.window_ft(m, nos, 2.0, k) == pytest.approx(ref, rel=1e-12)


def test_window_transform_close_to_kaiser_bessel_closed_form():
    """The untruncated window's transform is I0(m sqrt(b^2 - (2 pi k / n_os)^2)) up to
    normalisation; truncation changes it only at the window-error level."""
    import paper_2404_17344_amd as A
    from scipy.special import i0
    _lib()
    m, nos = 6, 128
    b = math.pi * 1.5
    norm = math.pi * m / math.sinh(b * m)  # psi = (pi m / sinh(b m)) * sinh(b s) / (pi s)
    for k in [0, 5, 20, 32]:
        closed = norm * i0(m * math.sqrt(b * b - (2 * math.pi * k / nos) ** 2))
        assert A.window_ft(m, nos, 2.0, k) == pytest.approx(closed, rel=1e-9)


def test_helpers_reject_bad_arguments():
    import paper_2404_17344_amd as A
    _lib()
    with pytest.raises(A.AddkError):
        A.torus_period(F.GAUSSIAN, 0.5, -1.0, 64)
    with pytest.raises(A.AddkError):
        A.window_ft(0, 128, 2.0, 0.0)


def test_header_documents_every_entry_point():
    header = open(os.path.join(ROOT, "include", "addk.h")).read()
    for name in ["addk_plan_create", "addk_matvec", "addk_dmatvec", "addk_vjp", "addk_batch_create"]:
        i = header.index(name + "(")
        assert "*/" in header[max(0, i - 1500):i], name  # a comment block precedes the declaration


@pytest.mark.parametrize("ell,tol,d", [(0.1, 1e-5, 2), (0.2, 1e-9, 2), (0.1, 1e-8, 1), (0.05, 1e-6, 1)])
def test_choose_n_meets_tolerance_on_the_trigonometric_sum(ell, tol, d):
    """The bandwidth picked for a tolerance makes the Fourier part of the method
    (the exact trigonometric sum of eq. (6), no window error) accurate to that
    tolerance against the FP64 direct sum, on a small uniform window."""
    import paper_2404_17344_amd as A
    from oracle.direct import oracle_direct
    _lib()
    rng = np.random.default_rng(5)
    N = 300
    X = rng.uniform(-0.25, 0.25, size=(N, d))
    V = rng.standard_normal((N, 1))
    L = float((X.max(axis=0) - X.min(axis=0)).max())
    n, est = A.choose_n(F.GAUSSIAN, L, ell, m=6, oversampling=2.0, tol=tol)
    assert n % 2 == 0 and est <= tol
    assert A.choose_n_for(X, [list(range(d))], [ell], m=6, tol=tol) == n
    Y = F.fast_sum_oracle(X, [list(range(d))], F.GAUSSIAN, [ell], [1.0], V, n)
    Yd = oracle_direct(X, [list(range(d))], F.GAUSSIAN, [ell], [1.0], V)
    assert np.linalg.norm(Y - Yd) / np.linalg.norm(Yd) <= tol


def test_choose_n_refuses_unreachable_tolerance():
    """l = 0.003 on an extent of 0.5 needs more than 256 grid points per edge;
    l = 0.01 is reachable only with the 256-point grid (n > 64)."""
    import paper_2404_17344_amd as A
    _lib()
    with pytest.raises(A.AddkError):
        A.choose_n(F.GAUSSIAN, 0.5, 0.003, m=6, oversampling=2.0, tol=1e-5)
    n, _ = A.choose_n(F.GAUSSIAN, 0.5, 0.01, m=6, oversampling=2.0, tol=1e-5)
    assert 64 < n <= 128
    with pytest.raises(A.AddkError):
        A.choose_n(F.GAUSSIAN, 0.5, 0.1, m=2, oversampling=2.0, tol=1e-12)


def test_near_field_flag_is_validated_before_any_device_work():
    """ADDK_NEAR_FIELD: refused for the Gaussian, with sampled coefficients or
    the paper's torus rule, and for n < 16; these checks run on the host."""
    import ctypes
    L = _lib()
    lib = L.load()
    X = np.zeros((2, 2))
    off = (ctypes.c_int32 * 2)(0, 2)
    feat = (ctypes.c_int32 * 2)(0, 1)
    ell = np.array([0.1])
    sig = np.array([1.0])

    def create(kernel, n, flags):
        h = ctypes.c_void_p()
        return lib.addk_plan_create(ctypes.byref(h), 2, 2, X.ctypes.data, 2, 1, off, feat, kernel,
                                    ell.ctypes.data_as(L._pd), sig.ctypes.data_as(L._pd), n, 2, 2.0, L.ADDK_FP64,
                                    flags, None)
    nf = L.ADDK_NEAR_FIELD
    assert create(L.ADDK_GAUSSIAN, 32, nf) == L.ADDK_ERR_UNSUPPORTED
    assert create(L.ADDK_MATERN12, 32, nf | L.ADDK_COEF_SAMPLED) == L.ADDK_ERR_UNSUPPORTED
    assert create(L.ADDK_MATERN12, 32, nf | L.ADDK_TORUS_PAPER) == L.ADDK_ERR_UNSUPPORTED
    assert create(L.ADDK_MATERN12, 8, nf) == L.ADDK_ERR_UNSUPPORTED
    assert create(L.ADDK_MATERN12, 32, 1 << 20) == L.ADDK_ERR_INVALID_ARG
    assert lib.addk_stage_name(L.ADDK_NSTAGES - 1).decode() == "near"


def test_choose_n_windows_is_the_largest_window_choice():
    """addk_choose_n_windows over a plan's windows (host points): the largest of
    the per-window choices, with the window extent taken as the largest
    per-feature range of its points."""
    import paper_2404_17344_amd as A
    _lib()
    rng = np.random.default_rng(6)
    X = np.concatenate([rng.uniform(-0.25, 0.25, (400, 3)), rng.uniform(-0.1, 0.1, (400, 2)),
                        rng.uniform(-0.05, 0.3, (400, 1))], axis=1)
    wins = [[0, 1, 2], [3, 4], [5]]
    ell = [0.08, 0.05, 0.2]
    per = []
    for w, f in enumerate(wins):
        L = float((X[:, f].max(axis=0) - X[:, f].min(axis=0)).max())
        per.append(A.choose_n(F.GAUSSIAN, L, ell[w], m=6, oversampling=2.0, tol=1e-6))
    n, est = A.choose_n_for(X, wins, ell, m=6, tol=1e-6, with_estimate=True)
    assert n == max(q[0] for q in per)
    assert est <= 1e-6 and est >= max(q[1] for q in per if q[0] == n) * (1 - 1e-12)
