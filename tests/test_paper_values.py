"""Pins against numbers the paper prints (tests/golden/paper_printed_values.txt)."""
import math
import os

import numpy as np
import pytest

from oracle import fourier as F

_GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_printed_values.txt")


def _gold():
    out = {}
    for line in open(_GOLD):
        if line.startswith("#") or not line.strip():
            continue
        name, value, _cite = line.rstrip("\n").split("\t")
        out[name] = float(value)
    return out


def test_sup_of_A_at_eta_one_matches_printed_value():
    """sup over l of A(1, l) is the printed 0.377 (reached as l -> 1/2 from below)."""
    g = _gold()
    ells = np.concatenate([np.linspace(0.01, 0.4999999, 20000), np.linspace(0.5, 5.0, 2000)])
    sup = max(F.A_bound(1.0, float(l)) for l in ells)
    assert sup == pytest.approx(g["A_sup_eta_ge_1"], abs=5e-4)
    assert all(F.A_bound(e, 0.3) <= g["A_sup_eta_ge_1"] + 5e-4 for e in np.linspace(1.0, 10.0, 50))


@pytest.mark.parametrize("ell", [0.05, 0.1, 0.2, 0.3, 0.45, 0.7, 2.0])
@pytest.mark.parametrize("n", [16, 32, 64])
def test_low_mode_coefficient_sum_bound(ell, n):
    """sum_{k=1}^{n/2} |c_k| <= 3/4 for the truncated Gaussian; <= 1/2 + 0.202 for l >= 1/2."""
    g = _gold()
    s = float(np.sum(np.abs(F.truncated_gauss_coeff_1d(np.arange(1, n // 2 + 1), ell))))
    assert s <= g["sum_low_coeffs_bound"]
    if ell >= 0.5:
        assert s <= 0.5 + g["low_coeffs_large_l"] + 1e-3


def test_presets():
    g = _gold()
    assert (g["preset_fine"], g["preset_default"], g["preset_rough"]) == (64, 32, 16)
    # eta = l pi m / sqrt(2) >= 1 holds for l = 0.1 in every preset except 'rough'
    assert F.eta(0.1, 16) > 1 and F.eta(0.02, 16) < 1
