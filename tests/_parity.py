"""Error measures of the GPU parity tests (no arithmetic of the method).

relerr(a, b) compares a result a with a reference b of shape (rows, columns)
column by column and returns the worse of two relative errors over all
columns: the Euclidean one ||a - b||_2 / ||b||_2 and the element-wise one
max |a - b| / max |b|.  A tolerance on relerr therefore bounds both, so an
error confined to a few rows (one tile class, one cell) cannot hide under a
small 2-norm.
"""
import numpy as np


def relerr(a, b):
    a = np.asarray(a, dtype=np.float64).reshape(len(a), -1)
    b = np.asarray(b, dtype=np.float64).reshape(len(b), -1)
    worst = 0.0
    for r in range(b.shape[1]):
        d = a[:, r] - b[:, r]
        worst = max(worst, np.linalg.norm(d) / np.linalg.norm(b[:, r]), np.max(np.abs(d)) / np.max(np.abs(b[:, r])))
    return worst


def inner_err(got, ref, norm_a, norm_b):
    """Error of a computed inner product <a, b> on the scale that the
    Cauchy-Schwarz inequality gives it: |got - ref| / (||a|| ||b||).  An error
    of relative size e in the vector b moves <a, b> by at most e ||a|| ||b||,
    however much the sum cancels."""
    return abs(got - ref) / (norm_a * norm_b)
