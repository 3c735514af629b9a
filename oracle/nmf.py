"""Nonnegative matrix factorisation by alternating nonnegative least squares
on the CPU -- TEST INFRASTRUCTURE ONLY.

The application the paper's conclusions name for NNLS with many right-hand
sides: A (m x n, nonnegative) ~ W H with W (m x q) >= 0 and H (q x n) >= 0,
found by alternating the two convex half-steps
    H   <- argmin_{H >= 0}   ||W H - A||_F      (n NNLS problems sharing W)
    W^T <- argmin_{W^T >= 0} ||H^T W^T - A^T||_F (m NNLS problems sharing H^T)
each solved here exactly, column by column, with the oracle's Lawson-Hanson.
Since each half-step minimises the objective exactly over one factor with the
other fixed, the objective never increases from one half-step to the next.
"""
from __future__ import annotations

import numpy as np

from . import nnls


def objective(A: np.ndarray, W: np.ndarray, H: np.ndarray) -> float:
    return float(np.linalg.norm(np.asarray(A, np.float64) - W @ H))


def anls(A: np.ndarray, W0: np.ndarray, iters: int):
    """(W, H, objective after every half-step), starting from W0."""
    A = np.asarray(A, dtype=np.float64)
    W = np.asarray(W0, dtype=np.float64).copy()
    m, n = A.shape
    hist = []
    H = None
    for _ in range(iters):
        H = np.column_stack([nnls.lawson_hanson(W, A[:, j]).x for j in range(n)])
        hist.append(objective(A, W, H))
        W = np.column_stack([nnls.lawson_hanson(H.T, A[i, :]).x for i in range(m)]).T
        hist.append(objective(A, W, H))
    return W, H, hist
