"""Quantities from the analysis of Algorithm 1 -- TEST INFRASTRUCTURE ONLY.

* Lemma 1: for Phi = U Sigma V^T and the sampling S, write U^T S^T S U = I + E.
  Then | ||Phi y||^2 - ||S Phi y||^2 | <= ||E||_2 ||Phi y||^2 for every y.  The
  realised distortion eps' = ||E||_2 is computed here for a concrete draw.
* Proof of Theorem 1: with Phi = H_n D [A, -b] and eps' < 1, the chain of
  inequalities gives ||A x~ - b||^2 <= (1 + eps') / (1 - eps') ||A x_opt - b||^2
  deterministically for that draw (H_n D is orthogonal, so the full residuals
  equal the transformed ones).
* Lemma 2: for orthonormal U (n x k), every row of H_n D U has squared norm at
  most 4.2 k log2(n) / n with probability at least 0.9 (n >= 20); the proof of
  Theorem 1 applies it with k = d + 1.
"""
from __future__ import annotations

import numpy as np

from . import hadamard


def orthonormal_basis(M: np.ndarray) -> np.ndarray:
    """Left singular vectors of M (thin SVD), FP64."""
    U, s, _ = np.linalg.svd(np.asarray(M, dtype=np.float64), full_matrices=False)
    keep = s > s[0] * 1e-12 if s.size else s.astype(bool)
    return U[:, keep]


def realised_eps(A: np.ndarray, b: np.ndarray, rows: np.ndarray, D: np.ndarray,
                 r: int) -> float:
    """eps' = ||(S H D U)^T (S H D U) - I||_2 for U = basis of [A, -b], with S
    the kept rows scaled so that S H D equals (1/sqrt r) x unnormalised rows."""
    n = A.shape[0]
    n_pad = D.shape[0]
    U = orthonormal_basis(np.column_stack([np.asarray(A, np.float64),
                                           -np.asarray(b, np.float64)]))
    X = hadamard.pad_rows(U, n_pad) * D[:, None]
    SU = hadamard.fwht(X)[rows] / np.sqrt(r)
    E = SU.T @ SU - np.eye(U.shape[1])
    return float(np.linalg.norm(E, 2))


def chain_bound(eps: float) -> float:
    """(1 + eps') / (1 - eps'): the factor on the squared residual."""
    return (1.0 + eps) / (1.0 - eps)


def lemma2_max_row_norm(U: np.ndarray, D: np.ndarray) -> float:
    """max_i ||(H_n D U)_(i)||^2 with the normalised H_n."""
    n_pad = D.shape[0]
    X = hadamard.pad_rows(U, n_pad) * D[:, None]
    Y = hadamard.fwht(X) / np.sqrt(n_pad)
    return float(np.max(np.sum(Y * Y, axis=1)))


def lemma2_bound(k: int, n_pad: int) -> float:
    return 4.2 * k * np.log2(n_pad) / n_pad
