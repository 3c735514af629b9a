"""Nonnegative matrix factorisation by alternating nonnegative least squares
on the device, each half-step solved by Algorithm 1 for many right-hand sides
(rnnls_rand_nnls_multi) -- the application the paper's conclusions name for
NNLS with multiple right-hand sides.

A (m x n, FP32, column-major, nonnegative) ~ W H, W (m x q) >= 0, H (q x n) >= 0:
    H   <- argmin_{H >= 0}   ||W H - A||_F      one sketch of [W | A] (m rows)
    W^T <- argmin_{W^T >= 0} ||H^T W^T - A^T||_F one sketch of [H^T | A^T] (n rows)
Every column of a right-hand side is an NNLS problem that shares the sketch
and the Gram matrix of the factor; more than RNNLS_MAX_K columns are taken in
chunks (each chunk sketches the factor with the same seed).  A^T is kept as a
second column-major copy (A stored row-major), made once.  The sketched
objective of a half-step is the sum of its sketched squared residuals.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import torch

from . import rnnls


@dataclass
class NmfResult:
    W: torch.Tensor                 # (m, q) FP32, column-major
    H: torch.Tensor                 # (q, n) FP32, column-major
    sketched_objective: list = field(default_factory=list)  # per half-step, Frobenius norm


def _solve_all(M: torch.Tensor, B: torch.Tensor, r: int, seed: int, opts, stream):
    """X (d x k, FP64) and the summed squared sketched residuals for every column of B."""
    k = B.shape[1]
    xs, rn = [], torch.zeros((), dtype=torch.float64, device=M.device)
    for j0 in range(0, k, rnnls.MAX_K):
        sol = rnnls.rand_nnls_multi(M, B[:, j0:j0 + rnnls.MAX_K], r, seed, opts=opts, stream=stream)
        xs.append(sol.X)
        rn = rn + (sol.rnorm ** 2).sum()
    return (xs[0] if len(xs) == 1 else torch.cat(xs, dim=1)), rn


def _colmajor_transpose(X: torch.Tensor) -> torch.Tensor:
    """X (a x b, FP64) -> X^T (b x a) as an FP32 column-major tensor."""
    return X.float().contiguous().t()


def nmf_als(A: torch.Tensor, q: int, iters: int, r_h: int, r_w: int, seed: int = 0,
            W0: torch.Tensor | None = None, opts: rnnls.Opts | None = None,
            stream=None) -> NmfResult:
    """A (m x n) column-major FP32 on the device; r_h < m' and r_w < n' rows
    of the two sketches (m', n' the next powers of two)."""
    m, n = A.shape
    At = A.contiguous().t() if A.stride(0) == 1 else A.t().contiguous().t()
    if W0 is None:
        g = torch.Generator().manual_seed(seed)
        W0 = torch.rand((m, q), generator=g, dtype=torch.float32)
    W = W0.to(A.device, torch.float32).t().contiguous().t()   # column-major (m, q)
    out = NmfResult(W, None)
    hist = []
    for t in range(iters):
        X, rn = _solve_all(W, A, r_h, seed + 2 * t, opts, stream)          # H: (q, n)
        hist.append(rn)
        Ht = _colmajor_transpose(X)                                          # H^T (n, q)
        Xw, rn = _solve_all(Ht, At, r_w, seed + 2 * t + 1, opts, stream)    # W^T: (q, m)
        hist.append(rn)
        W = _colmajor_transpose(Xw)                                          # W (m, q)
        out.H = X.float().t().contiguous().t()                               # (q, n) column-major
    out.W = W
    out.sketched_objective = [float(v.sqrt().item()) for v in hist]
    return out
