"""Nonnegative least squares on the CPU (oracle side) -- TEST INFRASTRUCTURE ONLY.

Definition 1 (NNLS): x_opt = argmin_{x >= 0} ||A x - b||_2^2.  It is a convex
quadratic program (Section 3.4 restates it as min x^T Q x - 2 q^T x with
Q = A^T A, q = A^T b), so x is optimal exactly when the KKT conditions hold:
x >= 0, w = A^T (b - A x) <= 0 where x_j = 0, and w_j = 0 where x_j > 0.

Algorithm 1 ends with "any standard NNLS solver"; the paper's exact solvers are
the Lawson-Hanson active-set method [LH74] (Matlab's lsqnonneg) and KSD07.  The
oracle implements Lawson-Hanson as published (LH74, Chapter 23), with each
least-squares sub-problem solved by Householder QR of the passive columns.

Readings the paper leaves open (shared with the GPU solver, each implemented on
its own):
  * tolerance  tau = 10 * eps64 * ||A||_1 * max(m, d)  (lsqnonneg's default);
    the outer loop stops when max_{j in Z} w_j <= tau;
  * ties in argmax w_j go to the lowest index;
  * a column is refused on entry when it is numerically dependent on the passive
    set (its new triangular-factor diagonal satisfies R_tt^2 <= 1e-14 ||a_t||^2)
    or when its fresh least-squares coefficient is not positive; a refused
    column is skipped for the rest of that outer step (w_t treated as 0);
  * the outer loop is capped at max_iter (default 3d) entries; hitting the cap
    is reported as status 1;
  * after an interpolation step every passive index with x_j <= tau is moved
    back to Z (and the index that defined the step always is).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from scipy.linalg import solve_triangular

EPS64 = np.finfo(np.float64).eps
DEPENDENCE_RATIO = 1e-14

STATUS_OK = 0
STATUS_MAX_ITER = 1
STATUS_KKT_FAIL = 2


@dataclass
class NNLSResult:
    x: np.ndarray
    w: np.ndarray
    rnorm: float
    iters: int
    status: int
    passive: np.ndarray


def default_tol(A: np.ndarray) -> float:
    """tau = 10 * eps * ||A||_1 * max(m, d), ||A||_1 the largest column 1-norm."""
    A = np.asarray(A, dtype=np.float64)
    m, d = A.shape
    norm1 = float(np.max(np.sum(np.abs(A), axis=0))) if A.size else 0.0
    return 10.0 * EPS64 * norm1 * max(m, d)


def _ls_on(A: np.ndarray, b: np.ndarray, P: list[int]) -> tuple[np.ndarray, np.ndarray]:
    """Least squares restricted to the columns P, by Householder QR.
    Returns (z_P, diag(R)) in the order of P."""
    Q, R = np.linalg.qr(A[:, P], mode="reduced")
    z = solve_triangular(R, Q.T @ b, lower=False)
    return z, np.diag(R)


def lawson_hanson(A: np.ndarray, b: np.ndarray, tol: float | None = None,
                  max_iter: int | None = None,
                  passive0: np.ndarray | None = None) -> NNLSResult:
    """Lawson-Hanson active-set NNLS (LH74 Ch. 23) in FP64.

    passive0: optional initial passive set (a warm start).  The least-squares
    solution on it is taken, nonpositive entries are dropped and the solve is
    repeated until every passive entry is positive; the main loop starts from
    that feasible point.  With passive0=None the start is x = 0, P empty, which
    is how the paper initialises every NNLS call (Section 4.1).
    """
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    m, d = A.shape
    if tol is None or tol <= 0:
        tol = default_tol(A)
    if max_iter is None or max_iter <= 0:
        max_iter = 3 * d
    col_sq = np.sum(A * A, axis=0)

    x = np.zeros(d)
    P: list[int] = []
    if passive0 is not None:
        P = sorted(int(j) for j in np.nonzero(np.asarray(passive0))[0]) \
            if np.asarray(passive0).dtype == bool else sorted(set(int(j) for j in passive0))
        while P:
            z, diag = _ls_on(A, b, P)
            ok = (z > 0) & (diag * diag > DEPENDENCE_RATIO * col_sq[P])
            if np.all(ok):
                x[P] = z
                break
            P = [j for j, keep in zip(P, ok) if keep]
    iters = 0
    status = STATUS_OK

    while True:
        # outer step: dual vector and the most violated free index
        w = A.T @ (b - A @ x)
        inP = np.zeros(d, dtype=bool)
        inP[P] = True
        refused = np.zeros(d, dtype=bool)
        t = -1
        while True:
            cand = np.where(~inP & ~refused, w, -np.inf)
            t = int(np.argmax(cand)) if d else -1   # argmax: lowest index on ties
            if t < 0 or not (cand[t] > tol):
                t = -1
                break
            # try to enter t: it must be independent of the passive columns and
            # its fresh coefficient must be positive
            z, diag = _ls_on(A, b, P + [t])
            if diag[-1] ** 2 <= DEPENDENCE_RATIO * col_sq[t] or z[-1] <= 0:
                refused[t] = True
                continue
            break
        if t < 0:
            break
        if iters >= max_iter:
            status = STATUS_MAX_ITER
            break
        iters += 1
        P = P + [t]
        # inner loop: stay feasible while the unconstrained LS on P is not > 0
        while True:
            z, _ = _ls_on(A, b, P)
            if np.all(z > 0):
                x[:] = 0.0
                x[P] = z
                break
            xP = x[P]
            neg = z <= 0
            ratios = np.where(neg, xP / np.where(neg, xP - z, 1.0), np.inf)
            q = int(np.argmin(ratios))
            alpha = ratios[q]
            xP = xP + alpha * (z - xP)
            keep = [k for k in range(len(P)) if k != q and xP[k] > tol]
            x[:] = 0.0
            x[[P[k] for k in keep]] = xP[keep]
            P = [P[k] for k in keep]
            if not P:
                break

    w = A.T @ (b - A @ x)
    rnorm = float(np.linalg.norm(A @ x - b))
    return NNLSResult(x=x, w=w, rnorm=rnorm, iters=iters, status=status,
                      passive=np.array(sorted(P), dtype=np.int64))


def kkt_violation(A: np.ndarray, b: np.ndarray, x: np.ndarray) -> dict:
    """Size of the KKT violations of x for Definition 1 (all FP64):
    negativity of x, positive dual off the support, nonzero dual on it."""
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    w = A.T @ (b - A @ x)
    on = x > 0
    return {
        "neg_x": float(max(0.0, -x.min())) if x.size else 0.0,
        "dual_off": float(max(0.0, w[~on].max())) if np.any(~on) else 0.0,
        "dual_on": float(np.abs(w[on]).max()) if np.any(on) else 0.0,
    }


def kkt_ok(A: np.ndarray, b: np.ndarray, x: np.ndarray, tau: float) -> bool:
    v = kkt_violation(A, b, x)
    return v["neg_x"] == 0.0 and v["dual_off"] <= tau and v["dual_on"] <= tau


def brute_force(A: np.ndarray, b: np.ndarray) -> tuple[np.ndarray, float]:
    """NNLS optimum by enumeration of every support S subset of [d] (d <= 12):
    the optimum's nonzero part is the least-squares fit on its support, so the
    best nonnegative fit among all supports is x_opt.  Least squares per support
    via numpy.linalg.lstsq (SVD), independent of the QR path above."""
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    m, d = A.shape
    if d > 12:
        raise ValueError("brute force limited to d <= 12")
    best_x = np.zeros(d)
    best = float(np.linalg.norm(b))
    for mask in range(1, 1 << d):
        S = [j for j in range(d) if mask >> j & 1]
        z = np.linalg.lstsq(A[:, S], b, rcond=None)[0]
        if np.all(z >= 0):
            x = np.zeros(d)
            x[S] = z
            res = float(np.linalg.norm(A @ x - b))
            if res < best:
                best, best_x = res, x
    return best_x, best


def unconstrained_ls(A: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Unconstrained least squares by Householder QR (full column rank)."""
    A = np.asarray(A, dtype=np.float64)
    Q, R = np.linalg.qr(A, mode="reduced")
    return solve_triangular(R, Q.T @ np.asarray(b, dtype=np.float64), lower=False)


def relative_residual_gap(A: np.ndarray, b: np.ndarray, x: np.ndarray,
                          x_ref: np.ndarray) -> float:
    """||A x - b|| / ||A x_ref - b|| - 1 in FP64 (the unsquared ratio of the
    paper's Relative Error, Section 4.1), with the denominator floored at
    1e-12 ||b|| so exact fits do not divide by zero."""
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    num = np.linalg.norm(A @ np.asarray(x, dtype=np.float64) - b)
    den = max(np.linalg.norm(A @ np.asarray(x_ref, dtype=np.float64) - b),
              1e-12 * np.linalg.norm(b))
    if den == 0.0:
        return 0.0 if num == 0.0 else np.inf
    return float(num / den - 1.0)
