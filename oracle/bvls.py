"""Least squares with bounds on the sketch (oracle side) -- TEST INFRASTRUCTURE ONLY.

The paper's conclusions remark that the sketch of Algorithm 1 does not depend on
the constraint set, so the same small problem can carry other constraints on x.
Box constraints are the simplest of them:

    x_box = argmin_{lo <= x <= hi} ||A x - b||_2^2,

with lo finite and hi >= lo (hi may be +inf).  With lo = 0 and hi = +inf this is
Definition 1.  A point is optimal exactly when, with w = A^T (b - A x),
w_j <= 0 where x_j = lo_j < hi_j, w_j >= 0 where x_j = hi_j > lo_j, and w_j = 0
where lo_j < x_j < hi_j.

The oracle is the bounded-variable active-set method of Stark and Parker
(BVLS, 1995), the Lawson-Hanson outer/inner loop with two bounds: every variable
is at its lower bound, at its upper bound or free; the outer loop frees the bound
variable whose dual most violates its condition, the inner loop solves the free
least-squares problem on the free columns themselves (LAPACK least squares, the
other variables fixed at their bounds; no normal equations) and walks back to the
box when the solution leaves it.

Readings (shared with the device solver, each implemented on its own):
  * tolerance tau = 10 * eps64 * ||A||_1 * max(m, d), as for Lawson-Hanson; the
    outer loop stops when no bound variable's dual exceeds tau in its direction;
  * ties in the choice of the entering variable go to the lowest index;
  * every variable starts at its lower bound; a variable with lo_j = hi_j never
    enters;
  * an entering variable is refused (for that outer step) when its column is
    numerically dependent on the free columns or when the first free solution
    does not move it into the box from its bound;
  * after an interpolation step a free variable within tau of a bound is put on
    that bound (the one that defined the step always is);
  * the outer loop is capped at max_iter entries (default 3d; status 1).
"""
from __future__ import annotations

from dataclasses import dataclass
from itertools import product

import numpy as np

from .nnls import default_tol

DEPENDENCE_RATIO = 1e-14
AT_LOW, AT_HIGH, FREE = 0, 1, 2

STATUS_OK = 0
STATUS_MAX_ITER = 1


@dataclass
class BoxResult:
    x: np.ndarray
    w: np.ndarray
    rnorm: float
    iters: int
    status: int
    state: np.ndarray


def _free_solve(A, b, x, F):
    """Least squares over the free columns with the others at their values:
    min || A_F z - (b - A_B x_B) ||; returns z and whether the newest column
    (the last of F) was independent of the rest."""
    B = [j for j in range(A.shape[1]) if j not in F]
    rhs = b - A[:, B] @ x[B] if B else b.copy()
    Q, R = np.linalg.qr(A[:, F], mode="reduced")
    t = F[-1]
    dep = R[-1, -1] ** 2 <= DEPENDENCE_RATIO * float(A[:, t] @ A[:, t])
    z = np.linalg.lstsq(A[:, F], rhs, rcond=None)[0]
    return z, not dep


def bvls(A: np.ndarray, b: np.ndarray, lo: np.ndarray, hi: np.ndarray,
         tol: float | None = None, max_iter: int | None = None) -> BoxResult:
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    m, d = A.shape
    if not (np.all(np.isfinite(lo)) and np.all(hi >= lo)):
        raise ValueError("bounds need finite lo and hi >= lo")
    tau = default_tol(A) if tol is None else float(tol)
    max_iter = 3 * d if max_iter is None else max_iter
    x = lo.copy()
    state = np.full(d, AT_LOW)
    free: list[int] = []
    iters, status = 0, STATUS_OK
    refused = np.zeros(d, dtype=bool)
    while True:
        w = A.T @ (b - A @ x)
        # a bound variable may enter when its dual points into the box
        score = np.full(d, -np.inf)
        low = (state == AT_LOW) & (hi > lo) & ~refused
        high = (state == AT_HIGH) & ~refused
        score[low] = w[low]
        score[high] = -w[high]
        t = int(np.argmax(score))
        if not score[t] > tau:
            break
        if iters >= max_iter:
            status = STATUS_MAX_ITER
            break
        iters += 1
        came_from = state[t]
        F = free + [t]
        z, indep = _free_solve(A, b, x, F)
        zt = z[-1]
        moves_in = (zt > x[t]) if came_from == AT_LOW else (zt < x[t])
        if not indep or not moves_in:
            refused[t] = True
            continue
        refused[:] = False
        state[t] = FREE
        free = F
        while True:
            Fa = np.array(free)
            below = z <= lo[Fa] + tau
            above = z >= hi[Fa] - tau
            if not (below.any() or above.any()):
                x[Fa] = z
                break
            # the longest step from x toward z that stays in the box
            alpha, arg = 1.0, -1
            for i, j in enumerate(free):
                if below[i] and x[j] > z[i]:
                    a = (x[j] - lo[j]) / (x[j] - z[i])
                elif above[i] and z[i] > x[j]:
                    a = (hi[j] - x[j]) / (z[i] - x[j])
                else:
                    continue
                if a < alpha:
                    alpha, arg = a, i
            alpha = min(max(alpha, 0.0), 1.0)
            x[Fa] = x[Fa] + alpha * (z - x[Fa])
            keep = []
            for i, j in enumerate(free):
                # the index that defined the step goes to the bound it reached
                to_low = below[i] if i == arg else x[j] <= lo[j] + tau
                to_high = (not below[i]) if i == arg else x[j] >= hi[j] - tau
                if to_low:
                    x[j], state[j] = lo[j], AT_LOW
                elif to_high:
                    x[j], state[j] = hi[j], AT_HIGH
                else:
                    keep.append(j)
            free = keep
            if not free:
                break
            z = _plain_free(A, b, x, free)
    w = A.T @ (b - A @ x)
    return BoxResult(x=x, w=w, rnorm=float(np.linalg.norm(A @ x - b)), iters=iters,
                     status=status, state=state.copy())


def _plain_free(A, b, x, F):
    B = [j for j in range(A.shape[1]) if j not in F]
    rhs = b - A[:, B] @ x[B] if B else b.copy()
    return np.linalg.lstsq(A[:, F], rhs, rcond=None)[0]


def kkt_box(A, b, x, lo, hi, tau):
    """Largest violation of the optimality conditions above, scaled by tau."""
    A = np.asarray(A, dtype=np.float64)
    w = A.T @ (np.asarray(b, dtype=np.float64) - A @ x)
    worst = 0.0
    for j in range(A.shape[1]):
        if x[j] < lo[j] - tau or x[j] > hi[j] + tau:
            return np.inf
        at_lo = x[j] <= lo[j] + tau
        at_hi = x[j] >= hi[j] - tau
        if at_lo and at_hi:
            continue
        if at_lo:
            worst = max(worst, w[j])
        elif at_hi:
            worst = max(worst, -w[j])
        else:
            worst = max(worst, abs(w[j]))
    return worst / tau if tau > 0 else worst


def brute_force(A, b, lo, hi):
    """Every assignment of each variable to its lower bound, its upper bound or
    free (3^d of them, d small): the free least-squares solution with the rest
    at their bounds, kept if it lies in the box; the least objective wins."""
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    d = A.shape[1]
    best_x, best_f = None, np.inf
    for assign in product((AT_LOW, AT_HIGH, FREE), repeat=d):
        x = np.zeros(d)
        ok = True
        for j, s in enumerate(assign):
            if s == AT_LOW:
                x[j] = lo[j]
            elif s == AT_HIGH:
                if not np.isfinite(hi[j]):
                    ok = False
                    break
                x[j] = hi[j]
        if not ok:
            continue
        F = [j for j, s in enumerate(assign) if s == FREE]
        if F:
            x[F] = _plain_free(A, b, x, F)
            if np.any(x[F] < np.asarray(lo)[F] - 1e-12) or np.any(x[F] > np.asarray(hi)[F] + 1e-12):
                continue
        f = float(np.sum((A @ x - b) ** 2))
        if f < best_f:
            best_x, best_f = x.copy(), f
    return best_x, best_f
