"""Algorithm 1 (RandomizedNNLS) end to end on the CPU -- TEST INFRASTRUCTURE ONLY.

Inputs A (n x d), b (n), a positive integer r < n' and the seed of the random
streams; output the nonnegative x~ that Lawson-Hanson finds for the sketched
problem min_{x >= 0} ||H~ D A x - H~ D b||^2 (Algorithm 1, step 5).

Repetition (Theorem 1 holds with probability at least 1/2; its footnote notes
that a few repetitions raise that): k independent runs with the random streams
of seeds seed, seed+1, ..., seed+k-1, keeping the x~ whose full residual
||A x~ - b|| is smallest.  Each run meets the (1+eps) bound with probability
at least 1/2, so the kept one does with probability at least 1 - 2^-k.
Readings: candidates whose solve did not finish with status 0 are passed over
unless none did; ties go to the lowest index.

Box constraints on the same sketch (the conclusions' remark that other
constraint sets can use it): steps 1-4 unchanged, step 5 replaced by the
bounded-variable solve of min_{lo <= x <= hi} ||H~ D A x - H~ D b||^2.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import bvls, hadamard, nnls


@dataclass
class RandNNLSResult:
    x: np.ndarray          # x~ (FP64)
    SA: np.ndarray         # sketched matrix, rows ascending
    Sb: np.ndarray         # sketched right-hand side
    rows: np.ndarray       # kept rows of H_n'
    solve: nnls.NNLSResult  # the Lawson-Hanson run on the sketch


def rand_nnls(A: np.ndarray, b: np.ndarray, r: int, seed: int,
              mode: str = "exact", tol: float | None = None,
              max_iter: int | None = None) -> RandNNLSResult:
    SA, Sb, R, _ = hadamard.srht_sketch(A, b, r, seed, mode)
    res = nnls.lawson_hanson(SA, Sb, tol=tol, max_iter=max_iter)
    return RandNNLSResult(x=res.x, SA=SA, Sb=Sb, rows=R, solve=res)


@dataclass
class BoostResult:
    x: np.ndarray            # the kept x~
    best: int                # its index i (seed + i)
    residuals: np.ndarray    # ||A x_i - b||_2 of every candidate, FP64
    statuses: np.ndarray     # Lawson-Hanson status of every candidate
    candidates: list         # the k RandNNLSResult runs


def rand_nnls_boost(A: np.ndarray, b: np.ndarray, r: int, k: int, seed: int,
                    mode: str = "exact", tol: float | None = None,
                    max_iter: int | None = None) -> BoostResult:
    A64 = np.asarray(A, dtype=np.float64)
    b64 = np.asarray(b, dtype=np.float64)
    runs = [rand_nnls(A, b, r, seed + i, mode, tol, max_iter) for i in range(k)]
    res = np.array([np.linalg.norm(A64 @ run.x - b64) for run in runs])
    st = np.array([run.solve.status for run in runs])
    ok = st == 0
    pool = np.flatnonzero(ok) if ok.any() else np.arange(k)
    best = int(pool[np.argmin(res[pool])])   # argmin takes the lowest index on ties
    return BoostResult(x=runs[best].x, best=best, residuals=res, statuses=st, candidates=runs)


@dataclass
class RandBoxResult:
    x: np.ndarray            # x~ in the box (FP64)
    SA: np.ndarray
    Sb: np.ndarray
    rows: np.ndarray
    solve: bvls.BoxResult


def rand_box(A: np.ndarray, b: np.ndarray, r: int, seed: int, lo: np.ndarray,
             hi: np.ndarray, mode: str = "exact", tol: float | None = None,
             max_iter: int | None = None) -> RandBoxResult:
    SA, Sb, R, _ = hadamard.srht_sketch(A, b, r, seed, mode)
    res = bvls.bvls(SA, Sb, lo, hi, tol=tol, max_iter=max_iter)
    return RandBoxResult(x=res.x, SA=SA, Sb=Sb, rows=R, solve=res)
