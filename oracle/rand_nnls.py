"""Algorithm 1 (RandomizedNNLS) end to end on the CPU -- TEST INFRASTRUCTURE ONLY.

Inputs A (n x d), b (n), a positive integer r < n' and the seed of the random
streams; output the nonnegative x~ that Lawson-Hanson finds for the sketched
problem min_{x >= 0} ||H~ D A x - H~ D b||^2 (Algorithm 1, step 5).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import hadamard, nnls


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
