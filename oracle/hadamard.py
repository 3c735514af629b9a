"""Walsh-Hadamard transform and the sketch of Algorithm 1 (oracle side).
TEST INFRASTRUCTURE ONLY.

Section 2 of the paper defines the non-normalised Hadamard-Walsh matrix by the
Sylvester recursion H_2 = [[1, 1], [1, -1]], H_n = [[H_{n/2}, H_{n/2}],
[H_{n/2}, -H_{n/2}]] and normalises it by 1/sqrt(n); n is a power of two and
A, b are padded with zero rows otherwise.  In 0-based indices the recursion
gives H[i, j] = (-1)^popcount(i & j) (natural, not sequency, order).

Algorithm 1 then forms H~ D A and H~ D b, where H~ holds the rows of S H_n that
S keeps, each scaled by sqrt(n/r).  With the normalised H_n this is
sqrt(n/r) * (1/sqrt(n)) = 1/sqrt(r) times the unnormalised rows, so

    [A~ | b~] = (1/sqrt(r)) * (H_n' D [A | b])[R, :]

with R the kept rows in ascending order and n' the padded size.
"""
from __future__ import annotations

import numpy as np

from . import rng


def next_pow2(n: int) -> int:
    """n' = 2^ceil(log2 n): the padded row count of Section 2."""
    if n < 1:
        raise ValueError("n must be positive")
    return 1 << (int(n) - 1).bit_length()


def hadamard_entry(i, j):
    """H_n[i, j] of the non-normalised Sylvester matrix, 0-based: the parity
    of the bits that i and j share decides the sign."""
    ij = np.bitwise_and(np.asarray(i, dtype=np.int64), np.asarray(j, dtype=np.int64))
    par = np.zeros_like(ij)
    while np.any(ij):
        par ^= ij & 1
        ij = ij >> 1
    return 1 - 2 * par


def hadamard_matrix(n: int) -> np.ndarray:
    """Explicit non-normalised H_n built by the Sylvester recursion (small n)."""
    H = np.ones((1, 1))
    while H.shape[0] < n:
        H = np.block([[H, H], [H, -H]])
    if H.shape[0] != n:
        raise ValueError("n must be a power of two")
    return H


def fwht(X: np.ndarray) -> np.ndarray:
    """Non-normalised H_n X along axis 0, in FP64, by unrolling the Sylvester
    recursion: at every level each block [top; bottom] of size 2h becomes
    [top + bottom; top - bottom].  Returns a new array."""
    X = np.array(X, dtype=np.float64, copy=True, order="C")
    n = X.shape[0]
    if n & (n - 1):
        raise ValueError("length must be a power of two")
    tail = X.shape[1:]
    h = 1
    while h < n:
        Y = X.reshape((n // (2 * h), 2, h) + tail)
        top = Y[:, 0].copy()
        bot = Y[:, 1]
        Y[:, 0] += bot
        Y[:, 1] = top - bot
        h *= 2
    return X


def pad_rows(M: np.ndarray, n_pad: int) -> np.ndarray:
    """Widen to FP64 (exact for FP32 data) and append zero rows up to n'."""
    M = np.asarray(M, dtype=np.float64)
    out = np.zeros((n_pad,) + M.shape[1:], dtype=np.float64)
    out[: M.shape[0]] = M
    return out


def srht_sketch(A: np.ndarray, b: np.ndarray | None, r: int, seed: int,
                mode: str = "exact"):
    """Sketch of Algorithm 1, steps 1-4, in FP64.

    A is n x d (any memory order), b has length n or is None.
    Returns (SA, Sb, rows, D) with SA of shape (len(rows), d), Sb of length
    len(rows) (None when b is None), rows ascending int64 and D the +-1 diagonal
    of length n'.
    """
    A = np.asarray(A)
    n, d = A.shape
    n_pad = next_pow2(n)
    if not (1 <= r < n_pad):
        raise ValueError("need 1 <= r < n'")
    D = rng.signs(seed, n_pad).astype(np.float64)
    R = rng.rows(seed, n_pad, r, mode)
    cols = A if b is None else np.column_stack([A, np.asarray(b)])
    X = pad_rows(cols, n_pad) * D[:, None]
    Y = fwht(X)[R] / np.sqrt(r)
    if b is None:
        return Y, None, R, D
    return Y[:, :d], Y[:, d], R, D


def sketch_row_direct(M: np.ndarray, D: np.ndarray, i: int, r: int) -> np.ndarray:
    """One row of the sketch computed straight from the definition, without the
    fast transform: (1/sqrt r) * sum_j H[i, j] D_jj M[j, :].  Used to spot-check
    the sketch at sizes where the full transform is too costly.  M is n x k."""
    M = np.asarray(M)
    n = M.shape[0]
    coef = hadamard_entry(i, np.arange(n, dtype=np.int64)) * D[:n]
    return (coef.astype(np.float64) @ M.astype(np.float64)) / np.sqrt(r)
