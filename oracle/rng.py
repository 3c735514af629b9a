"""Random streams of Algorithm 1 (oracle side) -- TEST INFRASTRUCTURE ONLY.

Algorithm 1 (RandomizedNNLS) draws two random objects:

* the diagonal D, each entry +1 or -1 with probability 1/2 (step 4);
* the sampling matrix S, which keeps row i of H_n with probability r/n and
  rescales it by sqrt(n/r) (step 2).

The paper fixes only these probabilities.  This project draws them from a
stateless counter-based hash so that the oracle and the GPU library can produce
the same D and S from a seed without sharing code: each side implements the
definition below on its own.

Definition (the project's reading; the same text sits in the C header):

  mix64(z)        SplitMix64 output function (Steele, Lea & Flood, OOPSLA 2014,
                  in the variant with shifts 30/27/31 and multipliers
                  0xBF58476D1CE4E5B9, 0x94D049BB133111EB), arithmetic mod 2^64.
  key(seed, s)    mix64(seed XOR (s * 0x9E3779B97F4A7C15 mod 2^64))
  h(seed, s, i)   mix64(key(seed, s) + i mod 2^64)
  streams         SIGN = 1, SAMPLE = 2, PERM = 3

  D_jj  = -1 if bit 63 of h(seed, SIGN, j) is set, else +1, for 0 <= j < n'.
  Bernoulli rows  {i : h(seed, SAMPLE, i) < r * 2^(64-m)}, m = log2 n'
                  (each row kept with probability exactly r/n').
  Exact-r rows    {pi(k) : 0 <= k < r} in ascending order, where pi is a keyed
                  bijection of [0, 2^m): four rounds of
                      x <- x XOR ka_t ;  x <- x * (kb_t | 1) mod 2^m ;
                      x <- x XOR (x >> ceil(m/2))
                  with ka_t = h(seed, PERM, 2t) mod 2^m,
                       kb_t = h(seed, PERM, 2t+1) mod 2^m, t = 0..3.
                  Every step is invertible mod 2^m, so the r rows are distinct
                  and each row is kept with marginal probability r/n'.

The oracle evaluates the hash with Python integers (``mix64``) and, for long
vectors, with numpy uint64 arithmetic (``mix64_array``); the tests check the two
against each other and against the published SplitMix64 outputs.
"""
from __future__ import annotations

import numpy as np

MASK64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15
MUL1 = 0xBF58476D1CE4E5B9
MUL2 = 0x94D049BB133111EB

STREAM_SIGN = 1
STREAM_SAMPLE = 2
STREAM_PERM = 3

PERM_ROUNDS = 4


def mix64(z: int) -> int:
    """SplitMix64 output function on one 64-bit integer (Python ints)."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * MUL1) & MASK64
    z = ((z ^ (z >> 27)) * MUL2) & MASK64
    return z ^ (z >> 31)


def splitmix64_sequence(state: int, count: int) -> list[int]:
    """The SplitMix64 generator itself: state += golden gamma, emit mix64(state).

    Only used to pin ``mix64`` against the generator's published outputs.
    """
    out = []
    for _ in range(count):
        state = (state + GOLDEN) & MASK64
        out.append(mix64(state))
    return out


def mix64_array(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function applied elementwise to a uint64 array."""
    z = np.asarray(z, dtype=np.uint64).copy()
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= np.uint64(MUL1)
        z ^= z >> np.uint64(27)
        z *= np.uint64(MUL2)
        z ^= z >> np.uint64(31)
    return z


def stream_key(seed: int, stream: int) -> int:
    return mix64((seed & MASK64) ^ ((stream * GOLDEN) & MASK64))


def h(seed: int, stream: int, i: int) -> int:
    """Counter hash h(seed, stream, i) for one index (Python ints)."""
    return mix64((stream_key(seed, stream) + i) & MASK64)


def h_array(seed: int, stream: int, idx: np.ndarray) -> np.ndarray:
    """Counter hash for a vector of indices (numpy uint64)."""
    base = np.uint64(stream_key(seed, stream))
    with np.errstate(over="ignore"):
        z = np.asarray(idx, dtype=np.uint64) + base
    return mix64_array(z)


def log2_exact(n_pad: int) -> int:
    m = int(n_pad).bit_length() - 1
    if n_pad <= 0 or (1 << m) != n_pad:
        raise ValueError("n' must be a power of two")
    return m


def signs(seed: int, n_pad: int) -> np.ndarray:
    """Diagonal of D (Algorithm 1, step 4) as int8 +-1 for rows 0..n'-1."""
    hv = h_array(seed, STREAM_SIGN, np.arange(n_pad, dtype=np.uint64))
    neg = (hv >> np.uint64(63)).astype(np.int8)
    return (1 - 2 * neg).astype(np.int8)


def rows_bernoulli(seed: int, n_pad: int, r: int) -> np.ndarray:
    """Rows kept by S of Algorithm 1, step 2 taken literally: each row i of
    H_n' is kept independently with probability r/n'.  Ascending int64."""
    m = log2_exact(n_pad)
    if not (1 <= r < n_pad):
        raise ValueError("need 1 <= r < n'")
    threshold = np.uint64(r << (64 - m))
    hv = h_array(seed, STREAM_SAMPLE, np.arange(n_pad, dtype=np.uint64))
    return np.nonzero(hv < threshold)[0].astype(np.int64)


def perm_keys(seed: int, m: int) -> list[tuple[int, int]]:
    mask = (1 << m) - 1
    keys = []
    for t in range(PERM_ROUNDS):
        ka = h(seed, STREAM_PERM, 2 * t) & mask
        kb = (h(seed, STREAM_PERM, 2 * t + 1) & mask) | 1
        keys.append((ka, kb))
    return keys


def perm(seed: int, m: int, k: int) -> int:
    """The keyed bijection pi of [0, 2^m) evaluated at k (Python ints)."""
    mask = (1 << m) - 1
    shift = (m + 1) // 2
    x = k & mask
    for ka, kb in perm_keys(seed, m):
        x ^= ka
        x = (x * kb) & mask
        x ^= x >> shift
    return x


def rows_exact(seed: int, n_pad: int, r: int) -> np.ndarray:
    """Exactly r distinct rows of H_n', uniformly without replacement, in
    ascending order: {pi(0), ..., pi(r-1)} sorted.  int64."""
    m = log2_exact(n_pad)
    if not (1 <= r < n_pad):
        raise ValueError("need 1 <= r < n'")
    out = np.array([perm(seed, m, k) for k in range(r)], dtype=np.int64)
    out.sort()
    return out


def rows(seed: int, n_pad: int, r: int, mode: str = "exact") -> np.ndarray:
    if mode == "exact":
        return rows_exact(seed, n_pad, r)
    if mode == "bernoulli":
        return rows_bernoulli(seed, n_pad, r)
    raise ValueError(mode)
