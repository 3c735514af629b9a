"""Seeded synthetic inputs for RandomizedNNLS (shared by tests, bench and oracle).

This module holds no part of the method's arithmetic: it only draws A, b and
the planted solution x* with numpy's PCG64 (``numpy.random.default_rng``), so
the GPU library and the CPU oracle see exactly the same bytes.

Matrices are returned column-major (``numpy`` Fortran order, shape (n, d)):
every column of A is one contiguous vector of length n, the layout the C
library expects (leading dimension lda = n).

Workloads
---------
uniform_planted   A with U[0,1] entries, x* with a fixed number of zeros and
                  U[0,2] nonzeros, b = A x* + N(0, sigma^2) noise.
tfidf_like        stand-in for the term-document matrices of Section 4.1
                  (TechTC300 is not available here): sparse nonnegative columns
                  whose densities follow a Zipf rank law with mean density rho,
                  lognormal(0,1) values, every column L2-normalised, stored
                  dense; b = A x* + noise of a given relative size.
batch_shapes      the (n, d, r) triples of a batch of uneven instances:
                  n log-uniform in [2^14, 2^18], d uniform in [8, 96],
                  r = max(32 d, 1024).
density_sweep     random n x (d+1) matrices of a target density with U[0,1]
                  nonzeros; b is one column, A the rest (Section 4.2).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Problem:
    A: np.ndarray        # (n, d) float32, Fortran order
    b: np.ndarray        # (n,) float32
    x_star: np.ndarray   # planted solution (float64), or None
    name: str = ""

    @property
    def n(self) -> int:
        return self.A.shape[0]

    @property
    def d(self) -> int:
        return self.A.shape[1]


def uniform_planted(n: int = 4096, d: int = 16, zeros: int = 8, sigma: float = 0.01,
                    seed: int = 1) -> Problem:
    """U[0,1] matrix, x* with `zeros` zero entries and U[0,2] nonzeros,
    b = A x* + N(0, sigma^2).  Defaults: the 4096 x 16 single-instance case."""
    g = np.random.default_rng(seed)
    A = np.asfortranarray(g.random((n, d), dtype=np.float64).astype(np.float32))
    x = g.uniform(0.0, 2.0, size=d)
    x[g.choice(d, size=min(zeros, d), replace=False)] = 0.0
    b = A.astype(np.float64) @ x + sigma * g.standard_normal(n)
    return Problem(A=A, b=b.astype(np.float32), x_star=x,
                   name=f"uniform_planted n={n} d={d}")


def density_matrix(n: int, cols: int, density: float, seed: int) -> np.ndarray:
    """n x cols FP32 random matrix of the sparse-versus-dense experiment
    (Section 4.2): each entry nonzero with probability `density`, nonzero
    values uniform in [0, 1] (the text's "normally distributed in [0,1]"
    taken as uniform), stored dense."""
    g = np.random.default_rng(seed)
    M = g.random((n, cols)) * (g.random((n, cols)) < density)
    return M.astype(np.float32)


def density_problem(M: np.ndarray, col: int) -> Problem:
    """b = column `col` of M, A = the remaining columns (Section 4.2)."""
    keep = [c for c in range(M.shape[1]) if c != col]
    return Problem(A=np.asfortranarray(M[:, keep]), b=np.ascontiguousarray(M[:, col]),
                   x_star=None, name=f"density column {col}")


def zipf_densities(d: int, mean_density: float, s: float, g) -> np.ndarray:
    """Column densities rho_k = mean * d * k^-s / sum_j j^-s for ranks
    k = 1..d, randomly permuted over the columns."""
    k = np.arange(1, d + 1, dtype=np.float64)
    w = k ** (-s)
    rho = mean_density * d * w / w.sum()
    return g.permutation(np.minimum(rho, 1.0))


def tfidf_like(n: int, d: int, seed: int, mean_density: float = 0.01,
               zipf_s: float = 1.1, zero_frac: float = 0.3, noise: float = 0.05,
               dtype=np.float32) -> Problem:
    """Term-document-like NNLS instance (see module docstring)."""
    g = np.random.default_rng(seed)
    rho = zipf_densities(d, mean_density, zipf_s, g)
    A = np.zeros((n, d), dtype=dtype, order="F")
    x = g.uniform(0.0, 2.0, size=d)
    x[g.choice(d, size=int(round(zero_frac * d)), replace=False)] = 0.0
    Ax = np.zeros(n, dtype=np.float64)
    for k in range(d):
        nnz = int(min(max(round(rho[k] * n), 1), n))
        rows = g.choice(n, size=nnz, replace=False)
        vals = g.lognormal(0.0, 1.0, size=nnz)
        vals /= np.linalg.norm(vals)
        vals32 = vals.astype(dtype)
        A[rows, k] = vals32
        if x[k] != 0.0:
            np.add.at(Ax, rows, x[k] * vals32.astype(np.float64))
    e = g.standard_normal(n)
    e *= noise * np.linalg.norm(Ax) / np.linalg.norm(e)
    b = (Ax + e).astype(dtype)
    return Problem(A=A, b=b, x_star=x, name=f"tfidf_like n={n} d={d}")


def tfidf_multi_rhs(n: int, d: int, k: int, seed: int, mean_density: float = 0.01,
                    zipf_s: float = 1.1, zero_frac: float = 0.3, noise: float = 0.05):
    """One tf-idf-like A with k right-hand sides B = A X* + E (5% noise per
    column), as in a nonnegative-matrix-factorisation update.  Returns
    (A, B, X*) with B of shape (n, k), Fortran order."""
    p = tfidf_like(n, d, seed, mean_density, zipf_s, zero_frac, noise)
    g = np.random.default_rng(seed + 7919)
    X = g.uniform(0.0, 2.0, size=(d, k))
    for c in range(k):
        X[g.choice(d, size=int(round(zero_frac * d)), replace=False), c] = 0.0
    A64 = p.A.astype(np.float64)
    AX = A64 @ X
    E = g.standard_normal((n, k))
    E *= noise * np.linalg.norm(AX, axis=0) / np.linalg.norm(E, axis=0)
    B = np.asfortranarray((AX + E).astype(np.float32))
    return p.A, B, X


def batch_shapes(count: int = 256, seed: int = 4, log2_n=(14.0, 18.0),
                 d_range=(8, 96), r_per_col: int = 32, r_min: int = 1024):
    """(n_i, d_i, r_i) for a batch of uneven instances."""
    g = np.random.default_rng(seed)
    ns = np.rint(2.0 ** g.uniform(log2_n[0], log2_n[1], size=count)).astype(np.int64)
    ds = g.integers(d_range[0], d_range[1] + 1, size=count)
    rs = np.maximum(r_per_col * ds, r_min)
    return [(int(n), int(d), int(r)) for n, d, r in zip(ns, ds, rs)]


def batch_instance(i: int, n: int, d: int, batch_seed: int = 4) -> Problem:
    """Instance i of a batch: tf-idf-like with a seed derived from (batch, i)."""
    return tfidf_like(n, d, seed=batch_seed * 1_000_003 + i)


def tfidf_like_device(n: int, d: int, seed: int, device="cuda", mean_density: float = 0.01,
                      zipf_s: float = 1.1, zero_frac: float = 0.3, noise: float = 0.05):
    """Device-side tf-idf-like instance for large training sets: the column
    densities and x* are drawn on the host as in tfidf_like, the entries on
    the device (each entry nonzero with its column's density, values
    lognormal(0,1), columns L2-normalised; a column left empty gets one
    entry), b = A x* + e with ||e|| = noise ||A x*||.  Returns (A, b, x*) with
    A an (n, d) column-major float32 tensor (leading dimension n rounded up to
    a multiple of 4) and b float32 (n,)."""
    import torch
    g = np.random.default_rng(seed)
    rho = zipf_densities(d, mean_density, zipf_s, g)
    x = g.uniform(0.0, 2.0, size=d)
    x[g.choice(d, size=int(round(zero_frac * d)), replace=False)] = 0.0
    fill_rows = g.integers(0, n, size=d)
    tg = torch.Generator(device=device)
    tg.manual_seed(int(seed) & 0x7FFFFFFFFFFFFFFF)
    M = torch.rand((d, n), generator=tg, device=device)
    vals = torch.randn((d, n), generator=tg, device=device).exp_()
    rho_t = torch.from_numpy(rho.astype(np.float32)).to(device).unsqueeze(1)
    M = torch.where(M < rho_t, vals, torch.zeros((), device=device))
    del vals
    empty = (M.abs().sum(dim=1) == 0).nonzero().flatten()
    if empty.numel():
        fr = torch.from_numpy(fill_rows).to(device)
        M[empty, fr[empty]] = 1.0
    M /= M.norm(dim=1, keepdim=True)
    xs = torch.from_numpy(x).to(device)
    Ax = (M.t().double() @ xs)
    e = torch.randn(n, generator=tg, device=device, dtype=torch.float64)
    e *= noise * Ax.norm() / e.norm()
    b = (Ax + e).float()
    # leading dimension rounded up to a multiple of 4: 16-byte aligned columns
    lda = (n + 3) // 4 * 4
    P = torch.zeros((d, lda), dtype=torch.float32, device=device)
    P[:, :n] = M
    return P[:, :n].t(), b, x


def density_sweep(n: int, d: int, density: float, seed: int) -> Problem:
    """Random n x (d+1) matrix of the given density with U[0,1] nonzeros; one
    random column is b, the other d columns form A (Section 4.2)."""
    g = np.random.default_rng(seed)
    M = np.zeros((n, d + 1), dtype=np.float32, order="F")
    mask = g.random((n, d + 1)) < density
    M[mask] = g.random(int(mask.sum())).astype(np.float32)
    j = int(g.integers(d + 1))
    cols = [c for c in range(d + 1) if c != j]
    return Problem(A=np.asfortranarray(M[:, cols]), b=M[:, j].copy(), x_star=None,
                   name=f"density_sweep n={n} d={d} rho={density}")
