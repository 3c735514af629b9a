"""The oracle over many columns or problems at once, in worker processes.
TEST INFRASTRUCTURE ONLY (imports the oracle; nothing of the library).

Workers are spawned, not forked, so they inherit no GPU state; each runs the
plain oracle functions unchanged on its share (columns of one sketch, whole
problems).  Used by the parity tests that compare every output at the
benchmark sizes, where one host core would take minutes.
"""
from __future__ import annotations

import multiprocessing as mp
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np


def workers() -> int:
    """Host cores this process may use, at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _executor(tasks: int) -> ProcessPoolExecutor:
    # one BLAS thread per worker, one worker per core (spawned workers read
    # these when they import numpy)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"
    return ProcessPoolExecutor(max_workers=max(1, min(workers(), tasks)),
                               mp_context=mp.get_context("spawn"))


def _sketch_cols(M, r, seed, mode):
    from oracle import hadamard
    Y, _, R, _ = hadamard.srht_sketch(M, None, r, seed, mode)
    return Y, R


def sketch(M: np.ndarray, r: int, seed: int, mode: str = "exact", chunk: int = 16):
    """(Y, rows): the oracle's sketch (1/sqrt r)(H D M)[rows] of every column of
    M (n x k), computed column chunk by column chunk (a column's sketch does not
    depend on the other columns)."""
    k = M.shape[1]
    parts = [np.ascontiguousarray(M[:, c:c + chunk]) for c in range(0, k, chunk)]
    with _executor(len(parts)) as ex:
        futs = [ex.submit(_sketch_cols, P, r, seed, mode) for P in parts]
        res = [f.result() for f in futs]
    rows = res[0][1]
    assert all(np.array_equal(R, rows) for _, R in res)
    return np.column_stack([Y for Y, _ in res]), rows


def _lh_many(SA, SB, tol, max_iter):
    from oracle import nnls
    out = [nnls.lawson_hanson(SA, SB[:, j], tol=tol, max_iter=max_iter) for j in range(SB.shape[1])]
    return np.column_stack([o.x for o in out]), np.array([o.status for o in out])


def lawson_hanson_many(SA: np.ndarray, SB: np.ndarray, chunk: int = 32, tol=None, max_iter=None):
    """The oracle's Lawson-Hanson for every right-hand side SB[:, j] with the
    shared matrix SA; returns (X (d x k), statuses)."""
    k = SB.shape[1]
    with _executor((k + chunk - 1) // chunk) as ex:
        futs = [ex.submit(_lh_many, SA, np.ascontiguousarray(SB[:, c:c + chunk]), tol, max_iter)
                for c in range(0, k, chunk)]
        res = [f.result() for f in futs]
    return np.column_stack([X for X, _ in res]), np.concatenate([s for _, s in res])


def _batch_case(i, n, d, r, seed, batch_seed, x, mode):
    from oracle import hadamard, nnls
    from paper_0812_4547_amd import workloads
    p = workloads.batch_instance(i, n, d, batch_seed=batch_seed)
    SA, Sb, _, _ = hadamard.srht_sketch(p.A.astype(np.float64), p.b.astype(np.float64), r, seed,
                                        mode)
    ref = nnls.lawson_hanson(SA, Sb)
    gap_sk = nnls.relative_residual_gap(SA, Sb, x, ref.x)
    gap_full = nnls.relative_residual_gap(p.A, p.b, x, ref.x)
    return gap_sk, gap_full, ref.status


def batch_gaps(cases, batch_seed: int, mode: str = "exact"):
    """For every batch instance (i, n, d, r, sketch seed, device x~): the
    relative residual gap of x~ against the oracle's Algorithm 1 on the
    oracle's own sketch, and on the full problem, and the oracle's status.
    Instances are regenerated in the workers from their seeds."""
    with _executor(len(cases)) as ex:
        futs = [ex.submit(_batch_case, i, n, d, r, s, batch_seed, x, mode)
                for i, n, d, r, s, x in cases]
        return [f.result() for f in futs]
