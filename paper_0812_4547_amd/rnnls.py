"""Python binding of librnnls.so (ctypes).  Argument marshalling only: every
step of the computation runs in the library's HIP kernels.  torch provides the
device memory and the stream.

Matrices cross the boundary column-major: a torch tensor of shape (n, d) with
stride (1, lda), lda >= n (``colmajor`` builds one from a numpy array).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "librnnls.so")

OK = 0
E_HIP, E_WORKSPACE, E_UNSUPPORTED = -100, -101, -102
SOLVE_OK, SOLVE_MAX_ITER, SOLVE_KKT_FAIL, SOLVE_NO_ROWS, SOLVE_OVERFLOW = 0, 1, 2, 3, 4
SOLVE_BAD_BOUNDS = 5
SAMPLE_EXACT, SAMPLE_BERNOULLI = 0, 1
PREC_FP32, PREC_SPLIT_BF16 = 0, 1
OP_SKETCH, OP_SOLVE, OP_RAND_NNLS = 0, 1, 2
MAX_D, MAX_R, MAX_K, MAX_BOOST, MAX_BOX_D = 128, 32768, 4096, 8, 64
MAX_D_SOLVE = 512
NOALLOC_SCRATCH_BYTES = 64 << 20

EXPORTS = (
    "rnnls_version", "rnnls_device_cus", "rnnls_workspace_bytes", "rnnls_srht_sketch",
    "rnnls_nnls_solve", "rnnls_rand_nnls", "rnnls_multi_workspace_bytes",
    "rnnls_rand_nnls_multi", "rnnls_batch_workspace_bytes", "rnnls_batch_create",
    "rnnls_batch_run", "rnnls_batch_autotune", "rnnls_batch_capture", "rnnls_batch_launch",
    "rnnls_batch_destroy", "rnnls_features", "rnnls_mlp_sync_bf16", "rnnls_mlp_forward",
    "rnnls_mlp_workspace_bytes", "rnnls_mlp_gradient", "rnnls_mlp_adam", "rnnls_mlp_train_step",
    "rnnls_batch_columns", "rnnls_batch_features", "rnnls_batch_set_model",
    "rnnls_batch_warm_used", "rnnls_timing_enable", "rnnls_timing_read",
    "rnnls_set_tuning", "rnnls_get_tuning", "rnnls_stream_read_blocks", "rnnls_stream_read",
    "rnnls_boost_workspace_bytes", "rnnls_rand_nnls_boost", "rnnls_rand_box",
    "rnnls_rand_nnls_noalloc", "rnnls_batch_proposal", "rnnls_tuning_cache_entries",
    "rnnls_tuning_cache_clear", "rnnls_tuning_cache_save", "rnnls_tuning_cache_load",
)
MLP_FEATURES, MLP_WIDTH, MLP_PARAMS, MLP_BF16_WEIGHTS = 8, 128, 17793, 17536
TIMER_SKETCH, TIMER_MOMENTS, TIMER_SOLVE, TIMER_STREAM_READ, TIMER_RESIDUAL = 0, 1, 2, 3, 4
TIMER_STREAMS, TIMER_REDUCE = 5, 6


class Opts(ctypes.Structure):
    _fields_ = [("sample_mode", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("max_iter", ctypes.c_int32), ("r_cap", ctypes.c_int32),
                ("tol", ctypes.c_double)]


class Tuning(ctypes.Structure):
    _fields_ = [("srht_log_tile", ctypes.c_int32), ("srht_wgs_per_cu", ctypes.c_int32)]


class Problem(ctypes.Structure):
    """rnnls_problem: one problem of a batch (device pointers)."""
    _fields_ = [("n", ctypes.c_int64), ("d", ctypes.c_int32), ("r", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("A", ctypes.c_void_p), ("lda", ctypes.c_int64),
                ("b", ctypes.c_void_p), ("x", ctypes.c_void_p), ("rnorm", ctypes.c_void_p),
                ("iters", ctypes.c_void_p), ("status", ctypes.c_void_p)]


class RnnlsError(RuntimeError):
    pass


_lib = None

_p = ctypes.c_void_p
_i32, _i64, _u64, _sz, _f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_size_t, ctypes.c_double
_SIGS = {
    "rnnls_version": ([], ctypes.c_int),
    "rnnls_device_cus": ([], ctypes.c_int),
    "rnnls_workspace_bytes": ([_i32, _i64, _i32, _i32, _p], _sz),
    "rnnls_srht_sketch": ([_i64, _i32, _i32, _u64, _p, _i64, _p, _p, _i64, _p, _p, _p, _p, _p,
                           _p, _p, _sz, _p], ctypes.c_int),
    "rnnls_nnls_solve": ([_i64, _i32, _p, _i64, _p, _p, _p, _p, _p, _p, _p, _p, _p, _sz, _p],
                         ctypes.c_int),
    "rnnls_rand_nnls": ([_i64, _i32, _i32, _u64, _p, _i64, _p, _p, _p, _p, _p, _p, _i64, _p, _p,
                         _p, _p, _p, _sz, _p], ctypes.c_int),
    "rnnls_rand_nnls_noalloc": ([_i64, _i32, _i32, _u64, _p, _i64, _p, _p, _p, _p, _p, _p, _i64,
                                 _p, _p, _p, _p, _p], ctypes.c_int),
    "rnnls_rand_box": ([_i64, _i32, _i32, _u64, _p, _i64, _p, _p, _p, _p, _p, _p, _p, _p, _p,
                        _sz, _p], ctypes.c_int),
    "rnnls_multi_workspace_bytes": ([_i64, _i32, _i32, _i32, _p], _sz),
    "rnnls_boost_workspace_bytes": ([_i64, _i32, _i32, _i32, _p], _sz),
    "rnnls_rand_nnls_boost": ([_i64, _i32, _i32, _i32, _u64, _p, _i64, _p, _p, _p, _p, _p, _p,
                               _p, _sz, _p], ctypes.c_int),
    "rnnls_rand_nnls_multi": ([_i64, _i32, _i32, _i32, _u64, _p, _i64, _p, _i64, _p, _i64, _p,
                               _p, _p, _p, _p, _sz, _p], ctypes.c_int),
    "rnnls_batch_workspace_bytes": ([_i32, _p, _p], _sz),
    "rnnls_batch_create": ([_p, _i32, _p, _p, _p, _sz, _p], ctypes.c_int),
    "rnnls_batch_run": ([_p, _p], ctypes.c_int),
    "rnnls_batch_autotune": ([_p, _p, _p], ctypes.c_int),
    "rnnls_batch_capture": ([_p], ctypes.c_int),
    "rnnls_batch_launch": ([_p, _p], ctypes.c_int),
    "rnnls_batch_destroy": ([_p], ctypes.c_int),
    "rnnls_features": ([_i32, _p, _p, _p, _p, _p], ctypes.c_int),
    "rnnls_mlp_sync_bf16": ([_p, _p, _p], ctypes.c_int),
    "rnnls_mlp_forward": ([_i64, _p, _p, _p, _p, _p, ctypes.c_float, _p], ctypes.c_int),
    "rnnls_mlp_workspace_bytes": ([_i64], _sz),
    "rnnls_mlp_gradient": ([_i64, _p, _p, _p, _p, _p, _p, _p, _sz, _p], ctypes.c_int),
    "rnnls_mlp_adam": ([_p, _p, _p, _p, _p, _i32, ctypes.c_float, ctypes.c_float,
                        ctypes.c_float, ctypes.c_float, _p], ctypes.c_int),
    "rnnls_mlp_train_step": ([_i64, _p, _p, _p, _p, _p, _p, _i32, ctypes.c_float, _p, _p, _sz,
                              _p], ctypes.c_int),
    "rnnls_batch_columns": ([_p, _p], ctypes.c_int),
    "rnnls_batch_features": ([_p, _p, _p, _p], ctypes.c_int),
    "rnnls_batch_set_model": ([_p, _p, _p, ctypes.c_float], ctypes.c_int),
    "rnnls_batch_warm_used": ([_p, _p, _p], ctypes.c_int),
    "rnnls_batch_proposal": ([_p, _p, _p], ctypes.c_int),
    "rnnls_tuning_cache_entries": ([], ctypes.c_int),
    "rnnls_tuning_cache_clear": ([], ctypes.c_int),
    "rnnls_tuning_cache_save": ([ctypes.c_char_p], ctypes.c_int),
    "rnnls_tuning_cache_load": ([ctypes.c_char_p], ctypes.c_int),
    "rnnls_timing_enable": ([ctypes.c_int], ctypes.c_int),
    "rnnls_timing_read": ([_i32, _p, _p], ctypes.c_int),
    "rnnls_set_tuning": ([_p], ctypes.c_int),
    "rnnls_get_tuning": ([_p], ctypes.c_int),
    "rnnls_stream_read_blocks": ([], ctypes.c_int),
    "rnnls_stream_read": ([_p, ctypes.c_int64, _p, _p], ctypes.c_int),
}


def load(path: str = LIB_PATH):
    """Load librnnls.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RnnlsError(f"{path} is missing: build it with python -m paper_0812_4547_amd.build")
        lib = ctypes.CDLL(path)
        for name, (args, res) in _SIGS.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


def _ptr(t):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _check(rc: int, what: str):
    if rc != OK:
        raise RnnlsError(f"{what} returned {rc}")


def make_opts(sample_mode: str = "exact", precision: str = "fp32", max_iter: int = 0,
              r_cap: int = 0, tol: float = 0.0) -> Opts:
    return Opts(SAMPLE_EXACT if sample_mode == "exact" else SAMPLE_BERNOULLI,
                PREC_FP32 if precision == "fp32" else PREC_SPLIT_BF16,
                int(max_iter), int(r_cap), float(tol))


def row_capacity(r: int, opts: Opts, n: int) -> int:
    """Rows the sketch buffers hold: r (exact), else opts.r_cap or
    r + 8 ceil(sqrt r) + 64, clamped to n' (the library's rule)."""
    if opts.sample_mode == SAMPLE_EXACT:
        return r
    want = opts.r_cap if opts.r_cap > 0 else r + 8 * int(np.ceil(np.sqrt(r))) + 64
    return min(want, 1 << max(0, (n - 1).bit_length()))


def colmajor(M: np.ndarray, device="cuda") -> torch.Tensor:
    """Column-major device copy of a 2-D array: shape (n, d), stride (1, lda)
    with lda = n rounded up to a multiple of 4, so that every column starts
    16-byte aligned (the sketch's vector loads need it)."""
    M = np.asarray(M, dtype=np.float32)
    n, d = M.shape
    lda = (n + 3) // 4 * 4
    out = torch.zeros((d, lda), dtype=torch.float32, device=device)
    out[:, :n] = torch.from_numpy(np.ascontiguousarray(M.T)).to(device)
    return out[:, :n].t()


def _check_colmajor(A: torch.Tensor, name: str) -> int:
    if A.dim() != 2 or A.dtype != torch.float32 or not A.is_cuda:
        raise ValueError(f"{name} must be a 2-D float32 CUDA tensor")
    if A.shape[1] > 1 and A.stride(0) != 1:
        raise ValueError(f"{name} must be column-major (stride (1, lda))")
    return A.stride(1) if A.shape[1] > 1 else max(A.shape[0], 1)


def workspace_bytes(op: int, n: int, d: int, r: int, opts: Opts | None = None) -> int:
    return int(load().rnnls_workspace_bytes(op, n, d, r, ctypes.byref(opts or Opts())))


def workspace(op: int, n: int, d: int, r: int, opts: Opts | None = None, device="cuda"):
    nbytes = workspace_bytes(op, n, d, r, opts)
    if nbytes == 0:
        raise RnnlsError("invalid sizes for the workspace query")
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


@dataclass
class Sketch:
    SA: torch.Tensor      # (R_cap, d) column-major
    Sb: torch.Tensor | None
    rows: torch.Tensor    # int32 (R_cap,)
    count: torch.Tensor   # int32 (1,)
    status: torch.Tensor  # int32 (1,)
    sign_bits: torch.Tensor | None


def srht_sketch(A: torch.Tensor, b: torch.Tensor | None, r: int, seed: int,
                opts: Opts | None = None, export_signs: bool = False, ws=None,
                stream=None) -> Sketch:
    """[SA | Sb] = (1/sqrt r) (H D [A | b])[rows] on the device (rnnls_srht_sketch)."""
    opts = opts or Opts()
    n, d = A.shape
    lda = _check_colmajor(A, "A")
    dev = A.device
    rc_ = row_capacity(r, opts, n)
    SA = torch.empty((d, rc_), dtype=torch.float32, device=dev).t()
    Sb = torch.empty(rc_, dtype=torch.float32, device=dev) if b is not None else None
    rows = torch.empty(rc_, dtype=torch.int32, device=dev)
    count = torch.empty(1, dtype=torch.int32, device=dev)
    status = torch.empty(1, dtype=torch.int32, device=dev)
    n_pad = 1 << max(0, (n - 1).bit_length())
    signs = torch.empty((n_pad + 31) // 32, dtype=torch.int32, device=dev) if export_signs else None
    if ws is None:
        ws = workspace(OP_SKETCH, n, d, r, opts, dev)
    rc = load().rnnls_srht_sketch(n, d, r, seed & (2**64 - 1), _ptr(A), lda, _ptr(b), _ptr(SA), rc_,
                                  _ptr(Sb), _ptr(rows), _ptr(count), _ptr(signs), _ptr(status),
                                  ctypes.byref(opts), _ptr(ws), ws.numel(), _stream(stream))
    _check(rc, "rnnls_srht_sketch")
    return Sketch(SA, Sb, rows, count, status, signs)


@dataclass
class Solution:
    x: torch.Tensor           # float64 (d,)
    w: torch.Tensor | None    # float64 (d,)
    rnorm: torch.Tensor       # float64 (1,)
    iters: torch.Tensor       # int32 (1,)
    status: torch.Tensor      # int32 (1,)
    sketch: Sketch | None = None


def nnls_solve(M: torch.Tensor, f: torch.Tensor, m_dev: torch.Tensor | None = None,
               opts: Opts | None = None, ws=None, stream=None) -> Solution:
    """x = argmin_{x >= 0} ||M x - f|| on the device (rnnls_nnls_solve)."""
    opts = opts or Opts()
    m, d = M.shape
    ldm = _check_colmajor(M, "M")
    dev = M.device
    x = torch.empty(d, dtype=torch.float64, device=dev)
    w = torch.empty(d, dtype=torch.float64, device=dev)
    rnorm = torch.empty(1, dtype=torch.float64, device=dev)
    iters = torch.empty(1, dtype=torch.int32, device=dev)
    status = torch.empty(1, dtype=torch.int32, device=dev)
    if ws is None:
        ws = workspace(OP_SOLVE, m, d, 0, opts, dev)
    rc = load().rnnls_nnls_solve(m, d, _ptr(M), ldm, _ptr(f), _ptr(m_dev), _ptr(x), _ptr(w),
                                 _ptr(rnorm), _ptr(iters), _ptr(status), ctypes.byref(opts),
                                 _ptr(ws), ws.numel(), _stream(stream))
    _check(rc, "rnnls_nnls_solve")
    return Solution(x, w, rnorm, iters, status)


def rand_nnls(A: torch.Tensor, b: torch.Tensor, r: int, seed: int, opts: Opts | None = None,
              keep_sketch: bool = False, ws=None, out=None, stream=None) -> Solution:
    """Algorithm 1 end to end on the device (rnnls_rand_nnls)."""
    opts = opts or Opts()
    n, d = A.shape
    lda = _check_colmajor(A, "A")
    dev = A.device
    if out is None:
        out = Solution(torch.empty(d, dtype=torch.float64, device=dev), None,
                       torch.empty(1, dtype=torch.float64, device=dev),
                       torch.empty(1, dtype=torch.int32, device=dev),
                       torch.empty(1, dtype=torch.int32, device=dev))
    sk = None
    if keep_sketch:
        rc_ = row_capacity(r, opts, n)
        sk = Sketch(torch.empty((d, rc_), dtype=torch.float32, device=dev).t(),
                    torch.empty(rc_, dtype=torch.float32, device=dev),
                    torch.empty(rc_, dtype=torch.int32, device=dev),
                    torch.empty(1, dtype=torch.int32, device=dev), out.status, None)
    if ws is None:
        ws = workspace(OP_RAND_NNLS, n, d, r, opts, dev)
    rc = load().rnnls_rand_nnls(
        n, d, r, seed & (2**64 - 1), _ptr(A), lda, _ptr(b), _ptr(out.x), _ptr(out.rnorm),
        _ptr(out.iters), _ptr(out.status),
        _ptr(sk.SA) if sk else None, row_capacity(r, opts, n) if sk else 0,
        _ptr(sk.Sb) if sk else None, _ptr(sk.rows) if sk else None,
        _ptr(sk.count) if sk else None, ctypes.byref(opts), _ptr(ws), ws.numel(),
        _stream(stream))
    _check(rc, "rnnls_rand_nnls")
    out.sketch = sk
    return out


def rand_nnls_noalloc(A: torch.Tensor, b: torch.Tensor, r: int, seed: int,
                      opts: Opts | None = None, keep_sketch: bool = False, out=None,
                      stream=None) -> Solution:
    """Algorithm 1 end to end without a workspace (rnnls_rand_nnls_noalloc):
    the library's fixed per-device scratch array takes its place."""
    opts = opts or Opts()
    n, d = A.shape
    lda = _check_colmajor(A, "A")
    dev = A.device
    if out is None:
        out = Solution(torch.empty(d, dtype=torch.float64, device=dev), None,
                       torch.empty(1, dtype=torch.float64, device=dev),
                       torch.empty(1, dtype=torch.int32, device=dev),
                       torch.empty(1, dtype=torch.int32, device=dev))
    sk = None
    rc_ = row_capacity(r, opts, n)
    if keep_sketch:
        sk = Sketch(torch.empty((d, rc_), dtype=torch.float32, device=dev).t(),
                    torch.empty(rc_, dtype=torch.float32, device=dev),
                    torch.empty(rc_, dtype=torch.int32, device=dev),
                    torch.empty(1, dtype=torch.int32, device=dev), out.status, None)
    rc = load().rnnls_rand_nnls_noalloc(
        n, d, r, seed & (2**64 - 1), _ptr(A), lda, _ptr(b), _ptr(out.x), _ptr(out.rnorm),
        _ptr(out.iters), _ptr(out.status),
        _ptr(sk.SA) if sk else None, rc_ if sk else 0,
        _ptr(sk.Sb) if sk else None, _ptr(sk.rows) if sk else None,
        _ptr(sk.count) if sk else None, ctypes.byref(opts), _stream(stream))
    _check(rc, "rnnls_rand_nnls_noalloc")
    out.sketch = sk
    return out


@dataclass
class MultiSolution:
    X: torch.Tensor       # float64 (d, k) column-major
    rnorm: torch.Tensor   # float64 (k,)
    iters: torch.Tensor   # int32 (k,)
    status: torch.Tensor  # int32 (k,)


def rand_box(A: torch.Tensor, b: torch.Tensor, r: int, seed: int, lo: torch.Tensor,
             hi: torch.Tensor, opts: Opts | None = None, ws=None, out=None,
             stream=None) -> Solution:
    """Algorithm 1 with box bounds lo <= x <= hi in step 5 (rnnls_rand_box);
    lo, hi are float64 device vectors of length d."""
    opts = opts or Opts()
    n, d = A.shape
    lda = _check_colmajor(A, "A")
    dev = A.device
    for name, v in (("lo", lo), ("hi", hi)):
        if v.dtype != torch.float64 or v.numel() != d or not v.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float64 vector of length d")
    if out is None:
        out = Solution(torch.empty(d, dtype=torch.float64, device=dev), None,
                       torch.empty(1, dtype=torch.float64, device=dev),
                       torch.empty(1, dtype=torch.int32, device=dev),
                       torch.empty(1, dtype=torch.int32, device=dev))
    if ws is None:
        ws = workspace(OP_RAND_NNLS, n, d, r, opts, dev)
    rc = load().rnnls_rand_box(n, d, r, seed & (2**64 - 1), _ptr(A), lda, _ptr(b), _ptr(lo),
                               _ptr(hi), _ptr(out.x), _ptr(out.rnorm), _ptr(out.iters),
                               _ptr(out.status), ctypes.byref(opts), _ptr(ws), ws.numel(),
                               _stream(stream))
    _check(rc, "rnnls_rand_box")
    return out


def boost_workspace(n: int, d: int, r: int, k: int, opts: Opts | None = None, device="cuda"):
    nbytes = int(load().rnnls_boost_workspace_bytes(n, d, r, k, ctypes.byref(opts or Opts())))
    if nbytes == 0:
        raise RnnlsError("invalid sizes for the workspace query")
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


@dataclass
class BoostSolution:
    x: torch.Tensor       # float64 (d,): the kept x~
    resid: torch.Tensor   # float64 (k,): ||A x_i - b|| of every candidate
    best: torch.Tensor    # int32 (1,): index of the kept candidate (seed + i)
    status: torch.Tensor  # int32 (1,): its solve status


def rand_nnls_boost(A: torch.Tensor, b: torch.Tensor, r: int, k: int, seed: int,
                    opts: Opts | None = None, ws=None, stream=None) -> BoostSolution:
    """k repetitions of Algorithm 1 (seeds seed .. seed+k-1), keeping the x~
    with the least full residual (rnnls_rand_nnls_boost)."""
    opts = opts or Opts()
    n, d = A.shape
    lda = _check_colmajor(A, "A")
    dev = A.device
    out = BoostSolution(torch.empty(d, dtype=torch.float64, device=dev),
                        torch.empty(max(k, 1), dtype=torch.float64, device=dev),
                        torch.empty(1, dtype=torch.int32, device=dev),
                        torch.empty(1, dtype=torch.int32, device=dev))
    if ws is None:
        ws = boost_workspace(n, d, r, k, opts, dev)
    rc = load().rnnls_rand_nnls_boost(n, d, r, k, seed & (2**64 - 1), _ptr(A), lda, _ptr(b),
                                      _ptr(out.x), _ptr(out.resid), _ptr(out.best),
                                      _ptr(out.status), ctypes.byref(opts), _ptr(ws), ws.numel(),
                                      _stream(stream))
    _check(rc, "rnnls_rand_nnls_boost")
    return out


def multi_workspace(n: int, d: int, k: int, r: int, opts: Opts | None = None, device="cuda"):
    nbytes = int(load().rnnls_multi_workspace_bytes(n, d, k, r, ctypes.byref(opts or Opts())))
    if nbytes == 0:
        raise RnnlsError("invalid sizes for the workspace query")
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def rand_nnls_multi(A: torch.Tensor, B: torch.Tensor, r: int, seed: int,
                    opts: Opts | None = None, ws=None, out: MultiSolution | None = None,
                    stream=None) -> MultiSolution:
    """Algorithm 1 for k right-hand sides sharing A (rnnls_rand_nnls_multi)."""
    opts = opts or Opts()
    n, d = A.shape
    k = B.shape[1]
    lda = _check_colmajor(A, "A")
    ldb = _check_colmajor(B, "B")
    dev = A.device
    if out is None:
        out = MultiSolution(torch.empty((k, d), dtype=torch.float64, device=dev).t(),
                            torch.empty(k, dtype=torch.float64, device=dev),
                            torch.empty(k, dtype=torch.int32, device=dev),
                            torch.empty(k, dtype=torch.int32, device=dev))
    if ws is None:
        ws = multi_workspace(n, d, k, r, opts, dev)
    ldx = out.X.stride(1) if k > 1 else d
    rc = load().rnnls_rand_nnls_multi(n, d, k, r, seed & (2**64 - 1), _ptr(A), lda, _ptr(B), ldb,
                                      _ptr(out.X), ldx, _ptr(out.rnorm), _ptr(out.iters),
                                      _ptr(out.status), ctypes.byref(opts), _ptr(ws), ws.numel(),
                                      _stream(stream))
    _check(rc, "rnnls_rand_nnls_multi")
    return out


class Batch:
    """A batch plan (rnnls_batch_*) over problems given as (A, b, r, seed)
    with A column-major (n, d) and b (n,) on the device.  Owns the outputs
    x[i] (float64 (d_i,)), rnorm, iters, status (one entry per problem) and
    the workspace; keeps references to A and b for the plan's life."""

    def __init__(self, problems, opts: Opts | None = None, device="cuda"):
        self.opts = opts or Opts()
        self._keep = []
        count = len(problems)
        self.x = []
        self.rnorm = torch.empty(count, dtype=torch.float64, device=device)
        self.iters = torch.empty(count, dtype=torch.int32, device=device)
        self.status = torch.empty(count, dtype=torch.int32, device=device)
        arr = (Problem * count)()
        for i, (A, b, r, seed) in enumerate(problems):
            n, d = A.shape
            lda = _check_colmajor(A, "A")
            x = torch.empty(d, dtype=torch.float64, device=device)
            self.x.append(x)
            self._keep.append((A, b))
            arr[i] = Problem(n, d, r, seed & (2**64 - 1), A.data_ptr(), lda, b.data_ptr(),
                             x.data_ptr(), self.rnorm[i:].data_ptr(), self.iters[i:].data_ptr(),
                             self.status[i:].data_ptr())
        self._arr = arr
        lib = load()
        self._plan = ctypes.c_void_p()
        bad = ctypes.c_int32(-1)
        nbytes = int(lib.rnnls_batch_workspace_bytes(count, arr, ctypes.byref(self.opts)))
        if nbytes == 0:  # let the library name the invalid argument / problem
            rc = lib.rnnls_batch_create(ctypes.byref(self._plan), count, arr,
                                        ctypes.byref(self.opts), None, 0, ctypes.byref(bad))
            raise RnnlsError(f"rnnls_batch_create (problem {bad.value}) returned {rc}")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        rc = lib.rnnls_batch_create(ctypes.byref(self._plan), count, arr, ctypes.byref(self.opts),
                                    _ptr(self.ws), self.ws.numel(), ctypes.byref(bad))
        _check(rc, f"rnnls_batch_create (problem {bad.value})")

    def run(self, stream=None):
        _check(load().rnnls_batch_run(self._plan, _stream(stream)), "rnnls_batch_run")

    def autotune(self, stream=None) -> tuple[int, int]:
        t = Tuning()
        _check(load().rnnls_batch_autotune(self._plan, _stream(stream), ctypes.byref(t)),
               "rnnls_batch_autotune")
        return t.srht_log_tile, t.srht_wgs_per_cu

    def capture(self):
        _check(load().rnnls_batch_capture(self._plan), "rnnls_batch_capture")

    def launch(self, stream=None):
        _check(load().rnnls_batch_launch(self._plan, _stream(stream)), "rnnls_batch_launch")

    def columns(self) -> int:
        n = ctypes.c_int64(0)
        _check(load().rnnls_batch_columns(self._plan, ctypes.byref(n)), "rnnls_batch_columns")
        return int(n.value)

    def features(self, with_passive: bool = True, stream=None):
        """(X (columns, 8) float32, passive flags (columns,) uint8 or None) of
        the last pass, problems in order."""
        cols = self.columns()
        dev = self.rnorm.device
        X = torch.empty((cols, MLP_FEATURES), dtype=torch.float32, device=dev)
        y = torch.empty(cols, dtype=torch.uint8, device=dev) if with_passive else None
        _check(load().rnnls_batch_features(self._plan, _ptr(X), _ptr(y), _stream(stream)),
               "rnnls_batch_features")
        return X, y

    def set_model(self, mlp, threshold: float = 0.5):
        """Warm-start later passes from the perceptron `mlp` (None: cold)."""
        self._mlp = mlp
        theta = _ptr(mlp.theta) if mlp is not None else None
        wb = _ptr(mlp.wb) if mlp is not None else None
        _check(load().rnnls_batch_set_model(self._plan, theta, wb, float(threshold)),
               "rnnls_batch_set_model")

    def warm_used(self, stream=None) -> torch.Tensor:
        out = torch.empty(len(self.x), dtype=torch.int32, device=self.rnorm.device)
        _check(load().rnnls_batch_warm_used(self._plan, _ptr(out), _stream(stream)),
               "rnnls_batch_warm_used")
        return out

    def proposal(self, stream=None) -> torch.Tensor:
        """The last warm-started pass's proposal flags (columns,) uint8."""
        out = torch.empty(self.columns(), dtype=torch.uint8, device=self.rnorm.device)
        _check(load().rnnls_batch_proposal(self._plan, _ptr(out), _stream(stream)),
               "rnnls_batch_proposal")
        return out

    def close(self):
        if self._plan:
            load().rnnls_batch_destroy(self._plan)
            self._plan = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def features(G: torch.Tensor, q: torch.Tensor, c: torch.Tensor, stream=None) -> torch.Tensor:
    """Per-column features (d, 8) of one problem from its device Gram form."""
    d = q.numel()
    X = torch.empty((d, MLP_FEATURES), dtype=torch.float32, device=q.device)
    _check(load().rnnls_features(d, _ptr(G.contiguous()), _ptr(q), _ptr(c), _ptr(X),
                                 _stream(stream)), "rnnls_features")
    return X


class Mlp:
    """Device parameters of the passive-set perceptron: FP32 master theta,
    BF16 copy wb of the weights, Adam moments m, v."""

    def __init__(self, theta: torch.Tensor):
        assert theta.numel() == MLP_PARAMS and theta.dtype == torch.float32 and theta.is_cuda
        self.theta = theta.contiguous()
        self.wb = torch.empty(MLP_BF16_WEIGHTS, dtype=torch.int16, device=theta.device)
        self.m = torch.zeros_like(self.theta)
        self.v = torch.zeros_like(self.theta)
        self.step = 0
        self._ws = None
        _check(load().rnnls_mlp_sync_bf16(_ptr(self.theta), _ptr(self.wb),
                                          _stream(None)), "rnnls_mlp_sync_bf16")

    def _workspace(self, rows):
        need = int(load().rnnls_mlp_workspace_bytes(rows))
        if need == 0:
            raise RnnlsError("invalid row count")
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device=self.theta.device)
        return self._ws

    def forward(self, X: torch.Tensor, threshold: float = 0.5, stream=None):
        rows = X.shape[0]
        prob = torch.empty(rows, dtype=torch.float32, device=X.device)
        flags = torch.empty(rows, dtype=torch.uint8, device=X.device)
        _check(load().rnnls_mlp_forward(rows, _ptr(X.contiguous()), _ptr(self.theta),
                                        _ptr(self.wb), _ptr(prob), _ptr(flags),
                                        float(threshold), _stream(stream)), "rnnls_mlp_forward")
        return prob, flags

    def gradient(self, X: torch.Tensor, y: torch.Tensor, stream=None):
        rows = X.shape[0]
        ws = self._workspace(rows)
        grad = torch.empty(MLP_PARAMS, dtype=torch.float32, device=X.device)
        loss = torch.empty(1, dtype=torch.float32, device=X.device)
        _check(load().rnnls_mlp_gradient(rows, _ptr(X.contiguous()), _ptr(y.contiguous()),
                                         _ptr(self.theta), _ptr(self.wb), _ptr(grad), _ptr(loss),
                                         _ptr(ws), ws.numel(), _stream(stream)),
               "rnnls_mlp_gradient")
        return grad, loss

    def adam(self, grad: torch.Tensor, lr: float, stream=None):
        self.step += 1
        _check(load().rnnls_mlp_adam(_ptr(self.theta), _ptr(self.wb), _ptr(grad), _ptr(self.m),
                                     _ptr(self.v), self.step, float(lr), 0.9, 0.999, 1e-8,
                                     _stream(stream)), "rnnls_mlp_adam")

    def train_step(self, X: torch.Tensor, y: torch.Tensor, lr: float, loss=None, stream=None):
        rows = X.shape[0]
        ws = self._workspace(rows)
        self.step += 1
        _check(load().rnnls_mlp_train_step(rows, _ptr(X), _ptr(y), _ptr(self.theta),
                                           _ptr(self.wb), _ptr(self.m), _ptr(self.v), self.step,
                                           float(lr), _ptr(loss), _ptr(ws), ws.numel(),
                                           _stream(stream)), "rnnls_mlp_train_step")


def timing_enable(on: bool = True) -> None:
    _check(load().rnnls_timing_enable(1 if on else 0), "rnnls_timing_enable")


def timing_read(which: int) -> tuple[float, int]:
    """(summed ms, launches) of one kernel timer since its last read."""
    ms = ctypes.c_double(0.0)
    k = ctypes.c_int64(0)
    _check(load().rnnls_timing_read(which, ctypes.byref(ms), ctypes.byref(k)), "rnnls_timing_read")
    return ms.value, k.value


def set_tuning(srht_log_tile: int = 0, srht_wgs_per_cu: int = 0) -> None:
    """Launch shape of the sketch kernel (0 = automatic), process-wide."""
    t = Tuning(int(srht_log_tile), int(srht_wgs_per_cu))
    _check(load().rnnls_set_tuning(ctypes.byref(t)), "rnnls_set_tuning")


def stream_read(x: torch.Tensor, partials: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Read x (contiguous FP32 on the device) once on the streaming-read
    reference kernel (rnnls_stream_read); returns the per-workgroup partial sums."""
    if x.dtype != torch.float32 or not x.is_contiguous():
        raise RnnlsError("stream_read needs a contiguous float32 tensor")
    nb = load().rnnls_stream_read_blocks()
    if partials is None:
        partials = torch.empty(nb, dtype=torch.float32, device=x.device)
    elif partials.numel() < nb or partials.dtype != torch.float32:
        raise RnnlsError(f"stream_read needs {nb} float32 partials")
    _check(load().rnnls_stream_read(_ptr(x), x.numel(), _ptr(partials), _stream(stream)),
           "rnnls_stream_read")
    return partials


def get_tuning() -> tuple[int, int]:
    t = Tuning()
    _check(load().rnnls_get_tuning(ctypes.byref(t)), "rnnls_get_tuning")
    return t.srht_log_tile, t.srht_wgs_per_cu


def tuning_cache_entries() -> int:
    """Entries of the autotuner's process-wide cache (one per plan shape)."""
    return int(load().rnnls_tuning_cache_entries())


def tuning_cache_clear() -> None:
    _check(load().rnnls_tuning_cache_clear(), "rnnls_tuning_cache_clear")


def tuning_cache_save(path: str) -> None:
    """Write the autotuner's cache to a text file."""
    _check(load().rnnls_tuning_cache_save(os.fsencode(path)), "rnnls_tuning_cache_save")


def tuning_cache_load(path: str) -> None:
    """Merge a file written by tuning_cache_save into the autotuner's cache."""
    _check(load().rnnls_tuning_cache_load(os.fsencode(path)), "rnnls_tuning_cache_load")
