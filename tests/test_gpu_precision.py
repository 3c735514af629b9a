"""GPU parity of the precision form: the in-tile Hadamard factors on BF16
matrix cores with split hi + lo operands and FP32 accumulation, against the
FP64 oracle.

Bars: rows and counts bit-exact; sketch columns within 2e-4 relative
(norm-wise per column); x~ within 1e-6 relative residual gap of the oracle's
Lawson-Hanson on the oracle's FP64 sketch (the solve stays FP64).  Each test
prints the measured errors.
"""
import numpy as np
import pytest
import torch

from oracle import hadamard, nnls, rng
from paper_0812_4547_amd import rnnls, workloads

pytestmark = pytest.mark.gpu

SPLIT_TOL = 2e-4
FP32_TOL = 1e-5
GAP_TOL = 1e-6
SPLIT = rnnls.make_opts(precision="split_bf16")


@pytest.fixture(scope="module", autouse=True)
def _lib():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    rnnls.load()
    yield
    torch.cuda.synchronize()


def _colwise_rel(got, want):
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    if got.ndim == 1:
        got, want = got[:, None], want[:, None]
    num = np.linalg.norm(got - want, axis=0)
    den = np.maximum(np.linalg.norm(want, axis=0), 1e-30)
    return float(np.max(num / den))


@pytest.mark.parametrize("n,d,r,seed", [(32768, 16, 1000, 1), (3 * 32768 + 1234, 20, 2048, 2),
                                        (16384, 9, 700, 3), (20000, 5, 4096, 4),
                                        (131072, 64, 8192, 5), (70001, 1, 300, 6)])
def test_split_sketch_against_oracle(n, d, r, seed):
    p = workloads.tfidf_like(n, d, seed=seed, mean_density=0.05)
    A = rnnls.colmajor(p.A)
    b = torch.from_numpy(p.b).cuda()
    sk = rnnls.srht_sketch(A, b, r, seed, opts=SPLIT)
    torch.cuda.synchronize()
    SA, Sb, R, _ = hadamard.srht_sketch(p.A.astype(np.float64), p.b.astype(np.float64), r, seed)
    assert int(sk.count.item()) == r
    assert np.array_equal(sk.rows.cpu().numpy(), R)
    err = max(_colwise_rel(sk.SA.cpu().numpy(), SA), _colwise_rel(sk.Sb.cpu().numpy(), Sb))
    print(f"split-bf16 sketch n={n} d={d} r={r}: max column error {err:.2e}", flush=True)
    assert err <= SPLIT_TOL


def test_split_sketch_unaligned_columns():
    n, d, r, seed = 40000, 6, 900, 7
    p = workloads.tfidf_like(n, d, seed=seed, mean_density=0.05)
    big = torch.zeros((d, n + 3), dtype=torch.float32, device="cuda")
    big[:, :n] = torch.from_numpy(np.ascontiguousarray(p.A.T)).cuda()
    A = big.t()[:n]  # lda = n + 3: not a multiple of 4
    sk = rnnls.srht_sketch(A, None, r, seed, opts=SPLIT)
    torch.cuda.synchronize()
    SA, _, _, _ = hadamard.srht_sketch(p.A.astype(np.float64), None, r, seed)
    assert _colwise_rel(sk.SA.cpu().numpy(), SA) <= SPLIT_TOL


def test_small_problems_use_the_fp32_transform():
    n, d, r, seed = 5000, 7, 600, 8
    p = workloads.tfidf_like(n, d, seed=seed, mean_density=0.05)
    sk = rnnls.srht_sketch(rnnls.colmajor(p.A), None, r, seed, opts=SPLIT)
    torch.cuda.synchronize()
    SA, _, _, _ = hadamard.srht_sketch(p.A.astype(np.float64), None, r, seed)
    assert _colwise_rel(sk.SA.cpu().numpy(), SA) <= FP32_TOL


def test_split_rejects_too_many_rows():
    A = torch.zeros((1, 1 << 15), dtype=torch.float32, device="cuda").t()
    with pytest.raises(rnnls.RnnlsError, match="-102"):
        rnnls.srht_sketch(A, None, 17000, 1, opts=SPLIT)


@pytest.mark.parametrize("n,d,r,seed", [(65536, 24, 1500, 11), (200000, 64, 4096, 12)])
def test_split_rand_nnls_against_oracle(n, d, r, seed):
    p = workloads.tfidf_like(n, d, seed=seed)
    sol = rnnls.rand_nnls(rnnls.colmajor(p.A), torch.from_numpy(p.b).cuda(), r, seed,
                          opts=SPLIT, keep_sketch=True)
    torch.cuda.synchronize()
    assert int(sol.status.item()) == rnnls.SOLVE_OK
    SA, Sb, _, _ = hadamard.srht_sketch(p.A.astype(np.float64), p.b.astype(np.float64), r, seed)
    ref = nnls.lawson_hanson(SA, Sb)
    x = sol.x.cpu().numpy()
    gap = nnls.relative_residual_gap(SA, Sb, x, ref.x)
    full = (np.linalg.norm(p.A.astype(np.float64) @ x - p.b) /
            np.linalg.norm(p.A.astype(np.float64) @ ref.x - p.b) - 1.0)
    err = _colwise_rel(sol.sketch.SA.cpu().numpy(), SA)
    print(f"split-bf16 rand_nnls n={n} d={d}: sketch error {err:.2e}, gap on the oracle sketch "
          f"{gap:.2e}, full-problem residual vs the oracle's x~ {full:+.2e}", flush=True)
    assert err <= SPLIT_TOL
    assert gap <= GAP_TOL
    assert abs(full) <= 1e-5


