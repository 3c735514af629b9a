"""GPU parity of whole outputs at the benchmark sizes, against the FP64 oracle
(its sketch computed column chunk by column chunk in worker processes).

  * tf-idf-like 2^22 x 128, r = 8192 (the precision form's size): every
    column of the FP32 sketch within 1e-5 and of the split-BF16 sketch within
    2e-4 (norm-wise per column) of the oracle's; x~ of both transforms within
    1e-6 relative residual gap of the oracle's Lawson-Hanson on the oracle's
    own sketch, and on the full problem (where both residuals are stationary
    on the support, so the gap is second order in the sketch difference).
  * the exact solve of a whole 2^20 x 64 problem (all rows: the plain
    comparison of Section 4.1), against the oracle's Lawson-Hanson on the
    equivalent 64-row problem (R, Q^T b) of the thin QR A = QR: the two
    problems share every x's residual up to the constant ||(I - QQ^T) b||^2.
  * every instance of the 256-problem batch and every one of the 512
    right-hand sides of the multi-RHS workload.
"""
import numpy as np
import pytest
import torch

import oracle_pool
from oracle import nnls, rng
from paper_0812_4547_amd import rnnls, workloads

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5
SPLIT_TOL = 2e-4
GAP_TOL = 1e-6


@pytest.fixture(scope="module", autouse=True)
def _lib():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    rnnls.load()
    yield
    torch.cuda.synchronize()


def _colwise_rel(got, want):
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    num = np.linalg.norm(got - want, axis=0)
    den = np.maximum(np.linalg.norm(want, axis=0), 1e-30)
    return num / den


def _full_gap(A, b, x, x_ref):
    A64 = np.asarray(A, np.float64)
    b64 = np.asarray(b, np.float64)
    return float(np.linalg.norm(A64 @ x - b64) / np.linalg.norm(A64 @ x_ref - b64) - 1.0)


@pytest.fixture(scope="module")
def big():
    n, d, r, seed = 1 << 22, 128, 8192, 3
    print("2^22 x 128: data and the oracle sketch", flush=True)
    p = workloads.tfidf_like(n, d, seed=seed)
    Y, R = oracle_pool.sketch(np.column_stack([p.A, p.b]), r, seed)
    ref = nnls.lawson_hanson(Y[:, :d], Y[:, d])
    return p, r, seed, Y, R, ref


@pytest.mark.parametrize("precision,tol", [("fp32", FP32_TOL), ("split_bf16", SPLIT_TOL)])
def test_whole_sketch_and_solution_2p22x128(big, precision, tol):
    p, r, seed, Y, R, ref = big
    d = p.A.shape[1]
    print(f"2^22 x 128 r={r} {precision}", flush=True)
    sol = rnnls.rand_nnls(rnnls.colmajor(p.A), torch.from_numpy(p.b).cuda(), r, seed,
                          opts=rnnls.make_opts(precision=precision), keep_sketch=True)
    torch.cuda.synchronize()
    assert int(sol.status.item()) == rnnls.SOLVE_OK
    assert int(sol.sketch.count.item()) == r
    assert np.array_equal(sol.sketch.rows.cpu().numpy(), R)
    got = np.column_stack([sol.sketch.SA.cpu().numpy(), sol.sketch.Sb.cpu().numpy()])
    err = _colwise_rel(got, Y)
    print(f"  column errors: max {err.max():.2e}, median {np.median(err):.2e}", flush=True)
    assert err.max() <= tol
    x = sol.x.cpu().numpy()
    assert (x >= 0).all()
    g_sk = nnls.relative_residual_gap(Y[:, :d], Y[:, d], x, ref.x)
    g_full = _full_gap(p.A, p.b, x, ref.x)
    print(f"  gap on the oracle sketch {g_sk:+.2e}, on the full problem {g_full:+.2e}", flush=True)
    assert abs(g_sk) <= GAP_TOL
    assert abs(g_full) <= GAP_TOL


def test_exact_full_problem_solve_2p20x64():
    n, d = 1 << 20, 64
    print("exact solve on all 2^20 rows", flush=True)
    p = workloads.tfidf_like(n, d, seed=2)
    sol = rnnls.nnls_solve(rnnls.colmajor(p.A), torch.from_numpy(p.b).cuda())
    torch.cuda.synchronize()
    assert int(sol.status.item()) == rnnls.SOLVE_OK
    A64, b64 = p.A.astype(np.float64), p.b.astype(np.float64)
    Q, Rq = np.linalg.qr(A64, mode="reduced")
    # the full problem's tolerance (its 1-norm and row count), not the 64-row one's
    ref = nnls.lawson_hanson(Rq, Q.T @ b64, tol=nnls.default_tol(A64))
    x = sol.x.cpu().numpy()
    assert (x >= 0).all()
    gap = _full_gap(A64, b64, x, ref.x)
    print(f"  full-problem gap {gap:+.2e}, support {(x > 0).sum()} vs {(ref.x > 0).sum()}",
          flush=True)
    assert abs(gap) <= GAP_TOL
    # the returned dual is A^T (b - A x) of the returned x, and certifies it
    w = A64.T @ (b64 - A64 @ x)
    scale = np.abs(A64).sum(axis=0).max() * np.abs(b64).max()
    assert np.max(np.abs(sol.w.cpu().numpy() - w)) <= 1e-10 * scale
    tau = nnls.default_tol(A64)
    assert np.all(w[x == 0] <= 1e3 * tau)


def test_every_batch_instance_against_oracle():
    shapes = workloads.batch_shapes()
    print(f"all {len(shapes)} instances of the batch", flush=True)
    dev = []
    for i, (n, d, r) in enumerate(shapes):
        p = workloads.batch_instance(i, n, d, batch_seed=4)
        dev.append((rnnls.colmajor(p.A), torch.from_numpy(p.b).cuda(), r, 1000 + i))
    batch = rnnls.Batch(dev)
    batch.run()
    torch.cuda.synchronize()
    st = batch.status.cpu().numpy()
    assert (st == rnnls.SOLVE_OK).all()
    cases = [(i, n, d, r, 1000 + i, batch.x[i].cpu().numpy())
             for i, (n, d, r) in enumerate(shapes)]
    batch.close()
    del dev, batch
    res = oracle_pool.batch_gaps(cases, batch_seed=4)
    g_sk = np.array([g for g, _, _ in res])
    g_full = np.array([g for _, g, _ in res])
    print(f"  max |gap| on the oracle sketches {np.abs(g_sk).max():.2e}, "
          f"on the full problems {np.abs(g_full).max():.2e}", flush=True)
    assert all(s == 0 for _, _, s in res)
    assert np.abs(g_sk).max() <= GAP_TOL
    assert np.abs(g_full).max() <= GAP_TOL


def test_every_right_hand_side_2p20x64_k512():
    n, d, k, r, seed = 1 << 20, 64, 512, 2048, 4
    print("multi-RHS 2^20 x 64 with 512 right-hand sides, all of them", flush=True)
    A, B, _ = workloads.tfidf_multi_rhs(n, d, k, seed=seed)
    sol = rnnls.rand_nnls_multi(rnnls.colmajor(A), rnnls.colmajor(B), r, seed)
    torch.cuda.synchronize()
    assert (sol.status.cpu().numpy() == rnnls.SOLVE_OK).all()
    Xd = sol.X.cpu().numpy()
    rows = rng.rows_exact(seed, n, r)
    Y, R = oracle_pool.sketch(np.column_stack([A, B]), r, seed)
    assert np.array_equal(R, rows)
    SA, SB = Y[:, :d], Y[:, d:]
    Xo, so = oracle_pool.lawson_hanson_many(SA, SB)
    assert (so == 0).all()
    gaps = np.array([nnls.relative_residual_gap(SA, SB[:, j], Xd[:, j], Xo[:, j])
                     for j in range(k)])
    print(f"  max |gap| over the {k} right-hand sides {np.abs(gaps).max():.2e}", flush=True)
    assert (Xd >= 0).all()
    assert np.abs(gaps).max() <= GAP_TOL
