"""GPU parity of the batching forms: many right-hand sides sharing A
(rnnls_rand_nnls_multi) and batch plans of uneven problems (rnnls_batch_*),
against the FP64 oracle, plus graph-replay and autotune consistency.

Bars as for the single path: x~ within 1e-6 relative residual gap of the
oracle's Lawson-Hanson on the oracle's sketch, statuses OK, KKT held.
"""
import numpy as np
import pytest
import torch

from oracle import hadamard, nnls
from paper_0812_4547_amd import rnnls, workloads

pytestmark = pytest.mark.gpu

GAP_TOL = 1e-6


@pytest.fixture(scope="module", autouse=True)
def _lib():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    rnnls.load()
    yield
    torch.cuda.synchronize()


def _gap_ok(SA, Sb, x):
    ref = nnls.lawson_hanson(SA, Sb)
    gap = nnls.relative_residual_gap(SA, Sb, np.asarray(x, np.float64), ref.x)
    return gap


# ------------------------------------------------------------ many right-hand sides
@pytest.mark.parametrize("n,d,k,r,seed", [(9000, 12, 20, 700, 21), (70000, 40, 70, 1300, 3),
                                          (40000, 90, 9, 3000, 8)])
def test_multi_rhs_against_oracle(n, d, k, r, seed):
    print(f"multi case n={n} d={d} k={k} r={r}", flush=True)
    A, B, _ = workloads.tfidf_multi_rhs(n, d, k, seed=seed)
    sol = rnnls.rand_nnls_multi(rnnls.colmajor(A), rnnls.colmajor(B), r, seed)
    torch.cuda.synchronize()
    assert (sol.status.cpu().numpy() == rnnls.SOLVE_OK).all()
    Y, _, _, _ = hadamard.srht_sketch(np.column_stack([A, B]).astype(np.float64), None, r, seed)
    SA, SB = Y[:, :d], Y[:, d:]
    X = sol.X.cpu().numpy()
    rn = sol.rnorm.cpu().numpy()
    for j in range(k):
        assert _gap_ok(SA, SB[:, j], X[:, j]) <= GAP_TOL, j
        assert (X[:, j] >= 0).all()
        res = np.linalg.norm(SA @ X[:, j] - SB[:, j])
        assert abs(rn[j] - res) <= 1e-5 * max(res, 1e-12) + 1e-9


def test_multi_rhs_one_column_equals_single_path():
    p = workloads.tfidf_like(50000, 30, seed=9)
    A = rnnls.colmajor(p.A)
    b = torch.from_numpy(p.b).cuda()
    one = rnnls.rand_nnls(A, b, 1500, 77)
    multi = rnnls.rand_nnls_multi(A, b[:, None], 1500, 77)
    torch.cuda.synchronize()
    assert torch.equal(one.x, multi.X[:, 0])


# ------------------------------------------------------------ batch plans
SMALL_BATCH = [(3000, 5, 1024), (5000, 40, 1280), (17000, 8, 1024), (33000, 20, 1024),
               (70000, 96, 3072), (2047, 3, 500), (40000, 64, 2048), (16384, 17, 1024),
               (65536, 33, 1056), (100000, 70, 2240), (4096, 1, 100), (131072, 128, 4096)]


def _make_batch(shapes, batch_seed, opts=None):
    probs, dev = [], []
    for i, (n, d, r) in enumerate(shapes):
        p = workloads.batch_instance(i, n, d, batch_seed=batch_seed)
        A = rnnls.colmajor(p.A)
        b = torch.from_numpy(p.b).cuda()
        seed = 1000 + i
        probs.append((p, r, seed))
        dev.append((A, b, r, seed))
    return probs, rnnls.Batch(dev, opts=opts)


def _check_against_oracle(probs, batch, which=None, mode="exact"):
    st = batch.status.cpu().numpy()
    for i, (p, r, seed) in enumerate(probs):
        if which is not None and i not in which:
            continue
        assert st[i] == rnnls.SOLVE_OK, (i, st[i])
        SA, Sb, _, _ = hadamard.srht_sketch(p.A.astype(np.float64), p.b.astype(np.float64), r,
                                            seed, mode)
        x = batch.x[i].cpu().numpy()
        assert (x >= 0).all()
        assert _gap_ok(SA, Sb, x) <= GAP_TOL, i


def test_batch_uneven_against_oracle_and_single_path():
    probs, batch = _make_batch(SMALL_BATCH, batch_seed=11)
    batch.run()
    torch.cuda.synchronize()
    _check_against_oracle(probs, batch)
    for i, (p, r, seed) in enumerate(probs):
        one = rnnls.rand_nnls(rnnls.colmajor(p.A), torch.from_numpy(p.b).cuda(), r, seed)
        torch.cuda.synchronize()
        xb = batch.x[i].cpu().numpy()
        xs = one.x.cpu().numpy()
        # same problem up to the FP32 rounding order of the sketch sums: same
        # support, x equal to ~cond(SA) * 1e-7
        assert np.array_equal(xb > 0, xs > 0), i
        assert np.abs(xb - xs).max() <= 1e-6 * max(1.0, np.abs(xs).max()), i
    batch.close()


def test_batch_bernoulli_mode():
    opts = rnnls.make_opts(sample_mode="bernoulli")
    probs, batch = _make_batch(SMALL_BATCH[:6], batch_seed=12, opts=opts)
    batch.run()
    torch.cuda.synchronize()
    _check_against_oracle(probs, batch, mode="bernoulli")
    batch.close()


def test_batch_autotune_capture_and_replay():
    probs, batch = _make_batch(SMALL_BATCH, batch_seed=13)
    choice = batch.autotune()
    assert choice in [(15, 1), (14, 1), (14, 2), (13, 2), (13, 3), (13, 4), (12, 4), (12, 8)]
    batch.run()
    torch.cuda.synchronize()
    eager = [x.clone() for x in batch.x]
    _check_against_oracle(probs, batch, which={0, 4, 5, 11})
    batch.capture()
    p0 = probs[1][0]
    for rep in range(3):
        for x in batch.x:
            x.fill_(-1.0)
        batch.launch()
        torch.cuda.synchronize()
        for i, x in enumerate(batch.x):
            assert torch.equal(x, eager[i]), (rep, i)
        # eager work of the program between replays
        one = rnnls.rand_nnls(rnnls.colmajor(p0.A), torch.from_numpy(p0.b).cuda(), 1280, rep)
        torch.cuda.synchronize()
        assert int(one.status.item()) == rnnls.SOLVE_OK
    batch.close()


def test_batch_rejects_invalid_problem():
    p = workloads.tfidf_like(5000, 4, seed=1)
    A = rnnls.colmajor(p.A)
    b = torch.from_numpy(p.b).cuda()
    with pytest.raises(rnnls.RnnlsError, match="problem 1"):
        rnnls.Batch([(A, b, 100, 1), (A, b, 9000, 2)])  # r >= n'


def test_autotune_choice_is_cached_by_plan_shape(tmp_path):
    """A second plan with the same shapes takes the first plan's choice from
    the cache (no new entry); the cache survives a save / clear / load."""
    rnnls.tuning_cache_clear()
    probs, b1 = _make_batch(SMALL_BATCH[:5], batch_seed=14)
    c1 = b1.autotune()
    assert rnnls.tuning_cache_entries() == 1
    probs2, b2 = _make_batch(SMALL_BATCH[:5], batch_seed=15)  # same shapes, other data
    assert b2.autotune() == c1 and rnnls.tuning_cache_entries() == 1
    path = str(tmp_path / "tune.txt")
    rnnls.tuning_cache_save(path)
    rnnls.tuning_cache_clear()
    rnnls.tuning_cache_load(path)
    assert rnnls.tuning_cache_entries() == 1
    probs3, b3 = _make_batch(SMALL_BATCH[:6], batch_seed=16)  # other shapes: timed, new entry
    b3.autotune()
    assert rnnls.tuning_cache_entries() == 2
    b2.run()
    torch.cuda.synchronize()
    _check_against_oracle(probs2, b2, which={0, 3})
    for b in (b1, b2, b3):
        b.close()
    rnnls.tuning_cache_clear()
