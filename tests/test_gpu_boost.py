"""Repetition of Algorithm 1 on the device (rnnls_rand_nnls_boost) against the
host and the oracle: the residual pass, the selection and the kept x~."""
import numpy as np
import pytest
import torch

from oracle import rand_nnls as orand
from paper_0812_4547_amd import rnnls, workloads

pytestmark = pytest.mark.gpu


def _colmajor(A: np.ndarray, pad: int) -> torch.Tensor:
    n, d = A.shape
    buf = torch.zeros((d, n + pad), dtype=torch.float32)
    buf[:, :n] = torch.from_numpy(np.ascontiguousarray(A.T))
    return buf.cuda().t()[:n]


def _expected_best(resid, status):
    ok = status == 0
    pool = np.flatnonzero(ok) if ok.any() else np.arange(len(resid))
    return int(pool[np.argmin(resid[pool])])


def _case(n, d, r, k, seed, ds, pad=0, with_oracle=True):
    print(f"boost n={n} d={d} r={r} k={k} seed={seed} pad={pad}", flush=True)
    p = workloads.tfidf_like(n, d, seed=ds)
    A = _colmajor(p.A, pad)
    b = torch.from_numpy(p.b).cuda()
    out = rnnls.rand_nnls_boost(A, b, r, k, seed)
    torch.cuda.synchronize()
    A64, b64 = p.A.astype(np.float64), p.b.astype(np.float64)
    runs = [rnnls.rand_nnls(A, b, r, seed + i) for i in range(k)]
    xs = [run.x.cpu().numpy() for run in runs]
    st = np.array([int(run.status.item()) for run in runs])
    res_host = np.array([np.linalg.norm(A64 @ x - b64) for x in xs])
    resid = out.resid.cpu().numpy()[:k]
    # the residual pass: FP64 residuals of the same candidates
    np.testing.assert_allclose(resid, res_host, rtol=1e-10, atol=0)
    # the selection: least residual among finished solves, lowest index on ties,
    # and the kept x~ is that candidate bit for bit (every run is deterministic)
    best = int(out.best.item())
    assert best == _expected_best(resid, st)
    assert np.array_equal(out.x.cpu().numpy(), xs[best])
    assert int(out.status.item()) == st[best]
    if with_oracle:
        ob = orand.rand_nnls_boost(p.A, p.b, r, k, seed)
        np.testing.assert_allclose(res_host, ob.residuals, rtol=1e-6, atol=0)
        assert res_host[best] <= ob.residuals.min() * (1 + 1e-6)


@pytest.mark.parametrize("n,d,r,k,seed,pad", [
    (3 * 16384 + 1234, 24, 600, 4, 7, 0),   # ragged n: guarded rows in the residual pass
    (1 << 15, 40, 1200, 8, 11, 1),          # odd leading dimension: element loads
    ((1 << 14) + 3, 10, 300, 1, 5, 0),      # one repetition is Algorithm 1
    (20000, 33, 900, 3, 21, 0),
])
def test_boost_against_host_and_oracle(n, d, r, k, seed, pad):
    _case(n, d, r, k, seed, ds=seed + 50, pad=pad)


def test_boost_full_size_residuals_and_selection():
    """The single-instance workload's size (2^20 x 64, r = 4096), four
    repetitions: residual pass and selection against the host."""
    _case(1 << 20, 64, 4096, 4, 2, ds=2, with_oracle=False)


def test_boost_single_repetition_equals_rand_nnls():
    p = workloads.tfidf_like(1 << 16, 20, seed=9)
    A = rnnls.colmajor(p.A)
    b = torch.from_numpy(p.b).cuda()
    out = rnnls.rand_nnls_boost(A, b, 700, 1, 123)
    one = rnnls.rand_nnls(A, b, 700, 123)
    torch.cuda.synchronize()
    assert int(out.best.item()) == 0
    assert torch.equal(out.x, one.x)


def test_boost_bernoulli_sampling():
    """Repetition with the paper's Bernoulli row sampling: each candidate is the
    Bernoulli-mode Algorithm 1 run of its seed."""
    print("boost bernoulli", flush=True)
    p = workloads.tfidf_like(40000, 30, seed=17)
    A = rnnls.colmajor(p.A)
    b = torch.from_numpy(p.b).cuda()
    opts = rnnls.make_opts("bernoulli")
    k, r, seed = 3, 900, 31
    out = rnnls.rand_nnls_boost(A, b, r, k, seed, opts=opts)
    torch.cuda.synchronize()
    runs = [rnnls.rand_nnls(A, b, r, seed + i, opts=opts) for i in range(k)]
    xs = [run.x.cpu().numpy() for run in runs]
    st = np.array([int(run.status.item()) for run in runs])
    A64, b64 = p.A.astype(np.float64), p.b.astype(np.float64)
    res = np.array([np.linalg.norm(A64 @ x - b64) for x in xs])
    np.testing.assert_allclose(out.resid.cpu().numpy()[:k], res, rtol=1e-10, atol=0)
    best = int(out.best.item())
    assert best == _expected_best(res, st)
    assert np.array_equal(out.x.cpu().numpy(), xs[best])
    ob = orand.rand_nnls_boost(p.A, p.b, r, k, seed, mode="bernoulli")
    np.testing.assert_allclose(res, ob.residuals, rtol=1e-6, atol=0)
