"""The allocation-free entry point (rnnls_rand_nnls_noalloc) against the
workspace entry point (rnnls_rand_nnls) through the C-ABI: two calls in a row,
the second on a smaller problem (the fixed scratch keeps the first call's
contents), each compared with the workspace path on the same inputs.  Both
run the same kernels on the same data, so the outputs must agree bit for bit;
x~ is also held to the oracle's bar (1e-6 relative residual gap on the
oracle's sketch)."""
import numpy as np
import pytest
import torch

from oracle import hadamard, nnls
from paper_0812_4547_amd import rnnls, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    rnnls.load()
    yield
    torch.cuda.synchronize()


def _both(p, r, seed, opts):
    A = rnnls.colmajor(p.A)
    b = torch.from_numpy(p.b).cuda()
    ref = rnnls.rand_nnls(A, b, r, seed, opts=opts, keep_sketch=True)
    got = rnnls.rand_nnls_noalloc(A, b, r, seed, opts=opts, keep_sketch=True)
    torch.cuda.synchronize()
    return ref, got


def _same(ref, got):
    cnt = int(ref.sketch.count.item())
    assert int(got.sketch.count.item()) == cnt
    assert torch.equal(got.sketch.rows[:cnt], ref.sketch.rows[:cnt])
    assert torch.equal(got.sketch.SA[:cnt], ref.sketch.SA[:cnt])
    assert torch.equal(got.sketch.Sb[:cnt], ref.sketch.Sb[:cnt])
    for name in ("x", "rnorm", "iters", "status"):
        assert torch.equal(getattr(got, name), getattr(ref, name)), name


@pytest.mark.parametrize("mode", ["exact", "bernoulli"])
def test_noalloc_matches_workspace_entry_twice(mode):
    opts = rnnls.make_opts(mode)
    cases = [(workloads.tfidf_like(1 << 20, 64, seed=2), 4096, 2),
             (workloads.tfidf_like(50000, 12, seed=5), 700, 9)]
    for p, r, seed in cases:
        print(f"noalloc {mode} n={p.A.shape[0]} d={p.A.shape[1]} r={r}", flush=True)
        ref, got = _both(p, r, seed, opts)
        _same(ref, got)
        assert int(got.status.item()) == rnnls.SOLVE_OK
        SA, Sb, _, _ = hadamard.srht_sketch(p.A.astype(np.float64), p.b.astype(np.float64), r,
                                            seed, mode)
        oref = nnls.lawson_hanson(SA, Sb)
        gap = nnls.relative_residual_gap(SA, Sb, got.x.cpu().numpy(), oref.x)
        assert abs(gap) <= 1e-6


def test_noalloc_rejects_sizes_beyond_its_scratch():
    n, d, r = 1 << 20, 128, 32768
    need = rnnls.workspace_bytes(rnnls.OP_RAND_NNLS, n, d, r)
    assert need > rnnls.NOALLOC_SCRATCH_BYTES
    A = torch.zeros((d, n), dtype=torch.float32, device="cuda").t()
    b = torch.zeros(n, dtype=torch.float32, device="cuda")
    with pytest.raises(rnnls.RnnlsError, match=str(rnnls.E_WORKSPACE)):
        rnnls.rand_nnls_noalloc(A, b, r, 1)
    # invalid arguments are named as by the workspace entry point
    with pytest.raises(rnnls.RnnlsError, match="-3"):
        rnnls.rand_nnls_noalloc(A[:1000], b[:1000], 2000, 1)
