"""End-to-end pins for the oracle from the analysis of Algorithm 1
(Theorem 1, Lemma 1, Lemma 2 and the proof of Theorem 1)."""
import numpy as np
from scipy import stats

from oracle import diagnostics, hadamard, nnls, rand_nnls, rng
from paper_0812_4547_amd import workloads


def _full_opt(p):
    return nnls.lawson_hanson(p.A, p.b)


def test_proof_chain_holds_for_every_draw():
    # proof of Theorem 1: whenever the realised eps' < 1, the residual of x~ is
    # within (1+eps')/(1-eps') of the optimum (squared), deterministically
    p = workloads.uniform_planted(seed=1)
    opt = _full_opt(p)
    base = opt.rnorm ** 2
    checked = 0
    for seed in range(40):
        res = rand_nnls.rand_nnls(p.A, p.b, 512, seed)
        D = rng.signs(seed, 4096).astype(np.float64)
        eps = diagnostics.realised_eps(p.A, p.b, res.rows, D, 512)
        got = float(np.linalg.norm(p.A.astype(np.float64) @ res.x - p.b.astype(np.float64)) ** 2)
        assert got >= base * (1 - 1e-12)            # x_opt is optimal
        if eps < 1:
            checked += 1
            assert got <= diagnostics.chain_bound(eps) * base * (1 + 1e-10)
    assert checked >= 30


def test_theorem1_success_frequency():
    # Theorem 1: ||A x~ - b||^2 <= (1 + eps) min ||A x - b||^2 with probability
    # at least 1/2.  c_o is unspecified, so eps is taken where r = 512 rows of a
    # 17-column system is ample; the count must pass a one-sided binomial test
    p = workloads.uniform_planted(seed=2)
    base = _full_opt(p).rnorm ** 2
    ok = 0
    trials = 100
    for seed in range(trials):
        x = rand_nnls.rand_nnls(p.A, p.b, 512, 1000 + seed).x
        got = float(np.linalg.norm(p.A.astype(np.float64) @ x - p.b.astype(np.float64)) ** 2)
        ok += got <= 1.5 * base
    assert stats.binomtest(ok, trials, 0.5, alternative="less").pvalue > 0.01
    assert ok >= 50


def _coherent(n, d, seed):
    # leverage concentrated on d rows: identity block plus a tiny dense part
    g = np.random.default_rng(seed)
    A = 1e-3 * g.random((n, d))
    A[:d, :d] += np.eye(d)
    x = g.random(d)
    b = A @ x
    b[:d] += 0.1 * g.standard_normal(d)
    return A, b


def test_lemma2_flattens_leverage_on_coherent_input():
    n, d = 4096, 12
    A, b = _coherent(n, d, 0)
    U = diagnostics.orthonormal_basis(np.column_stack([A, -b]))
    assert np.max(np.sum(U * U, axis=1)) > 0.5          # coherent before mixing
    k = U.shape[1]
    passes = 0
    for seed in range(30):
        D = rng.signs(seed, n).astype(np.float64)
        passes += diagnostics.lemma2_max_row_norm(U, D) <= diagnostics.lemma2_bound(k, n)
    assert passes >= 27                                 # probability >= 0.9


def test_ablation_without_HD_breaks_the_embedding():
    # the sampling alone (no H D) misses the heavy rows of a coherent input and
    # its distortion reaches 1; with the randomised Hadamard transform it stays small
    n, d, r = 4096, 12, 256
    A, b = _coherent(n, d, 1)
    U = diagnostics.orthonormal_basis(np.column_stack([A, -b]))
    eps_srht, eps_plain = [], []
    for seed in range(10):
        D = rng.signs(seed, n).astype(np.float64)
        R = rng.rows_exact(seed, n, r)
        eps_srht.append(diagnostics.realised_eps(A, b, R, D, r))
        SU = U[R] * np.sqrt(n / r)
        eps_plain.append(float(np.linalg.norm(SU.T @ SU - np.eye(U.shape[1]), 2)))
    assert max(eps_srht) < 0.75
    assert min(eps_plain) >= 0.99


def test_sketch_of_tfidf_like_problem_keeps_residual_close():
    p = workloads.tfidf_like(1 << 14, 24, seed=5)
    opt = _full_opt(p)
    res = rand_nnls.rand_nnls(p.A, p.b, 1024, 5)
    gap = nnls.relative_residual_gap(p.A, p.b, res.x, opt.x)
    assert -1e-12 <= gap < 0.2
    assert res.solve.status == nnls.STATUS_OK
    assert nnls.kkt_ok(res.SA, res.Sb, res.x, 1e3 * nnls.default_tol(res.SA))


def test_padding_ragged_rows():
    # n not a power of two: rows n..n'-1 are zero and never matter
    g = np.random.default_rng(3)
    n = 3000
    A = g.random((n, 4))
    b = g.random(n)
    SA, Sb, R, D = hadamard.srht_sketch(A, b, 100, 4)
    assert D.shape[0] == 4096 and R.max() < 4096


def test_repetition_single_run_is_algorithm1():
    p = workloads.uniform_planted(seed=3)
    one = rand_nnls.rand_nnls(p.A, p.b, 512, 77)
    rep = rand_nnls.rand_nnls_boost(p.A, p.b, 512, 1, 77)
    assert rep.best == 0
    assert np.array_equal(rep.x, one.x)


def test_repetition_keeps_the_smallest_full_residual_and_grows_monotone():
    # the runs of k seeds are a prefix of the runs of k + 1 seeds, so the kept
    # residual can only fall as k grows; it is the least full residual
    p = workloads.uniform_planted(seed=4)
    A64, b64 = p.A.astype(np.float64), p.b.astype(np.float64)
    prev = np.inf
    for k in range(1, 6):
        rep = rand_nnls.rand_nnls_boost(p.A, p.b, 40, k, 500)
        got = float(np.linalg.norm(A64 @ rep.x - b64))
        per_run = [float(np.linalg.norm(A64 @ rand_nnls.rand_nnls(p.A, p.b, 40, 500 + i).x - b64))
                   for i in range(k)]
        assert got == min(per_run)
        assert got <= prev
        prev = got


def test_repetition_raises_the_success_probability():
    # Theorem 1's footnote: with the threshold at the median residual of single
    # runs, one run succeeds about half the time; keeping the best of 4
    # independent runs fails only if all 4 fail (probability about 1/16)
    p = workloads.uniform_planted(seed=5)
    A64, b64 = p.A.astype(np.float64), p.b.astype(np.float64)
    r = 40
    single = [float(np.linalg.norm(A64 @ rand_nnls.rand_nnls(p.A, p.b, r, 10_000 + s).x - b64))
              for s in range(60)]
    thr = float(np.median(single))
    trials, ok = 50, 0
    for t in range(trials):
        rep = rand_nnls.rand_nnls_boost(p.A, p.b, r, 4, 20_000 + 4 * t)
        ok += float(np.linalg.norm(A64 @ rep.x - b64)) <= thr
    # expected about 47; a binomial with p = 15/16 falls below 40 with probability < 1e-3
    assert ok >= 40
