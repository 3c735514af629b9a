"""Pins for the oracle's random streams (D and S of Algorithm 1)."""
import json
import os

import numpy as np
import pytest
from scipy import stats

from oracle import rng

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_mix64_matches_published_splitmix64_outputs():
    with open(os.path.join(GOLDEN, "splitmix64.json")) as f:
        ref = json.load(f)
    for case in ref["cases"]:
        if "outputs_hex" in case:
            want = [int(v, 16) for v in case["outputs_hex"]]
        else:
            want = [int(v) for v in case["outputs_dec"]]
        assert rng.splitmix64_sequence(case["seed"], len(want)) == want


def test_vector_hash_equals_scalar_hash():
    g = np.random.default_rng(0)
    seeds = [0, 1, 2**63 + 5, 0xFFFFFFFFFFFFFFFF]
    idx = g.integers(0, 2**62, size=64, dtype=np.int64).astype(np.uint64)
    for seed in seeds:
        for stream in (rng.STREAM_SIGN, rng.STREAM_SAMPLE, rng.STREAM_PERM):
            vec = rng.h_array(seed, stream, idx)
            for i, v in zip(idx, vec):
                assert int(v) == rng.h(seed, stream, int(i))


@pytest.mark.parametrize("m", list(range(1, 15)))
def test_perm_is_a_bijection(m):
    for seed in (0, 1, 99):
        img = [rng.perm(seed, m, k) for k in range(1 << m)]
        assert sorted(img) == list(range(1 << m))


def test_rows_exact_distinct_sorted_in_range():
    for seed, n_pad, r in [(1, 4096, 512), (5, 2, 1), (9, 1 << 18, 3000), (4, 64, 63)]:
        R = rng.rows_exact(seed, n_pad, r)
        assert R.size == r
        assert np.all(np.diff(R) > 0)
        assert R[0] >= 0 and R[-1] < n_pad


def test_rows_exact_inclusion_is_uniform():
    # every row must be kept with probability r/n' (the marginal of step 2 of
    # Algorithm 1); chi-square over the per-row inclusion counts
    n_pad, r, seeds = 256, 32, 800
    counts = np.zeros(n_pad)
    for s in range(seeds):
        counts[rng.rows_exact(s, n_pad, r)] += 1
    expected = seeds * r / n_pad
    chi2 = float(np.sum((counts - expected) ** 2 / expected))
    # variance of a hypergeometric-like count is below the binomial one, so the
    # binomial chi-square is conservative
    assert stats.chi2.sf(chi2, n_pad - 1) > 1e-4


def test_rows_exact_pairs_are_not_structured():
    # pairwise co-inclusion: no pair of rows may be kept together far more or
    # less often than (r/n')^2 -- catches affine (XOR-subgroup) structure
    n_pad, r, seeds = 64, 8, 3000
    co = np.zeros((n_pad, n_pad))
    for s in range(seeds):
        R = rng.rows_exact(s, n_pad, r)
        co[np.ix_(R, R)] += 1
    off = co[~np.eye(n_pad, dtype=bool)]
    p = r * (r - 1) / (n_pad * (n_pad - 1))
    mean = seeds * p
    assert abs(off.mean() - mean) < 0.05 * mean
    assert off.max() < mean + 7 * np.sqrt(mean)
    assert off.min() > max(0.0, mean - 7 * np.sqrt(mean))


def test_signs_balanced():
    s = rng.signs(11, 1 << 16)
    assert set(np.unique(s)) == {-1, 1}
    k = int((s > 0).sum())
    assert stats.binomtest(k, s.size, 0.5).pvalue > 1e-4


def test_bernoulli_count_and_frequency():
    n_pad, r = 1 << 14, 700
    counts = [rng.rows_bernoulli(s, n_pad, r).size for s in range(60)]
    # r~ ~ Bin(n', r/n'): mean r, sd ~ sqrt(r)
    assert abs(np.mean(counts) - r) < 5 * np.sqrt(r / 60.0)
    R = rng.rows_bernoulli(3, n_pad, r)
    assert np.all(np.diff(R) > 0)


def test_bernoulli_threshold_is_exact_probability():
    # threshold r * 2^(64-m) over uniform 64-bit hashes is exactly r/n'
    n_pad, r = 1 << 12, 3
    m = 12
    assert (r << (64 - m)) / 2.0**64 == r / n_pad


def test_golden_streams_reproduce():
    with open(os.path.join(GOLDEN, "streams.json")) as f:
        gold = json.load(f)
    for c in gold["cases"]:
        assert list(rng.rows_exact(c["seed"], c["n_pad"], c["r"])) == c["rows_exact"]
        rb = rng.rows_bernoulli(c["seed"], c["n_pad"], c["r"])
        assert rb.size == c["rows_bernoulli_count"]
        assert list(rb[:512]) == c["rows_bernoulli_head"]
        s = rng.signs(c["seed"], c["n_pad"])
        assert int((s < 0).sum()) == c["neg_sign_count"]
        assert list(np.nonzero(s < 0)[0][:256]) == c["neg_sign_rows_head"]
