"""Pins for the oracle's Hadamard transform and sketch (Section 2, Algorithm 1)."""
import numpy as np
import pytest
import scipy.linalg

from oracle import hadamard, rng


@pytest.mark.parametrize("n", [1, 2, 4, 8, 64, 1024])
def test_sylvester_matrix_matches_scipy(n):
    # scipy.linalg.hadamard builds the same Sylvester construction
    assert np.array_equal(hadamard.hadamard_matrix(n), scipy.linalg.hadamard(n))


def test_closed_form_entries():
    n = 256
    H = scipy.linalg.hadamard(n)
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    assert np.array_equal(hadamard.hadamard_entry(i, j), H)


@pytest.mark.parametrize("n", [2, 16, 512, 2048])
def test_fwht_equals_explicit_product(n):
    g = np.random.default_rng(n)
    X = g.standard_normal((n, 3))
    H = scipy.linalg.hadamard(n).astype(np.float64)
    np.testing.assert_allclose(hadamard.fwht(X), H @ X, rtol=0, atol=1e-10 * np.sqrt(n))


def test_fwht_on_fortran_input():
    g = np.random.default_rng(3)
    X = np.asfortranarray(g.standard_normal((128, 4)))
    H = scipy.linalg.hadamard(128).astype(np.float64)
    np.testing.assert_allclose(hadamard.fwht(X), H @ X, atol=1e-11)


def test_orthogonality_involution_and_norm():
    n = 1 << 12
    H = scipy.linalg.hadamard(1024).astype(np.float64)
    assert np.array_equal(H.T @ H, 1024 * np.eye(1024))
    g = np.random.default_rng(1)
    x = g.standard_normal(n)
    np.testing.assert_allclose(hadamard.fwht(hadamard.fwht(x)), n * x, rtol=1e-12, atol=1e-9)
    # normalised H_n preserves the 2-norm (H_n D is orthogonal)
    D = rng.signs(5, n).astype(np.float64)
    y = hadamard.fwht(D * x) / np.sqrt(n)
    assert abs(np.linalg.norm(y) - np.linalg.norm(x)) < 1e-11 * np.linalg.norm(x)


def test_basis_vectors_and_constant():
    n = 64
    for j in (0, 1, 5, 63):
        e = np.zeros(n)
        e[j] = 1
        np.testing.assert_array_equal(hadamard.fwht(e), scipy.linalg.hadamard(n)[:, j])
    np.testing.assert_array_equal(hadamard.fwht(np.ones(n)), n * np.eye(n)[0])


@pytest.mark.parametrize("mode", ["exact", "bernoulli"])
def test_sketch_equals_explicit_SHD_product(mode):
    # the sketch written as an explicit FP64 matrix product S * H_n * D * [A b]
    n, d, r, seed = 1000, 5, 37, 21
    g = np.random.default_rng(4)
    A = g.random((n, d)).astype(np.float32)
    b = g.random(n).astype(np.float32)
    SA, Sb, R, D = hadamard.srht_sketch(A, b, r, seed, mode)
    n_pad = 1024
    Hn = scipy.linalg.hadamard(n_pad).astype(np.float64) / np.sqrt(n_pad)
    S = np.zeros((R.size, n_pad))
    S[np.arange(R.size), R] = np.sqrt(n_pad / r)
    M = np.zeros((n_pad, d + 1))
    M[:n, :d] = A
    M[:n, d] = b
    ref = S @ Hn @ np.diag(D) @ M
    np.testing.assert_allclose(SA, ref[:, :d], atol=1e-12)
    np.testing.assert_allclose(Sb, ref[:, d], atol=1e-12)
    assert np.array_equal(R, rng.rows(seed, n_pad, r, mode))
    assert np.array_equal(D, rng.signs(seed, n_pad))


def test_padding_equals_explicit_zero_rows():
    n, d, r = 777, 3, 50
    g = np.random.default_rng(8)
    A = g.random((n, d))
    b = g.random(n)
    SA, Sb, _, _ = hadamard.srht_sketch(A, b, r, 3)
    Ap = np.vstack([A, np.zeros((1024 - n, d))])
    bp = np.concatenate([b, np.zeros(1024 - n)])
    SA2, Sb2, _, _ = hadamard.srht_sketch(Ap, bp, r, 3)
    np.testing.assert_array_equal(SA, SA2)
    np.testing.assert_array_equal(Sb, Sb2)


def test_direct_row_matches_fast_transform():
    n, r, seed = 5000, 64, 9
    g = np.random.default_rng(2)
    M = g.standard_normal((n, 4))
    SA, _, R, D = hadamard.srht_sketch(M, None, r, seed)
    for k in (0, 7, 63):
        np.testing.assert_allclose(hadamard.sketch_row_direct(M, D, int(R[k]), r), SA[k],
                                   atol=1e-11)


def test_sketch_is_unbiased_in_norm():
    # E[S^T S] = I: the sketched squared norm of a fixed vector averages to
    # its squared norm over the random draws
    n, r = 512, 64
    g = np.random.default_rng(6)
    x = g.standard_normal((n, 1))
    vals = [np.sum(hadamard.srht_sketch(x, None, r, s)[0] ** 2) for s in range(400)]
    mean = np.mean(vals)
    sem = np.std(vals) / np.sqrt(len(vals))
    assert abs(mean - np.sum(x**2)) < 5 * sem
