"""Pins for the oracle's Lawson-Hanson solver (Definition 1)."""
import numpy as np
import pytest
import scipy.optimize

from oracle import nnls


def _problem(m, d, seed, planted_zeros=None, noise=0.1):
    g = np.random.default_rng(seed)
    A = g.standard_normal((m, d))
    x = g.standard_normal(d)
    if planted_zeros is not None:
        x = np.abs(x)
        x[g.choice(d, planted_zeros, replace=False)] = 0
    b = A @ x + noise * g.standard_normal(m)
    return A, b


@pytest.mark.parametrize("seed", range(12))
def test_matches_brute_force(seed):
    d = 3 + seed % 7
    A, b = _problem(40, d, seed)
    res = nnls.lawson_hanson(A, b)
    xb, rb = nnls.brute_force(A, b)
    assert abs(res.rnorm - rb) <= 1e-10 * max(rb, 1.0)
    np.testing.assert_allclose(res.x, xb, atol=1e-9)
    assert res.status == nnls.STATUS_OK


@pytest.mark.parametrize("seed", range(8))
def test_kkt_certificate(seed):
    A, b = _problem(200, 30, 100 + seed)
    res = nnls.lawson_hanson(A, b)
    assert res.status == nnls.STATUS_OK
    assert np.all(res.x >= 0)
    tau = nnls.default_tol(A)
    v = nnls.kkt_violation(A, b, res.x)
    assert v["dual_off"] <= tau
    assert v["dual_on"] <= 1e3 * tau


@pytest.mark.parametrize("seed", range(6))
def test_matches_scipy_nnls(seed):
    A, b = _problem(300, 25, 200 + seed)
    res = nnls.lawson_hanson(A, b)
    xs, rs = scipy.optimize.nnls(A, b)
    assert abs(res.rnorm - rs) <= 1e-9 * rs
    np.testing.assert_allclose(res.x, xs, atol=1e-8)


def test_equals_least_squares_when_ls_is_positive():
    g = np.random.default_rng(0)
    A = g.random((100, 8))
    x = 1.0 + g.random(8)
    b = A @ x + 1e-3 * g.standard_normal(100)
    ls = nnls.unconstrained_ls(A, b)
    assert np.all(ls > 0)
    res = nnls.lawson_hanson(A, b)
    np.testing.assert_allclose(res.x, ls, rtol=1e-10)
    np.testing.assert_allclose(ls, np.linalg.lstsq(A, b, rcond=None)[0], rtol=1e-10)


def test_single_column_closed_form():
    g = np.random.default_rng(1)
    a = g.standard_normal((50, 1))
    for b in (g.standard_normal(50), -a[:, 0] + 0.1 * g.standard_normal(50)):
        res = nnls.lawson_hanson(a, b)
        want = max(0.0, float(a[:, 0] @ b) / float(a[:, 0] @ a[:, 0]))
        assert abs(res.x[0] - want) <= 1e-12 * max(1.0, want)


def test_zero_rhs_gives_zero():
    A, _ = _problem(30, 6, 3)
    res = nnls.lawson_hanson(A, np.zeros(30))
    assert np.all(res.x == 0) and res.iters == 0


def test_all_negative_correlations_give_zero():
    g = np.random.default_rng(2)
    A = g.random((30, 5))
    b = -A @ g.random(5)
    res = nnls.lawson_hanson(A, b)
    assert np.all(res.x == 0)


def test_iteration_cap_reports_status():
    A, b = _problem(100, 20, 5, planted_zeros=5, noise=0.0)
    res = nnls.lawson_hanson(A, b, max_iter=1)
    assert res.status == nnls.STATUS_MAX_ITER
    assert res.iters == 1


def test_duplicate_column_is_refused_not_crashed():
    g = np.random.default_rng(9)
    A = g.random((60, 4))
    A = np.column_stack([A, A[:, 1]])
    b = A[:, :4] @ np.array([1.0, 2.0, 0.0, 0.5]) + 0.01 * g.standard_normal(60)
    res = nnls.lawson_hanson(A, b)
    ref, rb = nnls.brute_force(A, b)
    assert abs(res.rnorm - rb) <= 1e-9 * rb


@pytest.mark.parametrize("seed", range(5))
def test_warm_start_reaches_the_same_optimum(seed):
    A, b = _problem(120, 16, 300 + seed, planted_zeros=6)
    cold = nnls.lawson_hanson(A, b)
    for P0 in (cold.x > 0, np.ones(16, bool), ~(cold.x > 0), np.zeros(16, bool)):
        warm = nnls.lawson_hanson(A, b, passive0=P0)
        assert abs(warm.rnorm - cold.rnorm) <= 1e-10 * cold.rnorm
    exact = nnls.lawson_hanson(A, b, passive0=cold.x > 0)
    assert exact.iters == 0


def test_relative_gap_definition():
    A = np.eye(3)
    b = np.array([1.0, 0.0, 0.0])
    assert nnls.relative_residual_gap(A, b, np.array([0.5, 0, 0]), np.array([0.0, 0, 0])) == \
        pytest.approx(-0.5)
