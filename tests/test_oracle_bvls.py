"""Pins of the box-constrained oracle (least squares with lo <= x <= hi on the
sketch, the conclusions' remark on other constraint sets): brute force over
every bound/free assignment, scipy's independent solvers, and the special cases
that reduce to Definition 1 or to unconstrained least squares."""
import numpy as np
import pytest
from scipy.optimize import lsq_linear, nnls as scipy_nnls

from oracle import bvls
from oracle.nnls import default_tol


def _problem(m, d, seed, cond=1.0):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, d))
    if cond != 1.0:
        U, _, Vt = np.linalg.svd(A, full_matrices=False)
        A = U @ np.diag(np.geomspace(1.0, 1.0 / cond, d)) @ Vt
    b = rng.standard_normal(m) * 2.0
    return A, b


def _box(d, seed, inf_frac=0.3):
    rng = np.random.default_rng(seed + 1000)
    lo = rng.uniform(-1.0, 0.2, d)
    hi = lo + rng.uniform(0.1, 1.5, d)
    hi[rng.random(d) < inf_frac] = np.inf
    return lo, hi


@pytest.mark.parametrize("seed", range(12))
def test_bvls_matches_brute_force(seed):
    d = 2 + seed % 4
    A, b = _problem(12 + seed, d, seed)
    lo, hi = _box(d, seed)
    res = bvls.bvls(A, b, lo, hi)
    xb, fb = bvls.brute_force(A, b, lo, hi)
    assert res.status == 0
    f = float(np.sum((A @ res.x - b) ** 2))
    assert f <= fb * (1 + 1e-10) + 1e-12
    np.testing.assert_allclose(res.x, xb, atol=1e-8)


@pytest.mark.parametrize("seed", range(8))
def test_bvls_matches_scipy_bounded_solvers(seed):
    m, d = 200, 24
    A, b = _problem(m, d, 100 + seed, cond=30.0)
    lo, hi = _box(d, 100 + seed, inf_frac=0.0)
    res = bvls.bvls(A, b, lo, hi)
    ref = lsq_linear(A, b, bounds=(lo, hi), method="bvls", tol=1e-14)
    f = float(np.sum((A @ res.x - b) ** 2))
    f_ref = float(np.sum((A @ ref.x - b) ** 2))
    assert f <= f_ref * (1 + 1e-10)
    np.testing.assert_allclose(res.x, ref.x, atol=1e-7)
    assert bvls.kkt_box(A, b, res.x, lo, hi, default_tol(A)) <= 10.0


@pytest.mark.parametrize("seed", range(6))
def test_bvls_nonnegative_orthant_is_nnls(seed):
    A, b = _problem(120, 30, 200 + seed)
    res = bvls.bvls(A, b, np.zeros(30), np.full(30, np.inf))
    x_ref, rn = scipy_nnls(A, b)
    np.testing.assert_allclose(res.x, x_ref, atol=1e-9)
    assert abs(res.rnorm - rn) <= 1e-10 * max(rn, 1.0)


def test_bvls_shifted_lower_bound_is_nnls_of_shifted_rhs():
    A, b = _problem(90, 16, 7)
    c = np.linspace(-0.5, 0.5, 16)
    res = bvls.bvls(A, b, c, np.full(16, np.inf))
    y, _ = scipy_nnls(A, b - A @ c)
    np.testing.assert_allclose(res.x, c + y, atol=1e-9)


def test_bvls_wide_box_is_unconstrained_least_squares():
    A, b = _problem(80, 10, 3)
    x_ls = np.linalg.lstsq(A, b, rcond=None)[0]
    res = bvls.bvls(A, b, x_ls - 5.0, x_ls + 5.0)
    # every variable must leave its lower bound and end strictly inside
    assert np.all(res.state == bvls.FREE)
    np.testing.assert_allclose(res.x, x_ls, atol=1e-10)


def test_bvls_fixed_variables_stay_fixed():
    A, b = _problem(60, 8, 11)
    lo = np.full(8, -1.0)
    hi = np.full(8, 1.0)
    lo[[1, 4]] = hi[[1, 4]] = 0.25
    res = bvls.bvls(A, b, lo, hi)
    assert res.x[1] == 0.25 and res.x[4] == 0.25
    xb, fb = bvls.brute_force(A, b, lo, hi)
    np.testing.assert_allclose(res.x, xb, atol=1e-8)


def test_bvls_upper_bounds_become_active():
    """A right-hand side pulling every coefficient above its upper bound ends
    with the whole solution on the upper face."""
    rng = np.random.default_rng(5)
    A = np.abs(rng.standard_normal((50, 6))) + 0.1
    b = A @ np.full(6, 3.0)
    res = bvls.bvls(A, b, np.zeros(6), np.ones(6))
    np.testing.assert_allclose(res.x, np.ones(6))
    assert np.all(res.state == bvls.AT_HIGH)


def test_bvls_rejects_bad_bounds():
    A, b = _problem(10, 3, 1)
    with pytest.raises(ValueError):
        bvls.bvls(A, b, np.array([0.0, -np.inf, 0.0]), np.ones(3))
    with pytest.raises(ValueError):
        bvls.bvls(A, b, np.array([0.0, 2.0, 0.0]), np.ones(3))


def test_rand_box_on_the_orthant_is_rand_nnls():
    """With lo = 0, hi = +inf the box form of Algorithm 1 is Algorithm 1."""
    from oracle import rand_nnls as orand
    rng = np.random.default_rng(4)
    A = np.abs(rng.standard_normal((3000, 12)))
    b = A @ rng.uniform(-0.5, 1.5, 12) + 0.1 * rng.standard_normal(3000)
    one = orand.rand_nnls(A, b, 300, 9)
    box = orand.rand_box(A, b, 300, 9, np.zeros(12), np.full(12, np.inf))
    np.testing.assert_array_equal(box.rows, one.rows)
    np.testing.assert_allclose(box.x, one.x, atol=1e-9)
