"""Pins for the alternating-NNLS factorisation oracle: what the mathematics
fixes (monotone objective, exact recovery of a planted factorisation)."""
import numpy as np

from oracle import nmf


def _planted(m, n, q, seed):
    g = np.random.default_rng(seed)
    W = g.random((m, q)) * (g.random((m, q)) < 0.6)
    H = g.random((q, n)) * (g.random((q, n)) < 0.6)
    W[:q, :q] += np.eye(q)            # full column rank
    H[:, :q] += np.eye(q)
    return W, H


def test_anls_objective_never_increases():
    g = np.random.default_rng(3)
    A = g.random((120, 40)) * (g.random((120, 40)) < 0.3)
    W0 = g.random((120, 5))
    _, _, hist = nmf.anls(A, W0, 4)
    for a, b in zip(hist, hist[1:]):
        assert b <= a * (1 + 1e-9) + 1e-12
    assert hist[-1] < hist[0]


def test_anls_recovers_a_planted_factorisation_in_one_half_step():
    W, H = _planted(90, 30, 4, seed=5)
    A = W @ H
    _, H1, hist = nmf.anls(A, W, 1)
    assert hist[0] <= 1e-10 * np.linalg.norm(A)
    np.testing.assert_allclose(H1, H, atol=1e-10)
