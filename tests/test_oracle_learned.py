"""Pins of the learned-proposal oracle (features, perceptron, loss, gradient,
Adam) against facts that do not come from the oracle itself: the bfloat16
format's rounding rule and torch's independent conversion, central finite
differences, closed forms at special points, and invariances of the feature
definitions."""
import numpy as np
import pytest
import torch

from oracle import learned

RNG = np.random.default_rng(7)


# ------------------------------------------------------------------ bfloat16
def test_bf16_rounding_rule_examples():
    one = 1.0
    cases = {
        one: one,
        one + 2.0 ** -8: one,                        # midpoint, ties to even (down)
        one + 3 * 2.0 ** -8: one + 2.0 ** -6,        # midpoint, ties to even (up)
        one + 2.0 ** -8 + 2.0 ** -20: one + 2.0 ** -7,  # above the midpoint
        -(one + 2.0 ** -8 + 2.0 ** -20): -(one + 2.0 ** -7),
        0.0: 0.0,
        float(np.float32(3.4028235e38)): np.inf,     # rounds past the largest bf16
    }
    for a, want in cases.items():
        got = learned.bf16_round(np.array([a], np.float32))[0]
        assert got == np.float32(want), (a, got, want)
    assert np.isinf(learned.bf16_round(np.array([np.inf], np.float32))[0])
    assert np.isnan(learned.bf16_round(np.array([np.nan], np.float32))[0])


def test_bf16_rounding_matches_torch():
    a = (RNG.standard_normal(20000) * np.exp(RNG.uniform(-20, 20, 20000))).astype(np.float32)
    want = torch.from_numpy(a).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(learned.bf16_round(a), want)


# ------------------------------------------------------------------ network
def _params(scale=0.2):
    return RNG.standard_normal(learned.N_PARAMS) * scale


def _data(n=40):
    X = RNG.standard_normal((n, learned.F))
    y = (RNG.random(n) < 0.5).astype(np.float64)
    return X, y


def test_gradient_matches_central_differences():
    theta, (X, y) = _params(), _data()
    g = learned.gradient(theta, X, y, bf16=False)
    idx = RNG.choice(learned.N_PARAMS, size=80, replace=False)
    idx = np.concatenate([idx, [learned.N_PARAMS - 1, 0, 1024, 1152]])  # b3, W1, b1, W2
    h = 1e-6
    for i in idx:
        e = np.zeros_like(theta)
        e[i] = h
        fd = (learned.loss(theta + e, X, y, bf16=False) -
              learned.loss(theta - e, X, y, bf16=False)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, i


def test_bf16_gradient_is_the_gradient_at_the_rounded_weights():
    theta, (X, y) = _params(), _data()
    P = learned.unpack(theta)
    R = {k: (learned.bf16_round(P[k].astype(np.float32)).astype(np.float64)
             if k in learned.WEIGHTS else P[k]) for k in P}
    want = learned.gradient(learned.pack(R), X, y, bf16=False)
    got = learned.gradient(theta, X, y, bf16=True)
    assert np.allclose(got, want, rtol=1e-12, atol=1e-15)


def test_zero_network_closed_forms():
    theta = np.zeros(learned.N_PARAMS)
    X, y = _data(33)
    assert abs(learned.loss(theta, X, y) - np.log(2.0)) < 1e-15
    g = learned.gradient(theta, X, y)
    assert abs(g[-1] - np.mean(0.5 - y)) < 1e-15          # d/db3
    assert np.all(g[:-1] == 0.0)                           # relu(0) blocks the rest


def test_adam_first_step_is_lr_times_sign():
    theta = _params()
    grad = RNG.standard_normal(learned.N_PARAMS)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    new, m1, v1 = learned.adam_step(theta, grad, m, v, step=1, lr=1e-3)
    assert np.allclose(theta - new, 1e-3 * grad / (np.abs(grad) + 1e-8), rtol=1e-12)
    assert np.allclose(m1, 0.1 * grad) and np.allclose(v1, 0.001 * grad * grad)


# ------------------------------------------------------------------ features
def _gram(A, b):
    return A.T @ A, A.T @ b, float(b @ b)


def test_feature_invariances():
    A = np.abs(RNG.standard_normal((200, 9)))
    b = A @ RNG.uniform(0, 2, 9) + 0.1 * RNG.standard_normal(200)
    X = learned.features(*_gram(A, b))
    # positive scaling of b or of A changes nothing
    assert np.allclose(learned.features(*_gram(A, 3.5 * b)), X, atol=1e-12)
    assert np.allclose(learned.features(*_gram(0.25 * A, b)), X, atol=1e-12)
    # permuting columns permutes the rows
    perm = RNG.permutation(9)
    assert np.allclose(learned.features(*_gram(A[:, perm], b)), X[perm], atol=1e-12)
    # f2 is a z-score over the columns
    assert abs(X[:, 2].mean()) < 1e-12 and abs(X[:, 2].std() - 1.0) < 1e-12
    assert np.all(X[:, 7] == 9 / 128)


def test_feature_special_cases():
    n = 64
    Q, _ = np.linalg.qr(RNG.standard_normal((n, 4)))
    b = Q[:, 0] * 2.0
    X = learned.features(*_gram(Q, b))
    assert abs(X[0, 0] - 1.0) < 1e-12            # column parallel to b: cosine 1
    assert np.allclose(X[1:, 0], 0.0, atol=1e-12)  # orthogonal columns: cosine 0
    assert np.allclose(X[:, 3:6], 0.0, atol=1e-12)  # orthonormal columns: C = 0
    assert np.allclose(X[:, 6], 0.0, atol=1e-12)    # equal norms
    # a zero column
    A = np.column_stack([Q[:, :2], np.zeros(n)])
    X = learned.features(*_gram(A, b))
    assert X[2, 0] == 0.0 and X[2, 6] == -30.0 and X[2, 3] == 0.0
    # one column: no neighbours
    X = learned.features(*_gram(Q[:, :1], b))
    assert X[0, 3] == X[0, 4] == X[0, 5] == 0.0


def test_feature_values_on_a_hand_built_gram():
    """Every feature of a 3-column (G, q, c) worked out by hand from the
    definitions: C_01 = 2/(2*1) = 1, C_02 = 0, C_12 = 0.5/(1*4) = 1/8;
    f0 = q_j / sqrt(G_jj c) = (2/12, -6/6, 3/24); max|q| = 6 (not max q = 3);
    mean q = -1/3 and std q = sqrt(146)/3, so f2 = (7, -17, 10)/sqrt(146);
    f5_j averages C_jk f0_k over k != j; mean diag G = 7."""
    G = np.array([[4.0, 2.0, 0.0], [2.0, 1.0, 0.5], [0.0, 0.5, 16.0]])
    q = np.array([2.0, -6.0, 3.0])
    c = 36.0
    f0 = np.array([1 / 6, -1.0, 1 / 8])
    want = np.zeros((3, 8))
    want[:, 0] = f0
    want[:, 1] = [1 / 3, -1.0, 1 / 2]
    want[:, 2] = np.array([7.0, -17.0, 10.0]) / np.sqrt(146.0)
    want[:, 3] = [1 / 2, 9 / 16, 1 / 16]
    want[:, 4] = [1.0, 1.0, 1 / 8]
    want[:, 5] = [(1.0 * f0[1] + 0.0 * f0[2]) / 2,      # -1/2
                  (1.0 * f0[0] + 0.125 * f0[2]) / 2,    # 35/384
                  (0.0 * f0[0] + 0.125 * f0[1]) / 2]    # -1/16
    want[:, 6] = np.log(np.array([4.0, 1.0, 16.0]) / 7.0)
    want[:, 7] = 3 / 128
    assert abs(want[1, 5] - 35 / 384) < 1e-15
    got = learned.features(G, q, c)
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-15)
