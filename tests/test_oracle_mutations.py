"""The oracle's pins must bite: plant plausible mistakes in the oracle (on the
CPU, via monkeypatch) and check that the pin meant to catch each one fails."""
import json
import os

import numpy as np
import scipy.linalg

from oracle import hadamard, nnls, rng

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _sketch_matches_explicit_product():
    n, d, r, seed = 1000, 4, 37, 21
    g = np.random.default_rng(4)
    A = g.random((n, d))
    b = g.random(n)
    SA, Sb, R, D = hadamard.srht_sketch(A, b, r, seed)
    Hn = scipy.linalg.hadamard(1024) / np.sqrt(1024)
    M = np.zeros((1024, d + 1))
    M[:n, :d] = A
    M[:n, d] = b
    ref = np.sqrt(1024 / r) * (Hn @ (rng.signs(seed, 1024)[:, None] * M))[rng.rows_exact(seed, 1024, r)]
    return np.allclose(SA, ref[:, :d], atol=1e-12) and np.allclose(Sb, ref[:, d], atol=1e-12)


def _lh_matches_brute_force():
    g = np.random.default_rng(7)
    for _ in range(6):
        A = g.standard_normal((30, 6))
        b = A @ g.standard_normal(6) + 0.1 * g.standard_normal(30)
        res = nnls.lawson_hanson(A, b)
        _, rb = nnls.brute_force(A, b)
        if abs(res.rnorm - rb) > 1e-9 * rb or np.any(res.x < 0):
            return False
    return True


def _streams_match_golden():
    with open(os.path.join(GOLDEN, "streams.json")) as f:
        c = json.load(f)["cases"][0]
    return (list(rng.rows_exact(c["seed"], c["n_pad"], c["r"])) == c["rows_exact"]
            and int((rng.signs(c["seed"], c["n_pad"]) < 0).sum()) == c["neg_sign_count"])


def test_pins_pass_on_the_real_oracle():
    assert _sketch_matches_explicit_product()
    assert _lh_matches_brute_force()
    assert _streams_match_golden()


def test_wrong_butterfly_sign_is_caught(monkeypatch):
    real = hadamard.fwht

    def bad(X):
        Y = real(X)
        return np.concatenate([Y[: Y.shape[0] // 2], -Y[Y.shape[0] // 2:]])
    monkeypatch.setattr(hadamard, "fwht", bad)
    assert not _sketch_matches_explicit_product()


def test_wrong_scale_is_caught(monkeypatch):
    real = hadamard.srht_sketch

    def bad(A, b, r, seed, mode="exact"):
        SA, Sb, R, D = real(A, b, r, seed, mode)
        return SA * np.sqrt(r / 1024.0), Sb, R, D
    monkeypatch.setattr(hadamard, "srht_sketch", bad)
    assert not _sketch_matches_explicit_product()


def test_missing_sign_flip_is_caught(monkeypatch):
    monkeypatch.setattr(rng, "signs", lambda seed, n: np.ones(n, dtype=np.int8))
    assert not _streams_match_golden()


def test_off_by_one_rows_are_caught(monkeypatch):
    real = rng.rows_exact
    monkeypatch.setattr(rng, "rows_exact", lambda s, n, r: real(s, n, r) + 1)
    assert not _streams_match_golden()


def test_transposed_pass_order_is_caught(monkeypatch):
    # a transform applied along the wrong axis (columns instead of rows)
    real = hadamard.fwht
    monkeypatch.setattr(hadamard, "fwht",
                        lambda X: real(np.asarray(X).T).T if np.asarray(X).ndim == 2
                        and (np.asarray(X).shape[1] & (np.asarray(X).shape[1] - 1)) == 0
                        else real(X)[::-1])
    assert not _sketch_matches_explicit_product()


def test_wrong_dual_sign_is_caught(monkeypatch):
    real_qr = np.linalg.qr

    # flip the sign of the least-squares right-hand side: z solves A z = -b
    def bad_ls(A, b, P):
        Q, R = real_qr(A[:, P], mode="reduced")
        return scipy.linalg.solve_triangular(R, -(Q.T @ b)), np.diag(R)
    monkeypatch.setattr(nnls, "_ls_on", bad_ls)
    assert not _lh_matches_brute_force()


def test_dropped_interpolation_step_is_caught(monkeypatch):
    # a solver that clips negative least-squares coefficients instead of the
    # feasible interpolation of the inner loop
    def bad_lh(A, b, tol=None, max_iter=None, passive0=None):
        x = np.clip(np.linalg.lstsq(A, b, rcond=None)[0], 0, None)
        return nnls.NNLSResult(x=x, w=A.T @ (b - A @ x), rnorm=float(np.linalg.norm(A @ x - b)),
                               iters=1, status=0, passive=np.nonzero(x)[0])
    monkeypatch.setattr(nnls, "lawson_hanson", bad_lh)
    assert not _lh_matches_brute_force()


def _bvls_matches_brute_force():
    from oracle import bvls
    g = np.random.default_rng(12)
    for _ in range(6):
        A = g.standard_normal((20, 4))
        b = 2.0 * g.standard_normal(20)
        lo = g.uniform(-1.0, 0.2, 4)
        hi = lo + g.uniform(0.1, 1.0, 4)
        res = bvls.bvls(A, b, lo, hi)
        _, fb = bvls.brute_force(A, b, lo, hi)
        f = float(np.sum((A @ res.x - b) ** 2))
        if f > fb * (1 + 1e-9) + 1e-12:
            return False
    return True


def test_box_pin_passes_on_the_real_oracle():
    assert _bvls_matches_brute_force()


def test_free_solve_without_bound_terms_is_caught(monkeypatch):
    """The free least-squares problem forgets that the bound variables sit at
    nonzero values (right-hand side b instead of b - A_B x_B)."""
    from oracle import bvls

    def plain_free(A, b, x, F):
        return np.linalg.lstsq(A[:, F], b, rcond=None)[0]

    def free_solve(A, b, x, F):
        return plain_free(A, b, x, F), True

    monkeypatch.setattr(bvls, "_plain_free", plain_free)
    monkeypatch.setattr(bvls, "_free_solve", free_solve)
    assert not _bvls_matches_brute_force()


def _features_pin(feat):
    """The hand-built 3-column pin of the learned features (values worked out
    from the definitions; see test_oracle_learned)."""
    G = np.array([[4.0, 2.0, 0.0], [2.0, 1.0, 0.5], [0.0, 0.5, 16.0]])
    q = np.array([2.0, -6.0, 3.0])
    X = feat(G, q, 36.0)
    f0 = np.array([1 / 6, -1.0, 1 / 8])
    return (np.allclose(X[:, 1], [1 / 3, -1.0, 1 / 2], atol=1e-13)
            and np.allclose(X[:, 5], [-1 / 2, 35 / 384, -1 / 16], atol=1e-13)
            and np.allclose(X[:, 6], np.log(np.array([4.0, 1.0, 16.0]) / 7.0), atol=1e-13)
            and np.allclose(X[:, 0], f0, atol=1e-13))


def test_feature_mistakes_are_caught():
    from oracle import learned
    assert _features_pin(learned.features)

    def mutated(change):
        def feat(G, q, c):
            X = learned.features(G, q, c)
            change(X, G, q, c)
            return X
        return feat

    def f1_by_max_q(X, G, q, c):          # max q instead of max |q|
        X[:, 1] = q / np.max(q)

    def f5_own_cosine(X, G, q, c):        # f0_j instead of f0_k
        d = len(q)
        for j in range(d):
            C = [G[j, k] / np.sqrt(G[j, j] * G[k, k]) for k in range(d) if k != j]
            X[j, 5] = np.mean(C) * X[j, 0]

    def f6_by_max_norm(X, G, q, c):       # normalised by the largest diagonal
        X[:, 6] = np.log(np.diag(G) / np.max(np.diag(G)))

    for change in (f1_by_max_q, f5_own_cosine, f6_by_max_norm):
        assert not _features_pin(mutated(change)), change.__name__
