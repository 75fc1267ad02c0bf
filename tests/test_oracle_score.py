"""Pins for the oracle's SVM scoring and one-vs-rest trainer.

Scores: exact rational dot products bound the double-precision result; ties in
the argmax go to the lowest identity. Trainer: a two-point problem with a
closed-form maximum-margin solution, and agreement with an independent
library solver (liblinear's dual coordinate descent through scikit-learn) on
the same objective.
"""
from fractions import Fraction

import numpy as np
import pytest


def test_score_exact_rational(ref):
    rng = np.random.default_rng(11)
    N, K, D = 5, 4, 19
    X = rng.standard_normal((N, D)).astype(np.float32)
    W = rng.standard_normal((K, D)).astype(np.float32)
    b = rng.standard_normal(K).astype(np.float32)
    S, am = ref.score_f64(X, W, b)
    for n in range(N):
        for k in range(K):
            exact = sum(Fraction(float(W[k, j])) * Fraction(float(X[n, j])) for j in range(D))
            exact += Fraction(float(b[k]))
            scale = sum(abs(float(W[k, j]) * float(X[n, j])) for j in range(D)) + abs(float(b[k]))
            assert abs(Fraction(S[n, k]) - exact) <= Fraction((D + 2) * 2.0 ** -53 * scale)
    assert np.array_equal(am, np.argmax(S, axis=1))


def test_score_argmax_ties_lowest_index(ref):
    X = np.ones((3, 4), np.float32)
    W = np.array([[1, 0, 0, 0], [0.5, 0.5, 0, 0], [0, 0, 0, 1], [-1, 0, 0, 0]], np.float32)
    b = np.zeros(4, np.float32)
    S, am = ref.score_f64(X, W, b)
    assert np.all(S[:, :3] == 1.0)
    assert list(am) == [0, 0, 0]


def test_score_identity_rows(ref):
    """With W = I and b = 0 the scores are the features themselves."""
    rng = np.random.default_rng(12)
    X = rng.random((6, 9)).astype(np.float32)
    S, am = ref.score_f64(X, np.eye(9, dtype=np.float32), np.zeros(9, np.float32))
    assert np.array_equal(S, X.astype(np.float64))
    assert np.array_equal(am, np.argmax(X, axis=1))


def test_train_two_points_closed_form(ref):
    """Two points, one per class, large C: the solution is the minimum-norm
    augmented w~ = (w, b) with w~.x~1 = +1 and w~.x~2 = -1 on the scaled
    points (x~ = (sigma x, 1)), i.e. w~ = A^T (A A^T)^-1 (1, -1)."""
    X = np.array([[3.0, 1.0, 0.0], [1.0, 2.0, 2.0]], np.float32)
    y = np.array([0, 1], np.int32)
    W, b, ep = ref.train_ovr_f64(X, y, K=2, C=1e6, eps=1e-12, max_epochs=100000)
    norms = np.linalg.norm(X.astype(np.float64), axis=1)
    sigma = 1.0 / np.sort(norms)[0]
    A = np.hstack([sigma * X.astype(np.float64), np.ones((2, 1))])
    for k, target in ((0, np.array([1.0, -1.0])), (1, np.array([-1.0, 1.0]))):
        wt = A.T @ np.linalg.solve(A @ A.T, target)
        np.testing.assert_allclose(W[k], sigma * wt[:3], rtol=1e-8, atol=1e-10)
        np.testing.assert_allclose(b[k], wt[3], rtol=1e-8, atol=1e-10)
        s = X.astype(np.float64) @ W[k] + b[k]
        np.testing.assert_allclose(s, target, rtol=1e-8)


def test_train_matches_liblinear(ref):
    """Same objective (L2-regularised hinge loss, bias as a regularised constant
    feature, C = 1) solved by scikit-learn's LinearSVC (liblinear). The primal
    is strictly convex, so the oracle's objective may not exceed liblinear's and
    the hyperplanes must agree where liblinear converged (seeded order)."""
    sk = pytest.importorskip("sklearn.svm")
    rng = np.random.default_rng(13)
    K, per, D = 3, 20, 12
    centres = rng.standard_normal((K, D)) * 1.5
    X = np.vstack([centres[k] + rng.standard_normal((per, D)) for k in range(K)]).astype(np.float32)
    y = np.repeat(np.arange(K), per).astype(np.int32)
    W, b, ep = ref.train_ovr_f64(X, y, K=K, C=1.0, eps=1e-10, max_epochs=200000)
    sigma = 1.0 / np.sort(np.linalg.norm(X.astype(np.float64), axis=1))[(len(X) - 1) // 2]
    Xs = sigma * X.astype(np.float64)

    def primal(w, bias, k):
        yy = np.where(y == k, 1.0, -1.0)
        return 0.5 * (w @ w + bias * bias) + np.maximum(0.0, 1.0 - yy * (Xs @ w + bias)).sum()

    import warnings
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        clf = sk.LinearSVC(loss="hinge", C=1.0, dual=True, fit_intercept=True,
                           intercept_scaling=1.0, tol=1e-12, max_iter=10_000_000, random_state=0)
        clf.fit(Xs, y)
    for k in range(K):
        ours = primal(W[k] / sigma, b[k], k)
        theirs = primal(clf.coef_[k], clf.intercept_[k], k)
        assert ours <= theirs + 1e-9 * abs(theirs)
        assert abs(ours - theirs) <= 1e-7 * abs(theirs)
    np.testing.assert_allclose(W, sigma * clf.coef_, rtol=1e-6, atol=1e-8)
    np.testing.assert_allclose(b, clf.intercept_, rtol=1e-6, atol=1e-8)


def test_train_separates_synthetic_identities(ref):
    """On a tiny synthetic face set the trained scores classify every training
    crop correctly (a sanity check of the whole trainer, not a pin)."""
    from paper_1504_01883_amd import synth
    g, z, labels = synth.make_training_set(4, 5, 40, 40, synth.W_TINY)
    feat, _, _ = ref.features([(g.reshape(-1, 40), z.reshape(-1, 40))],
                              synth.stacked_boxes(len(labels), 40, 40))
    W, b, ep = ref.train_ovr_f64(feat, labels, K=4)
    _, am = ref.score_f64(feat, W.astype(np.float32), b.astype(np.float32))
    assert np.array_equal(am, labels)
