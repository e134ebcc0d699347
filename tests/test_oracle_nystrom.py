"""Pins of the oracle's Nystrom preconditioner (Algorithm 5, else-branch) to
facts that do not come from its own code: the textbook sampling formula
K[:, S] K_SS^{-1} K[S, :], exactness on the landmark rows, the dense inverse
of U Lambda U^T + mu I, the k = n limit, symmetry, the spectral bounds of
M^{-1}, and PCG's behaviour when the preconditioner is exact."""
import numpy as np
import pytest

import oracle
from paper_2304_05460_amd import workloads as W


def dense_K(X, l):
    D = ((X[:, None, :] - X[None, :, :]) ** 2).sum(-1)
    return np.exp(-D / l**2)


@pytest.fixture(scope="module")
def small():
    X = W.points("uniform", 300, 3, 71)
    l, mu, k = 0.15, 1e-3, 20
    idx, _ = oracle.fps(X, k)
    return X, l, mu, idx, oracle.nystrom_build(X, l, mu, idx)


def test_approximation_equals_textbook_sampling_formula(small):
    X, l, mu, idx, N = small
    K = dense_K(X, l)
    C = K[:, idx]
    Wss = K[np.ix_(idx, idx)]
    ref = C @ np.linalg.solve(Wss, C.T)
    kap = np.linalg.cond(Wss)
    assert np.linalg.norm(N.approx() - ref) <= 1e3 * kap * np.finfo(float).eps * np.linalg.norm(ref)


def test_landmark_rows_are_exact(small):
    X, l, mu, idx, N = small
    K = dense_K(X, l)
    kap = np.linalg.cond(K[np.ix_(idx, idx)])
    err = np.abs(N.approx()[idx, :] - K[idx, :]).max()
    assert err <= 1e3 * kap * np.finfo(float).eps


def test_u_orthonormal_and_spectrum_nonnegative(small):
    X, l, mu, idx, N = small
    assert np.allclose(N.U.T @ N.U, np.eye(N.k), atol=1e-12)
    assert np.all(N.lam >= 0) and np.all(np.diff(N.lam) <= 0)
    assert N.nu > 0 and N.nu < 1e-12


def test_apply_equals_dense_inverse(small):
    X, l, mu, idx, N = small
    M = N.approx() + mu * np.eye(X.shape[0])
    rng = np.random.default_rng(72)
    for _ in range(3):
        r = rng.standard_normal(X.shape[0])
        z = oracle.nystrom_apply(N, r)
        ref = np.linalg.solve(M, r)
        assert np.linalg.norm(z - ref) <= 1e-9 * np.linalg.norm(ref)


def test_apply_symmetric_and_within_spectral_bounds(small):
    X, l, mu, idx, N = small
    rng = np.random.default_rng(73)
    u, v = rng.standard_normal((2, X.shape[0]))
    a, b = u @ oracle.nystrom_apply(N, v), v @ oracle.nystrom_apply(N, u)
    assert abs(a - b) <= 1e-10 * (abs(a) + abs(b))
    lo, hi = 1.0 / (N.lam[0] + mu), 1.0 / mu
    for _ in range(5):
        r = rng.standard_normal(X.shape[0])
        q = (r @ oracle.nystrom_apply(N, r)) / (r @ r)
        assert lo * (1 - 1e-12) <= q <= hi * (1 + 1e-12)


def test_all_points_as_landmarks_gives_the_exact_inverse():
    # S = every point: the approximation is K itself, M = K + mu I
    X = W.points("uniform", 120, 2, 74)
    l, mu = 0.05, 1e-2
    idx, _ = oracle.fps(X, 120)
    N = oracle.nystrom_build(X, l, mu, idx)
    K = dense_K(X, l)
    r = np.random.default_rng(75).standard_normal(120)
    ref = np.linalg.solve(K + mu * np.eye(120), r)
    assert np.linalg.norm(oracle.nystrom_apply(N, r) - ref) <= 1e-10 * np.linalg.norm(ref)
    x, it, rel, conv = oracle.nystrom_pcg(N, r, 1e-12, 10, lambda v: (K + mu * np.eye(120)) @ v)
    assert conv and it <= 2


def test_pcg_reaches_tolerance_and_solves_the_system():
    X = W.points("uniform", 400, 3, 76)
    b = np.random.default_rng(77).standard_normal(400)
    l, mu = 0.3, 1e-3
    N, x, it, rel, conv = oracle.nystrom_solve(X, l, mu, 60, b, tol=1e-10, maxit=300)
    A = dense_K(X, l) + mu * np.eye(400)
    assert conv
    assert np.linalg.norm(b - A @ x) <= 2e-10 * np.linalg.norm(b) * 10
    xs = np.linalg.solve(A, b)
    assert np.linalg.norm(x - xs) <= np.linalg.cond(A) * 1e-9 * np.linalg.norm(xs)
