"""Pins of the oracle under the Matern-3/2 kernel (Section 5):
K(x, y) = (1 + sqrt(3) r / l) exp(-sqrt(3) r / l), r = ||x - y||.

Closed forms of the kernel, the textbook dense matrix, positive definiteness,
and the generic identities of the factorization (block form of M, exact
cases, PCG convergence) and of the Nystrom preconditioner, now with the
Matern kernel.  Every test restores the Gaussian kernel."""
import numpy as np
import pytest

import oracle


def matern_dense(X, l, Y=None):
    Y = X if Y is None else Y
    r = np.sqrt(((X[:, None, :] - Y[None, :, :]) ** 2).sum(-1))
    s = np.sqrt(3.0) * r / l
    return (1.0 + s) * np.exp(-s)


@pytest.fixture
def matern():
    oracle.set_kernel("matern32")
    yield
    oracle.set_kernel("gaussian")


def test_closed_forms(matern):
    o = np.zeros(3)
    l = 0.7
    e1 = np.array([1.0, 0.0, 0.0])
    assert oracle.kernel(o, o, l) == 1.0
    assert oracle.kernel(o, e1 * l / np.sqrt(3.0), l) == pytest.approx(2.0 / np.e, rel=1e-15)
    assert oracle.kernel(o, e1 * 2 * l / np.sqrt(3.0), l) == pytest.approx(3.0 * np.exp(-2.0), rel=1e-15)
    # small r: 1 - (3/2) (r/l)^2 + O(r^3)
    r = 1e-4
    assert oracle.kernel(o, e1 * r, l) == pytest.approx(1 - 1.5 * (r / l) ** 2, abs=1e-11)
    # the kind is restored by set_kernel("gaussian")
    oracle.set_kernel("gaussian")
    assert oracle.kernel(o, e1, 1.0) == pytest.approx(np.exp(-1.0), rel=1e-15)
    oracle.set_kernel("matern32")


def test_matvec_equals_textbook_matrix_and_is_positive_definite(matern):
    rng = np.random.default_rng(101)
    X = rng.random((60, 4))
    v = rng.standard_normal(60)
    K = matern_dense(X, 0.5)
    y = oracle.kernel_matvec(X, 0.5, 1e-3, v)
    np.testing.assert_allclose(y, K @ v + 1e-3 * v, rtol=1e-13, atol=1e-13)
    assert np.linalg.eigvalsh(K).min() > 0


def test_afn_block_identities(matern):
    rng = np.random.default_rng(102)
    n, k, w, l, mu = 120, 20, 8, 0.25, 1e-3
    X = rng.random((n, 3))
    idx, _ = oracle.fps(X, k)
    A = oracle.afn_build(X, l, mu, idx, w)
    Kp = matern_dense(X[A.perm], l) + mu * np.eye(n)
    # L = chol(K11 + mu I)
    np.testing.assert_allclose(A.L @ A.L.T, Kp[:k, :k], rtol=0, atol=1e-12)
    # M = [[L, 0], [K12^T L^-T, G^-1]] [[...]^T], with M11 = K11 + mu I, M12 = K12
    G = A.G_dense()
    Lo = np.zeros((n, n))
    Lo[:k, :k] = A.L
    Lo[k:, :k] = np.linalg.solve(A.L, Kp[:k, k:]).T
    Lo[k:, k:] = np.linalg.inv(G)
    M = Lo @ Lo.T
    np.testing.assert_allclose(M[:k, :], Kp[:k, :], atol=1e-10)
    assert np.linalg.eigvalsh(M).min() > 0
    r = rng.standard_normal(n)
    s = oracle.afn_apply(A, r)
    sp = np.linalg.solve(M, r[A.perm])
    np.testing.assert_allclose(s[A.perm], sp, rtol=1e-8, atol=1e-8 * np.abs(sp).max())


@pytest.mark.parametrize("case", ["k_eq_n", "full_pattern"])
def test_exact_cases_invert_the_regularized_matrix(matern, case):
    rng = np.random.default_rng(103)
    n, l, mu = 50, 0.3, 1e-2
    X = rng.random((n, 3))
    k = n if case == "k_eq_n" else 12
    idx, _ = oracle.fps(X, k)
    A = oracle.afn_build(X, l, mu, idx, n)
    r = rng.standard_normal(n)
    expect = np.linalg.solve(matern_dense(X, l) + mu * np.eye(n), r)
    np.testing.assert_allclose(oracle.afn_apply(A, r), expect, rtol=1e-8, atol=1e-10)
    x, it, rel, tr, st = oracle.pcg(A, r, 1e-10, 5)
    assert st == oracle.ORA_OK and it == 1


def test_pcg_solves_the_matern_system(matern):
    rng = np.random.default_rng(104)
    n, k, w, l, mu = 400, 40, 16, 0.2, 1e-3
    X = rng.random((n, 3))
    b = rng.standard_normal(n)
    idx, _ = oracle.fps(X, k)
    A = oracle.afn_build(X, l, mu, idx, w)
    x, it, rel, tr, st = oracle.pcg(A, b, 1e-10, 400)
    Kd = matern_dense(X, l) + mu * np.eye(n)
    assert st == oracle.ORA_OK
    assert np.linalg.norm(b - Kd @ x) <= 2e-10 * np.linalg.norm(b)


def test_rank_count_and_nystrom_follow_the_kernel(matern):
    rng = np.random.default_rng(105)
    X = rng.random((150, 3))
    l, mu = 0.4, 1e-3
    # eigenvalue count of the unscaled subsample matrix (m = n here)
    k, info = oracle.rank_estimate(X, l, mu, 150, kmax=2000)
    r, kest, eig_branch, eig_count = info
    assert eig_branch == 1
    assert eig_count == int((np.linalg.eigvalsh(matern_dense(X, l)) > 0.1 * mu).sum())
    # Nystrom: U Lambda U^T equals K[:, S] K_SS^{-1} K[S, :] for the Matern kernel
    idx, _ = oracle.fps(X, 15)
    N = oracle.nystrom_build(X, l, mu, idx)
    C = matern_dense(X, l, X[idx])
    ref = C @ np.linalg.solve(C[idx], C.T)
    assert np.linalg.norm(N.approx() - ref) <= 1e-9 * np.linalg.norm(ref)
