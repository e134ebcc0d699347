"""Pins for the oracle's AFN construction (Algorithms 1-2), application
(Algorithm 3), PCG and rank estimation (Algorithm 4).

Independent references used here: closed forms for 2x2 blocks, numpy/LAPACK
dense factorizations and solves (the oracle uses none of them), a full sort of
every predecessor for the kNN pattern, the dense block form of M (Eq. (3.1)
and its expansion), the exactness statement "G^T G = S^{-1} exactly gives
M = K + mu I", the FSAI orthogonality property of Kolotilina and Yeremin, a
textbook CG loop, published splitmix64 outputs and dense eigenvalues.
"""
import math

import numpy as np
import pytest

import oracle


def dense_K(X, l):
    D = ((X[:, None, :] - X[None, :, :]) ** 2).sum(-1)
    return np.exp(-D / l**2)


def dense_blocks(X, perm, k, l, mu):
    Xp = X[perm]
    K = dense_K(Xp, l)
    A = K + mu * np.eye(len(X))
    return A[:k, :k], A[:k, k:], A[k:, k:], K


def dense_schur(X, perm, k, l, mu):
    A11, A12, A22, _ = dense_blocks(X, perm, k, l, mu)
    if k == 0:
        return A22
    return A22 - A12.T @ np.linalg.solve(A11, A12)


# ----------------------------------------------------------------- Cholesky / solves

def test_cholesky_2x2_closed_form_and_not_spd():
    a, b, c = 4.0, 1.2, 3.0
    L = oracle.cholesky([[a, b], [b, c]])
    assert L[0, 0] == pytest.approx(math.sqrt(a), rel=1e-15)
    assert L[1, 0] == pytest.approx(b / math.sqrt(a), rel=1e-15)
    assert L[1, 1] == pytest.approx(math.sqrt(c - b * b / a), rel=1e-15)
    assert L[0, 1] == 0.0
    with pytest.raises(oracle.OracleError) as e:
        oracle.cholesky([[1.0, 2.0], [2.0, 1.0]])
    assert e.value.status == oracle.ORA_ENOTSPD


def test_cholesky_matches_lapack_and_reconstructs():
    rng = np.random.default_rng(0)
    B = rng.standard_normal((60, 60))
    A = B @ B.T + 60 * np.eye(60)
    L = oracle.cholesky(A)
    np.testing.assert_allclose(L, np.linalg.cholesky(A), rtol=1e-12, atol=1e-12)
    assert np.linalg.norm(L @ L.T - A) <= 60 * 1e-15 * np.linalg.norm(A) * 10
    b = rng.standard_normal(60)
    y = oracle.fwd_subst(L, b)
    x = oracle.bwd_subst(L, y)
    np.testing.assert_allclose(L @ y, b, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-10)


def test_landmark_cholesky_is_factor_of_regularized_K11():
    rng = np.random.default_rng(1)
    X = rng.random((50, 3))
    l, mu = 0.3, 1e-3
    L = oracle.landmark_cholesky(X, 20, l, mu)
    A11 = dense_K(X[:20], l) + mu * np.eye(20)
    np.testing.assert_allclose(L @ L.T, A11, rtol=0, atol=1e-12)
    assert np.all(np.triu(L, 1) == 0)


# ----------------------------------------------------------------- kNN pattern

def _knn_bruteforce(Xr, w):
    rows = []
    for p in range(len(Xr)):
        if p == 0:
            rows.append([0])
            continue
        d2 = ((Xr[:p] - Xr[p]) ** 2).sum(-1)
        order = np.lexsort((np.arange(p), d2))[: w - 1]      # by d2, then index
        rows.append(sorted(order.tolist()) + [p])
    return rows


@pytest.mark.parametrize("integer", [True, False])
@pytest.mark.parametrize("w", [1, 2, 5, 9])
def test_knn_pattern_matches_full_sort(integer, w):
    rng = np.random.default_rng(2 + w)
    Xr = (rng.integers(0, 4, size=(70, 3)).astype(float) if integer else rng.random((70, 3)))
    rowptr, cols = oracle.knn_pattern(Xr, w)
    expect = _knn_bruteforce(Xr, w)
    for p in range(70):
        got = cols[rowptr[p]:rowptr[p + 1]].tolist()
        assert got == expect[p], p
        assert len(got) == min(p + 1, w)
    sel = np.array([0, 1, 33, 69])
    out, ln = oracle.knn_rows(Xr, w, sel)
    for s, p in enumerate(sel):
        assert out[s, :ln[s]].tolist() == expect[p]


# ----------------------------------------------------------------- FSAI of the Schur complement

def _setup(n=120, k=20, w=8, l=0.25, mu=1e-3, seed=3, d=3):
    rng = np.random.default_rng(seed)
    X = rng.random((n, d))
    idx, _ = oracle.fps(X, k)
    A = oracle.afn_build(X, l, mu, idx, w)
    return X, A


def test_fsai_rows_satisfy_kolotilina_yeremin_conditions():
    # For G = FSAI(S) on pattern s_p: (G S)[p, s_a] = 0 for a != p and
    # (G S)[p, p] * G[p, p] = 1 (so (G S G^T)_pp = 1), diag(G) > 0.
    X, A = _setup()
    S = dense_schur(X, A.perm, A.k, A.l, A.mu)
    G = A.G_dense()
    GS = G @ S
    nr = S.shape[0]
    for p in range(nr):
        s = A.cols[A.rowptr[p]:A.rowptr[p + 1]]
        assert s[-1] == p
        off = GS[p, s[:-1]]
        assert np.max(np.abs(off), initial=0.0) <= 1e-9 * np.abs(GS[p]).max()
        assert GS[p, p] * G[p, p] == pytest.approx(1.0, rel=1e-9)
        assert G[p, p] > 0
    assert np.allclose(np.diag(G @ S @ G.T), 1.0, rtol=1e-9)


def test_fsai_row_2x2_closed_form():
    # S = [[a, b], [b, c]] with a full 2-entry pattern: G = chol(S)^{-1},
    # row 1 = [-b, a] / sqrt(a (ac - b^2)).
    rng = np.random.default_rng(4)
    X = rng.random((2, 2))
    l, mu = 0.7, 0.05
    A = oracle.afn_build(X, l, mu, np.zeros(0, dtype=np.int32), 2)
    S = dense_K(X, l) + mu * np.eye(2)
    a, b, c = S[0, 0], S[0, 1], S[1, 1]
    G = A.G_dense()
    assert G[0, 0] == pytest.approx(1 / math.sqrt(a), rel=1e-13)
    det = a * c - b * b
    assert G[1, 0] == pytest.approx(-b / math.sqrt(a * det), rel=1e-12)
    assert G[1, 1] == pytest.approx(a / math.sqrt(a * det), rel=1e-12)


def test_fsai_full_pattern_gives_exact_inverse_factor():
    # With w >= n - k every row holds all predecessors, so G^T G = S^{-1}.
    X, A = _setup(n=60, k=10, w=60)
    S = dense_schur(X, A.perm, A.k, A.l, A.mu)
    G = A.G_dense()
    np.testing.assert_allclose(G, np.linalg.inv(np.linalg.cholesky(S)), rtol=1e-7, atol=1e-7)


def test_fsai_rows_sampled_match_full_build():
    X, A = _setup(n=150, k=25, w=10)
    rows = np.array([0, 3, 9, 10, 77, 124])
    oc, ol, og = oracle.fsai_rows(X, A.l, A.mu, A.perm, A.L, A.w, rows)
    for s, p in enumerate(rows):
        a, b = A.rowptr[p], A.rowptr[p + 1]
        assert oc[s, :ol[s]].tolist() == A.cols[a:b].tolist()
        np.testing.assert_allclose(og[s, :ol[s]], A.gval[a:b], rtol=1e-13, atol=1e-13)


# ----------------------------------------------------------------- application (Algorithm 3)

def _dense_M(X, A):
    """Eq. (3.1): M = [[L, 0], [K12^T L^-T, G^-1]] [[L^T, L^-1 K12], [0, G^-T]]."""
    k = A.k
    A11, A12, A22, _ = dense_blocks(X, A.perm, k, A.l, A.mu)
    n = len(X)
    G = A.G_dense()
    Ginv = np.linalg.inv(G)
    Lo = np.zeros((n, n))
    Lo[:k, :k] = A.L
    Lo[k:, :k] = np.linalg.solve(A.L, A12).T if k else 0
    Lo[k:, k:] = Ginv
    return Lo @ Lo.T, A11, A12


def test_apply_equals_dense_inverse_of_block_factorization():
    X, A = _setup()
    M, A11, A12 = _dense_M(X, A)
    k = A.k
    np.testing.assert_allclose(M[:k, :k], A11, atol=1e-12)       # M11 = K11 + mu I
    np.testing.assert_allclose(M[:k, k:], A12, atol=1e-12)       # M12 = K12
    assert np.linalg.eigvalsh(M).min() > 0                        # M is SPD
    rng = np.random.default_rng(5)
    r = rng.standard_normal(len(X))
    s = oracle.afn_apply(A, r)
    sp = np.linalg.solve(M, r[A.perm])
    np.testing.assert_allclose(s[A.perm], sp, rtol=1e-8, atol=1e-8 * np.abs(sp).max())


def test_apply_is_symmetric_operator():
    X, A = _setup(seed=6)
    rng = np.random.default_rng(6)
    u, v = rng.standard_normal((2, len(X)))
    assert u @ oracle.afn_apply(A, v) == pytest.approx(v @ oracle.afn_apply(A, u), rel=1e-9)


@pytest.mark.parametrize("case", ["k_eq_n", "full_pattern"])
def test_apply_exact_cases_invert_regularized_K(case):
    # Section 3.2: G^T G = S^{-1} exactly (full pattern, or no Schur block when
    # k = n) gives M = K + mu I.
    rng = np.random.default_rng(7)
    n = 50
    X = rng.random((n, 3))
    l, mu = 0.3, 1e-2
    k = n if case == "k_eq_n" else 12
    idx, _ = oracle.fps(X, k)
    A = oracle.afn_build(X, l, mu, idx, n)
    r = rng.standard_normal(n)
    expect = np.linalg.solve(dense_K(X, l) + mu * np.eye(n), r)
    np.testing.assert_allclose(oracle.afn_apply(A, r), expect, rtol=1e-6, atol=1e-8)


def test_apply_k0_w1_is_scaled_identity():
    # k = 0, w = 1: G = I / sqrt(1 + mu), so M^{-1} r = r / (1 + mu).
    rng = np.random.default_rng(8)
    X = rng.random((40, 3))
    A = oracle.afn_build(X, 0.2, 0.5, np.zeros(0, dtype=np.int32), 1)
    r = rng.standard_normal(40)
    np.testing.assert_allclose(oracle.afn_apply(A, r), r / 1.5, rtol=1e-15)


# ----------------------------------------------------------------- PCG

def _cg_textbook(A, b, tol, maxit):
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = r @ r
    for it in range(1, maxit + 1):
        q = A @ p
        a = rr / (p @ q)
        x += a * p
        r -= a * q
        if np.linalg.norm(r) / np.linalg.norm(b) <= tol:
            return x, it
        rn = r @ r
        p = r + (rn / rr) * p
        rr = rn
    return x, maxit


def test_pcg_k0_w1_reproduces_plain_cg():
    rng = np.random.default_rng(9)
    n = 200
    X = rng.random((n, 3))
    l, mu = 0.1, 1e-2
    A = oracle.afn_build(X, l, mu, np.zeros(0, dtype=np.int32), 1)
    b = rng.standard_normal(n)
    x, its, rel, trel, st = oracle.pcg(A, b, 1e-10, 500)
    xc, itc = _cg_textbook(dense_K(X, l) + mu * np.eye(n), b, 1e-10, 500)
    assert st == oracle.ORA_OK
    assert abs(its - itc) <= 1
    np.testing.assert_allclose(x, xc, rtol=1e-7, atol=1e-9)


@pytest.mark.parametrize("case", ["k_eq_n", "full_pattern"])
def test_pcg_exact_preconditioner_converges_in_one_iteration(case):
    rng = np.random.default_rng(10)
    n = 60
    X = rng.random((n, 3))
    l, mu = 0.3, 1e-2
    k = n if case == "k_eq_n" else 15
    idx, _ = oracle.fps(X, k)
    A = oracle.afn_build(X, l, mu, idx, n)
    b = rng.standard_normal(n)
    x, its, rel, trel, st = oracle.pcg(A, b, 1e-8, 50)
    assert its == 1 and st == oracle.ORA_OK
    np.testing.assert_allclose(x, np.linalg.solve(dense_K(X, l) + mu * np.eye(n), b),
                               rtol=1e-6, atol=1e-8)


def test_pcg_forward_error_within_condition_bound():
    rng = np.random.default_rng(11)
    n = 400
    X = rng.random((n, 3))
    l, mu, tol = 0.15, 1e-3, 1e-9
    idx, _ = oracle.fps(X, 40)
    A = oracle.afn_build(X, l, mu, idx, 16)
    b = rng.standard_normal(n)
    x, its, rel, trel, st = oracle.pcg(A, b, tol, 500)
    Kr = dense_K(X, l) + mu * np.eye(n)
    xs = np.linalg.solve(Kr, b)
    kappa = np.linalg.cond(Kr)
    assert st == oracle.ORA_OK and rel <= tol
    assert trel <= 10 * tol
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= 10 * kappa * tol


def test_pcg_status_cases():
    rng = np.random.default_rng(12)
    n = 80
    X = rng.random((n, 3))
    idx, _ = oracle.fps(X, 10)
    A = oracle.afn_build(X, 0.1, 1e-4, idx, 8)
    x, its, *_ , st = oracle.pcg(A, np.zeros(n), 1e-8, 10)
    assert its == 0 and st == oracle.ORA_OK and not x.any()
    *_, st = oracle.pcg(A, rng.standard_normal(n), 1e-14, 1)
    assert st == oracle.ORA_ENOCONV
    b = rng.standard_normal(n)
    b[3] = np.nan
    *_, st = oracle.pcg(A, b, 1e-8, 10)
    assert st == oracle.ORA_EBREAKDOWN


def test_build_not_spd_with_duplicate_landmarks_and_zero_mu():
    X = np.zeros((10, 3))
    X[5:] = 1.0
    with pytest.raises(oracle.OracleError) as e:
        oracle.afn_build(X, 0.5, 0.0, np.array([0, 1], dtype=np.int32), 4)
    assert e.value.status == oracle.ORA_ENOTSPD


# ----------------------------------------------------------------- rank estimation (Algorithm 4)

def test_splitmix64_published_outputs():
    out = oracle.splitmix64_stream(0, 3)
    assert [int(v) for v in out] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def _fisher_yates_prefix(n, m, seed):
    """First m entries of the Fisher-Yates shuffle of 0..n-1 in which position
    i swaps with i + (draw_i mod (n - i)), draw_i the i-th splitmix64 output
    (the generator is pinned to its published outputs above)."""
    draws = [int(v) for v in oracle.splitmix64_stream(seed, m)]
    a = list(range(n))
    for i in range(m):
        j = i + draws[i] % (n - i)
        a[i], a[j] = a[j], a[i]
    return a[:m]


@pytest.mark.parametrize("n,m,seed", [(1000, 300, 42), (50, 50, 1), (12345, 2000, 7), (7, 1, 3)])
def test_subsample_is_the_fisher_yates_prefix(n, m, seed):
    assert oracle.subsample(n, m, seed).tolist() == _fisher_yates_prefix(n, m, seed)


def test_subsample_distinct_and_deterministic():
    a = oracle.subsample(1000, 300, 42)
    assert len(set(a.tolist())) == 300 and a.min() >= 0 and a.max() < 1000
    np.testing.assert_array_equal(a, oracle.subsample(1000, 300, 42))
    assert sorted(oracle.subsample(50, 50, 1).tolist()) == list(range(50))


def test_nystrom_scan_matches_direct_definition_and_is_monotone():
    rng = np.random.default_rng(13)
    X = rng.random((160, 3))
    K = dense_K(X, 0.3)
    ord_, _ = oracle.fps(X, 160)
    r, errs = oracle.nystrom_scan(K, ord_, step=8, tol=-1.0)   # never stops early
    checked = [i + 1 for i in range(160) if not np.isnan(errs[i])]
    assert checked[:3] == [8, 16, 24] and checked[-1] == 160
    e = np.array([errs[c - 1] for c in checked])
    assert np.all(np.diff(e) <= 1e-12)                        # nested prefixes: non-increasing
    assert e[-1] <= 1e-6                                       # r = m: exact
    for rr in (8, 16, 40):
        I = ord_[:rr]
        Kn = K[:, I] @ np.linalg.solve(K[np.ix_(I, I)], K[I, :])
        direct = np.linalg.norm(K - Kn) / np.linalg.norm(K)
        assert errs[rr - 1] == pytest.approx(direct, rel=1e-6, abs=1e-12)


def test_count_eigs_above_matches_dense_eigenvalues():
    rng = np.random.default_rng(14)
    for m in (5, 40, 150):
        B = rng.standard_normal((m, m))
        A = (B + B.T) / 2
        ev = np.linalg.eigvalsh(A)
        for tau in (-1.0, 0.0, 0.37, 2.5):
            if np.min(np.abs(ev - tau)) < 1e-8:
                continue
            assert oracle.count_eigs_above(A, tau) == int(np.sum(ev > tau))
    X = rng.random((120, 3))
    K = dense_K(X, 0.2)
    ev = np.linalg.eigvalsh(K)
    assert oracle.count_eigs_above(K, 1e-4) == int(np.sum(ev > 1e-4))


def test_rank_estimate_branches():
    rng = np.random.default_rng(15)
    X = rng.random((3000, 3))
    # smooth kernel: small rank -> eigenvalue branch, count of eig(K_m) > 0.1 mu
    k, info = oracle.rank_estimate(X, 1.0, 1e-3, 300, kmax=2000, kswitch=2000, seed=7)
    assert info[2] == 1 and k == info[3] and 1 <= k < 300
    sub = oracle.subsample(3000, 300, 7)
    ev = np.linalg.eigvalsh(dense_K(X[sub], 1.0))
    assert k == int(np.sum(ev > 1e-4))
    # rough kernel: r close to m -> k_est = floor(r n / m) >= switch -> capped
    k2, info2 = oracle.rank_estimate(X, 0.01, 1e-3, 300, kmax=500, kswitch=100, seed=7)
    assert info2[2] == 0 and (info2[0] % 8 == 0 or info2[0] == 300)
    assert info2[1] == (info2[0] * 3000) // 300 and k2 == min(500, info2[1])


def _fps_by_definition(X, k):
    """FPS written from its definition (Algorithm 6): the first point is the
    one nearest to the mean (each coordinate summed exactly by math.fsum), then
    repeatedly the unselected point farthest from the selected set; ties to the
    smallest index."""
    n, d = X.shape
    cen = np.array([math.fsum(X[:, t]) / n for t in range(d)])
    first = int(np.argmin(((X - cen) ** 2).sum(1)))
    D = ((X[:, None, :] - X[None, :, :]) ** 2).sum(-1)
    sel = [first]
    dist = D[first].copy()
    dist[first] = -1.0
    for _ in range(1, k):
        j = int(np.argmax(dist))
        sel.append(j)
        dist = np.minimum(dist, D[j])
        dist[sel] = -1.0
    return sel


def _nystrom_rank_by_definition(Xm, l, step=8, tol=0.1):
    """Smallest r in step, 2 step, ... (or m) whose Nystrom approximation
    K[:, I] K[I, I]^{-1} K[I, :] on the first r FPS points has relative
    Frobenius error below tol (Eq. (2.1)), each error formed directly."""
    m = Xm.shape[0]
    K = dense_K(Xm, l)
    order = _fps_by_definition(Xm, m)
    errs = {}
    for r in list(range(step, m, step)) + [m]:
        I = order[:r]
        Kn = K[:, I] @ np.linalg.solve(K[np.ix_(I, I)], K[I, :])
        errs[r] = np.linalg.norm(K - Kn) / np.linalg.norm(K)
        if errs[r] < tol:
            return r, errs
    return m, errs


def test_rank_estimate_scales_subsample_by_m_over_n():
    """Algorithm 4 on an interior case (8 < r < m, the eigenvalue branch not
    taken): the subsample's coordinates are scaled by (m/n)^(1/d) before the
    Nystrom error scan (Section 3.3), and k_est = floor(r n / m).  Every piece
    is recomputed here from its definition: the Fisher-Yates subsample, the
    scaled copy, a dense K, FPS and the Nystrom error of each prefix.  The
    other two readings of the scale, none and (n/m)^(1/d), give ranks far
    from it on this case, so either one would fail."""
    n, m, d, l = 3000, 300, 3, 0.1
    X = np.random.default_rng(16).random((n, d))
    k, info = oracle.rank_estimate(X, l, 1e-3, m, kmax=3000, kswitch=1, seed=11)
    sub = _fisher_yates_prefix(n, m, 11)
    ranks = {}
    for name, s in (("m/n", (m / n) ** (1 / d)), ("none", 1.0), ("n/m", (n / m) ** (1 / d))):
        ranks[name], errs = _nystrom_rank_by_definition(X[sub] * s, l)
        if name == "m/n":
            r = ranks[name]
            # the decision is not a rounding accident
            assert errs[r] < 0.1 * (1 - 1e-6) and errs[r - 8] > 0.1 * (1 + 1e-6)
    assert 8 < ranks["m/n"] < m
    assert abs(ranks["none"] - ranks["m/n"]) >= 64 and abs(ranks["n/m"] - ranks["m/n"]) >= 64
    assert info[2] == 0
    assert info[0] == ranks["m/n"]
    assert info[1] == (ranks["m/n"] * n) // m and k == info[1]


@pytest.mark.parametrize("c,per", [(100, 4), (150, 2), (37, 3)])
def test_rank_estimate_on_clusters_closed_form(c, per):
    """Alg. 4 on c clusters of `per` nearly coincident points one unit apart
    at l = 0.01 (m = n): K is block diagonal with c all-ones blocks of rank
    one, FPS takes one point per cluster before any second one, and after s
    eliminations the scan's error is sqrt((c - s) / c) (each block's Frobenius
    mass per^2), so the first multiple of 8 with error below 0.1 is
    8 ceil(c / 8); k_est = r < 2000 takes the eigenvalue branch, which counts
    the c eigenvalues near per above 0.1 mu (the rest are of the order of the
    squared jitter over l^2)."""
    rng = np.random.default_rng(500 + c)
    centres = np.stack([np.arange(c, dtype=float), np.zeros(c)], axis=1)
    X = np.repeat(centres, per, axis=0) + 1e-6 * rng.standard_normal((c * per, 2))
    X = X[rng.permutation(X.shape[0])]
    n = X.shape[0]
    k, info = oracle.rank_estimate(X, 0.01, 1e-3, n, kmax=n, kswitch=2000, seed=3)
    r, k_est, eig_branch, eig_count = info
    assert r == 8 * math.ceil(c / 8)
    assert k_est == r and eig_branch == 1
    assert eig_count == c and k == c
