"""GPU parity under the Matern-3/2 kernel (Section 5),
K(x, y) = (1 + sqrt(3) r / l) exp(-sqrt(3) r / l), against the oracle run
with the same kernel.

Tolerances (u = 2^-53, u32 = 2^-24).  The tile kernels evaluate
K = (1 + s ln 2) 2^-s with s = sqrt(t), t the squared distance of
coordinates pre-scaled by c = sqrt(3) log2(e) / l.  A relative error e_t of t
gives an absolute error s e_t / 2 in s, and the rounding of the scaled
coordinates an absolute error of at most sqrt(d) max|x| c u; both enter
K through 2^-s, so a term with s <= S has relative error at most
ln 2 (S (d + 4) / 2 + sqrt(d) max|x| c) u + 8 u.  Terms beyond S are
bounded absolutely (2^-60 for S = 66 in FP64, 1e-13 for S = 50 in FP32),
which also covers the pruned tile pairs (2^-64, 2^-44)."""
import math

import numpy as np
import pytest

import oracle
from paper_2304_05460_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U = 2.0 ** -53
U32 = 2.0 ** -24
LN2 = math.log(2.0)
LOG2E = 1.0 / LN2


@pytest.fixture(scope="module")
def afn():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2304_05460_amd import afn as mod
    mod.lib()
    return mod


@pytest.fixture(autouse=True)
def matern():
    with oracle.use_kernel("matern32"):
        yield


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def say(*a):
    print(*a, flush=True)


def dense_matern(X, l, Y=None):
    Y = X if Y is None else Y
    r = np.sqrt(((X[:, None, :] - Y[None, :, :]) ** 2).sum(-1))
    s = math.sqrt(3.0) * r / l
    return (1.0 + s) * np.exp(-s)


def term_error(X, l, S):
    """Per-term relative error of the tile kernels' Matern value (in units of u)."""
    d = X.shape[1]
    c = math.sqrt(3.0) * LOG2E / l
    # coordinates packed relative to a data point, with up to 2 u each
    spread = float((X.max(0) - X.min(0)).max())
    return LN2 * (S * (d + 4) / 2 + 4 * math.sqrt(d) * spread * c) + 8


def bound64(X, l, v, ab):
    n = X.shape[0]
    return (2 * (n + 4) + term_error(X, l, 66)) * U * ab + 2.0 ** -60 * np.abs(v).sum()


def bound32(X, l, v, ab):
    n = X.shape[0]
    return (term_error(X, l, 50) + n + 8) * U32 * ab + 1e-13 * np.abs(v).sum()


def sample_rows(n, seed, count=40):
    return np.concatenate([np.arange(5), np.random.default_rng(seed).integers(0, n, count),
                           np.arange(n - 5, n)])


# ------------------------------------------------------------------ kernel matvec

@pytest.mark.parametrize("n,d,l,pts", [(2000, 3, 0.1, "uniform"), (1037, 8, 2.0, "normal"),
                                       (300, 1, 0.05, "uniform"), (517, 12, 3.0, "normal"),
                                       (1, 2, 0.5, "uniform")])
def test_matvec_fp64_all_rows(afn, n, d, l, pts):
    say(f"matern kmv fp64 n={n} d={d} l={l}")
    X = W.points(pts, n, d, 111)
    v = np.random.default_rng(112).standard_normal(n)
    y = afn.kernel_matvec(dev(X), l, 1e-4, dev(v), kernel=afn.AFN_KERNEL_MATERN32).cpu().numpy()
    yo, ab = oracle.kernel_matvec_rows(X, l, 1e-4, v, np.arange(n))
    bound = bound64(X, l, v, ab)
    assert np.all(np.abs(y - yo) <= bound), np.max(np.abs(y - yo) / bound)
    # the oracle itself is the textbook matrix
    if n <= 2000:
        K = dense_matern(X, l)
        assert np.all(np.abs(K @ v + 1e-4 * v - yo) <= 1e-12 * ab)


@pytest.mark.parametrize("n,d,l,pts", [(2000, 3, 0.1, "uniform"), (1037, 8, 2.0, "normal"),
                                       (600, 12, 1.5, "normal")])
def test_matvec_fp32_tiles(afn, n, d, l, pts):
    X = W.points(pts, n, d, 113)
    v = np.random.default_rng(114).standard_normal(n)
    y = afn.kernel_matvec(dev(X), l, 1e-4, dev(v), precision=afn.AFN_FP32,
                          kernel=afn.AFN_KERNEL_MATERN32).cpu().numpy()
    yo, ab = oracle.kernel_matvec_rows(X, l, 1e-4, v, np.arange(n))
    bound = bound32(X, l, v, ab)
    assert np.all(np.abs(y - yo) <= bound), np.max(np.abs(y - yo) / bound)


@pytest.mark.parametrize("l", [0.1, 0.01])
def test_matvec_full_size_pruned_sampled(afn, l):
    # the benchmark's point set (n = 1e5 mixture in the unit cube); at l = 0.01
    # the Matern cut (boxes 27.9 l apart in FP64, 19.7 l in FP32) prunes pairs
    p = W.c2(l)
    X = W.points(p.points, p.n, p.d, p.seed)
    v = np.random.default_rng(115).standard_normal(p.n)
    rows = sample_rows(p.n, 116)
    yo, ab = oracle.kernel_matvec_rows(X, l, p.mu, v, rows)
    for prec, bnd in ((afn.AFN_FP64, bound64), (afn.AFN_FP32, bound32)):
        say(f"matern kmv n={p.n} l={l} prec={prec}")
        y = afn.kernel_matvec(dev(X), l, p.mu, dev(v), precision=prec,
                              kernel=afn.AFN_KERNEL_MATERN32).cpu().numpy()
        bound = bnd(X, l, v, ab)
        assert np.all(np.abs(y[rows] - yo) <= bound), np.max(np.abs(y[rows] - yo) / bound)


@pytest.mark.parametrize("n,d,nrhs,prec", [(1037, 3, 16, 0), (700, 8, 5, 1), (20000, 3, 8, 0),
                                           (20000, 3, 8, 1)])
def test_matvec_many_rhs(afn, n, d, nrhs, prec):
    say(f"matern kmv mrhs n={n} d={d} nrhs={nrhs} prec={prec}")
    X = W.points("uniform" if d == 3 else "normal", n, d, 117)
    l = (0.02 if n > 10000 else 0.15) if d == 3 else 2.0
    V = np.random.default_rng(118).standard_normal((n, nrhs))
    Vt = torch.tensor(V.T.copy(), device="cuda").t()
    Y = afn.kernel_matvec(dev(X), l, 1e-3, Vt, precision=prec,
                          kernel=afn.AFN_KERNEL_MATERN32).cpu().numpy()
    rows = np.arange(n) if n <= 2000 else sample_rows(n, 119)
    for c in sorted({0, nrhs // 2, nrhs - 1}):
        yo, ab = oracle.kernel_matvec_rows(X, l, 1e-3, V[:, c], rows)
        bound = (bound64 if prec == 0 else bound32)(X, l, V[:, c], ab)
        assert np.all(np.abs(Y[rows, c] - yo) <= bound), (c, np.max(np.abs(Y[rows, c] - yo) / bound))


def test_unknown_kernel_is_rejected(afn):
    X = dev(W.points("uniform", 100, 3, 120))
    v = dev(np.ones(100))
    with pytest.raises(afn.AFNError) as e:
        afn.kernel_matvec(X, 0.3, 1e-3, v, kernel=2)
    assert e.value.status == afn.AFN_EINVAL
    with pytest.raises(afn.AFNError) as e:
        afn.afn_setup(X, 0.3, 1e-3, k=10, w=8, kernel=-1)
    assert e.value.status == afn.AFN_EINVAL


# ------------------------------------------------------------------ preconditioner

@pytest.fixture(scope="module")
def case(afn):
    # built before the per-test kernel switch; every test restores the Gaussian
    oracle.set_kernel("matern32")
    n, d, l, mu, k, w = 3000, 3, 0.1, 1e-3, 200, 32
    X = W.points("uniform", n, d, 121)
    b = np.random.default_rng(122).standard_normal(n)
    say("matern setup")
    h = afn.afn_setup(dev(X), l, mu, k=k, w=w, kernel=afn.AFN_KERNEL_MATERN32,
                      landmarks=afn.AFN_LANDMARKS_FPS)
    idx, _ = oracle.fps(X, k)
    A = oracle.afn_build(X, l, mu, idx, w)
    yield dict(n=n, d=d, l=l, mu=mu, k=k, w=w, X=X, b=b, h=h, A=A)
    h.close()


def test_setup_landmarks_pattern_cholesky(afn, case):
    h, A, k = case["h"], case["A"], case["k"]
    np.testing.assert_array_equal(h.landmarks(), A.perm[:k])
    rowptr, cols, vals = h.fsai()
    np.testing.assert_array_equal(rowptr, A.rowptr)
    np.testing.assert_array_equal(cols, A.cols)
    L = h.cholesky()
    Xp = case["X"][A.perm]
    A11 = dense_matern(Xp[:k], case["l"]) + case["mu"] * np.eye(k)
    assert np.linalg.norm(L @ L.T - A11) <= 8 * k * U * np.linalg.norm(A11)
    kappa = np.linalg.cond(A11)
    assert np.linalg.norm(L - A.L) <= 8 * k * U * kappa * np.linalg.norm(A.L)


def test_setup_fsai_matches_oracle(afn, case):
    h, A, k = case["h"], case["A"], case["k"]
    rowptr, cols, vals = h.fsai()
    Xp = case["X"][A.perm]
    K = dense_matern(Xp, case["l"]) + case["mu"] * np.eye(case["n"])
    S = K[k:, k:] - K[:k, k:].T @ np.linalg.solve(K[:k, :k], K[:k, k:])
    worst = 0.0
    for q in np.concatenate([np.arange(3), np.random.default_rng(123).integers(0, case["n"] - k, 30)]):
        s = cols[rowptr[q]:rowptr[q + 1]]
        g = vals[rowptr[q]:rowptr[q + 1]]
        rel = np.linalg.norm(g - A.gval[rowptr[q]:rowptr[q + 1]]) / np.linalg.norm(g)
        bound = np.linalg.cond(S[np.ix_(s, s)]) * k * 1e3 * U
        worst = max(worst, rel / max(1e-9, bound))
        assert rel <= max(1e-9, bound)
    say("matern FSAI worst rel/bound", worst)


def test_apply_and_pcg_match_oracle(afn, case):
    h, A, X, b = case["h"], case["A"], case["X"], case["b"]
    R = np.random.default_rng(124).standard_normal((case["n"], 2))
    S = np.stack([oracle.afn_apply(A, R[:, c]) for c in range(2)], axis=1)
    Sg = afn.afn_apply(h, dev(R.T).t()).cpu().numpy()
    rel = np.linalg.norm(Sg - S) / np.linalg.norm(S)
    say("matern apply rel", rel)
    assert rel <= 1e-7
    tol = 1e-8
    x, info = afn.afn_pcg_solve(h, dev(b), tol=tol, maxit=500)
    xo, ito, *_ = oracle.pcg(A, b, tol, 500)
    r = b - oracle.kernel_matvec(X, case["l"], case["mu"], x.cpu().numpy())
    say("matern pcg", info, "oracle its", ito)
    assert info["status"] == afn.AFN_OK
    assert np.linalg.norm(r) <= 2 * tol * np.linalg.norm(b)
    assert abs(info["iterations"] - ito) <= 2


def test_mixed_precision_and_block_solve(afn, case):
    X, l, mu = case["X"], case["l"], case["mu"]
    h = afn.afn_setup(dev(X), l, mu, k=case["k"], w=case["w"], precision=afn.AFN_FP32,
                      kernel=afn.AFN_KERNEL_MATERN32)
    B = np.random.default_rng(125).standard_normal((case["n"], 4))
    tol = 1e-10
    x1, i1 = afn.afn_pcg_solve(h, dev(B[:, 0]), tol=tol, maxit=500)
    xb, ib = afn.afn_pcg_solve(h, dev(B.T).t(), tol=tol, maxit=500)
    h.close()
    say("matern mixed", i1, "block", ib)
    assert i1["status"] == afn.AFN_OK and ib["status"] == afn.AFN_OK
    r = B[:, 0] - oracle.kernel_matvec(X, l, mu, x1.cpu().numpy())
    assert np.linalg.norm(r) <= 2 * tol * np.linalg.norm(B[:, 0])
    Xb = xb.cpu().numpy()
    for c in range(4):
        r = B[:, c] - oracle.kernel_matvec(X, l, mu, Xb[:, c])
        assert np.linalg.norm(r) <= 2 * tol * np.linalg.norm(B[:, c])


@pytest.mark.parametrize("l", [0.03, 0.3])
def test_rank_estimate_matches_oracle(afn, l):
    n, m = 20000, 400
    X = W.points("mixture5", n, 3, 126)
    say(f"matern rank l={l}")
    h = afn.afn_setup(dev(X), l, 1e-3, k=-1, w=16, k_max=2000, m=m, seed=7,
                      kernel=afn.AFN_KERNEL_MATERN32)
    inf = h.info()
    h.close()
    ko, info = oracle.rank_estimate(X, l, 1e-3, m, kmax=2000, kswitch=2000, seed=7)
    say("gpu", inf.k, inf.rank_r, inf.rank_k_est, inf.rank_eig_count, "oracle", ko, info)
    assert inf.rank_r == info[0] and inf.rank_eig_branch == info[2]
    assert inf.k == ko


def test_nystrom_apply_matches_oracle(afn):
    n, d, l, mu, k = 1500, 3, 0.3, 1e-3, 100
    X = W.points("uniform", n, d, 127)
    h = afn.afn_setup(dev(X), l, mu, k=k, method=afn.AFN_METHOD_NYSTROM,
                      kernel=afn.AFN_KERNEL_MATERN32)
    inf = h.info()
    idx, _ = oracle.fps(X, k)
    N = oracle.nystrom_build(X, l, mu, idx)
    assert abs(inf.nu - N.nu) <= 1e-10 * N.nu
    R = np.random.default_rng(128).standard_normal((n, 2))
    Z = afn.afn_apply(h, dev(R.T).t()).cpu().numpy()
    bound = 1e3 * ((N.lam[0] + mu) / mu * U + N.nu / mu)
    for c in range(2):
        zo = oracle.nystrom_apply(N, R[:, c])
        assert np.linalg.norm(Z[:, c] - zo) <= bound * np.linalg.norm(zo)
    b = R[:, 0]
    x, info = afn.afn_pcg_solve(h, dev(b), tol=1e-8, maxit=500)
    h.close()
    r = b - oracle.kernel_matvec(X, l, mu, x.cpu().numpy())
    assert info["status"] == afn.AFN_OK and np.linalg.norm(r) <= 2e-8 * np.linalg.norm(b)


def test_high_dimension_uniform_landmarks(afn):
    # d > 10: uniform landmarks, FSAI columns recomputed per batch, generic tiles
    n, d, k, w, l, mu, seed = 2500, 12, 150, 16, 3.0, 1e-2, 5
    X = W.points("normal", n, d, 129)
    h = afn.afn_setup(dev(X), l, mu, k=k, w=w, seed=seed, kernel=afn.AFN_KERNEL_MATERN32)
    idx = oracle.subsample(n, k, seed + 1)
    np.testing.assert_array_equal(h.landmarks(), idx)
    A = oracle.afn_build(X, l, mu, idx, w)
    r = np.random.default_rng(130).standard_normal(n)
    s = afn.afn_apply(h, dev(r)).cpu().numpy()
    so = oracle.afn_apply(A, r)
    assert np.linalg.norm(s - so) <= 1e-8 * np.linalg.norm(so)
    x, info = afn.afn_pcg_solve(h, dev(r), tol=1e-8, maxit=500)
    h.close()
    res = r - oracle.kernel_matvec(X, l, mu, x.cpu().numpy())
    assert info["status"] == afn.AFN_OK and np.linalg.norm(res) <= 2e-8 * np.linalg.norm(r)


def test_pruning_reach_follows_the_kernel(afn):
    # the Matern tail is heavier: at the same l, fewer tile pairs can be skipped
    p = W.c2(0.01)
    X = dev(W.points(p.points, p.n, p.d, p.seed))
    kept = {}
    for kern in (afn.AFN_KERNEL_GAUSSIAN, afn.AFN_KERNEL_MATERN32):
        h = afn.afn_setup(X, p.l, p.mu, k=100, w=8, kernel=kern)
        kept[kern] = (h.info().kmv_kept_f64, h.info().kmv_kept_f32)
        h.close()
    say("kept fractions", kept)
    g, m = kept[afn.AFN_KERNEL_GAUSSIAN], kept[afn.AFN_KERNEL_MATERN32]
    assert g[0] < m[0] < 1.0 and g[1] < m[1] < 1.0
    assert m[1] <= m[0]
