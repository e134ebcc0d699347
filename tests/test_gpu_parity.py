"""GPU parity: the HIP path through the C-ABI against the FP64 oracle.

Tolerances (u = 2^-53 for FP64, u32 = 2^-24):
- kernel matvec FP64: any summation order of n terms, each with a faithfully
  rounded exp, is within (n + 4) u sum_j |K_ij v_j| of the exact sum; the
  same bound holds for the oracle, so |y_gpu - y_ora| <= 2 (n + 4) u abs_i.
- FP32 tiles: the exponent argument a = d^2 / l^2 carries a relative error of
  about (d + 4) u32 (coordinate rounding, d fma steps, scaling), so a term
  with a <= 30 has relative error <= 30 (d + 4) u32 ln 2; terms with a > 30
  are below 1e-13.  Accumulation adds L u32 (L = terms per partial sum).
- landmark indices, kNN patterns: bit-exact.
- L: backward error of a Cholesky factorization, ||L L^T - A|| <= 8 k u ||A||.
- G, apply, solutions: compared through invariants of the definitions and by
  relative differences bounded by the condition numbers stated in each test.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2304_05460_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U = 2.0 ** -53
U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def afn():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2304_05460_amd import afn as mod
    mod.lib()
    return mod


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def dense_K(X, l):
    D = ((X[:, None, :] - X[None, :, :]) ** 2).sum(-1)
    return np.exp(-D / l**2)


def say(*a):
    print(*a, flush=True)


# ------------------------------------------------------------------ kernel matvec

@pytest.mark.parametrize("n,d,l,pts", [(2000, 3, 0.1, "uniform"), (2000, 3, 1.0, "uniform"),
                                       (1037, 8, 2.0, "normal"), (1, 3, 0.5, "uniform"),
                                       (300, 1, 0.05, "uniform"), (517, 12, 3.0, "normal"),
                                       (777, 3, 1e-3, "uniform")])
def test_kernel_matvec_fp64_all_rows(afn, n, d, l, pts):
    say(f"kmv fp64 n={n} d={d} l={l}")
    X = W.points(pts, n, d, 11)
    v = np.random.default_rng(12).standard_normal(n)
    y = afn.kernel_matvec(dev(X), l, 1e-4, dev(v)).cpu().numpy()
    yo, ab = oracle.kernel_matvec_rows(X, l, 1e-4, v, np.arange(n))
    bound = 2 * (n + 4) * U * ab
    assert np.all(np.abs(y - yo) <= bound), np.max(np.abs(y - yo) / ab)


def test_kernel_matvec_multi_rhs_strided(afn):
    n, nrhs, ld = 901, 3, 1000
    X = W.points("uniform", n, 3, 13)
    V = np.random.default_rng(14).standard_normal((n, nrhs))
    Vt = torch.zeros((nrhs, ld), dtype=torch.float64, device="cuda")
    Vt[:, :n] = dev(V.T)
    Yt = torch.zeros((nrhs, ld), dtype=torch.float64, device="cuda")
    vin, yout = Vt.t()[:n], Yt.t()[:n]          # column-major views with ld = 1000
    afn.kernel_matvec(dev(X), 0.2, 1e-3, vin, out=yout)
    Y = Yt[:, :n].t().cpu().numpy()
    for c in range(nrhs):
        yo, ab = oracle.kernel_matvec_rows(X, 0.2, 1e-3, V[:, c], np.arange(n))
        assert np.all(np.abs(Y[:, c] - yo) <= 2 * (n + 4) * U * ab)
    assert not Yt[:, n:].any()                  # padding untouched


@pytest.mark.parametrize("n,d,l,pts", [(2000, 3, 0.1, "uniform"), (1037, 8, 2.0, "normal")])
def test_kernel_matvec_fp32_tiles(afn, n, d, l, pts):
    X = W.points(pts, n, d, 15)
    v = np.random.default_rng(16).standard_normal(n)
    y = afn.kernel_matvec(dev(X), l, 1e-4, dev(v), precision=afn.AFN_FP32).cpu().numpy()
    yo, ab = oracle.kernel_matvec_rows(X, l, 1e-4, v, np.arange(n))
    bound = (30 * (d + 4) * math.log(2) + n + 8) * U32 * ab + 1e-13 * np.abs(v).sum()
    assert np.all(np.abs(y - yo) <= bound), np.max(np.abs(y - yo) / ab)


# At n >= 8192 the kernels skip tile pairs whose kernel values are all below
# 2^-64 (FP64 tiles) or 2^-44 (FP32 tiles): each row may drop up to that
# bound times sum_j |v_j|, added to the rounding bounds below.
PRUNE64, PRUNE32 = 2.0 ** -64, 2.0 ** -44


def sample_rows(n, seed, count=40):
    return np.concatenate([np.arange(5), np.random.default_rng(seed).integers(0, n, count),
                           np.arange(n - 5, n)])


def test_kernel_matvec_large_sampled_rows(afn):
    p = W.c2(0.1)
    X = W.points(p.points, p.n, p.d, p.seed)
    v = np.random.default_rng(17).standard_normal(p.n)
    y = afn.kernel_matvec(dev(X), p.l, p.mu, dev(v)).cpu().numpy()
    rows = sample_rows(p.n, 18)
    yo, ab = oracle.kernel_matvec_rows(X, p.l, p.mu, v, rows)
    assert np.all(np.abs(y[rows] - yo) <= 2 * (p.n + 4) * U * ab + PRUNE64 * np.abs(v).sum())


def test_kernel_matvec_full_size_fp32_and_d8(afn):
    # the benchmark's mixture at n = 1e5 with FP32 tiles; 2e5 normal points in R^8 (FP64)
    p = W.c2(0.1)
    X = W.points(p.points, p.n, p.d, p.seed)
    v = np.random.default_rng(21).standard_normal(p.n)
    y = afn.kernel_matvec(dev(X), p.l, p.mu, dev(v), precision=afn.AFN_FP32).cpu().numpy()
    rows = sample_rows(p.n, 22)
    yo, ab = oracle.kernel_matvec_rows(X, p.l, p.mu, v, rows)
    bound = (30 * (p.d + 4) * math.log(2) + p.n + 8) * U32 * ab + (1e-13 + PRUNE32) * np.abs(v).sum()
    assert np.all(np.abs(y[rows] - yo) <= bound), np.max(np.abs(y[rows] - yo) / bound)
    q = W.C3
    X = W.points(q.points, q.n, q.d, q.seed)
    v = np.random.default_rng(23).standard_normal(q.n)
    y = afn.kernel_matvec(dev(X), q.l, q.mu, dev(v)).cpu().numpy()
    rows = sample_rows(q.n, 24, count=20)
    yo, ab = oracle.kernel_matvec_rows(X, q.l, q.mu, v, rows)
    assert np.all(np.abs(y[rows] - yo) <= 2 * (q.n + 4) * U * ab + PRUNE64 * np.abs(v).sum())


@pytest.mark.parametrize("kernel", [0, 1])
def test_kernel_matvec_compact_and_wide_tiles(afn, kernel):
    # a tight cluster (compact tiles: distances from norms and MFMA dot
    # products) and a sparse uniform background (tiles wider than the
    # centring limit: plain differences) in one pruned call
    rng = np.random.default_rng(25)
    n, l = 20000, 0.01
    X = np.concatenate([0.5 + 0.002 * rng.standard_normal((19000, 3)), rng.random((1000, 3))])
    v = rng.standard_normal(n)
    rows = np.concatenate([np.arange(8), 19000 + np.arange(8), rng.integers(0, n, 30)])
    with oracle.use_kernel("matern32" if kernel else "gaussian"):
        yo, ab = oracle.kernel_matvec_rows(X, l, 1e-3, v, rows)
    # Matern: the pruned pairs are below 2^-64 (2^-44) as well; its values
    # carry the extra sqrt rounding, covered by the factor 4
    for prec in (afn.AFN_FP64, afn.AFN_FP32):
        y = afn.kernel_matvec(dev(X), l, 1e-3, dev(v), precision=prec, kernel=kernel).cpu().numpy()
        if prec == afn.AFN_FP64:
            bound = 4 * 2 * (n + 4) * U * ab + PRUNE64 * np.abs(v).sum()
        else:
            bound = 4 * (30 * 7 * math.log(2) + n + 8) * U32 * ab + (1e-13 + PRUNE32) * np.abs(v).sum()
        err = np.abs(y[rows] - yo)
        say(f"compact+wide kernel={kernel} prec={prec}: worst err/bound {np.max(err / bound):.3f}")
        assert np.all(err <= bound)


@pytest.mark.parametrize("prec", [0, 1])
def test_kernel_matvec_full_size_64_columns(afn, prec):
    # 1.5e5 uniform points, l = 0.05, 64 columns: the MFMA tile kernel with pruning
    p = W.C4
    X = W.points(p.points, p.n, p.d, p.seed)
    V = np.random.default_rng(25).standard_normal((p.n, 64))
    Y = afn.kernel_matvec(dev(X), p.l, p.mu, dev(V.T).t(), precision=prec).cpu().numpy()
    rows = sample_rows(p.n, 26, count=15)
    for c in (0, 31, 63):
        yo, ab = oracle.kernel_matvec_rows(X, p.l, p.mu, V[:, c], rows)
        if prec == 0:
            bound = 2 * (p.n + 4) * U * ab + PRUNE64 * np.abs(V[:, c]).sum()
        else:
            bound = (30 * (p.d + 4) * math.log(2) + p.n + 8) * U32 * ab + (1e-13 + PRUNE32) * np.abs(V[:, c]).sum()
        assert np.all(np.abs(Y[rows, c] - yo) <= bound), (c, np.max(np.abs(Y[rows, c] - yo) / bound))


def test_kernel_matvec_invalid_arguments(afn):
    X = dev(np.zeros((10, 3)))
    v = dev(np.ones(10))
    for l, mu in [(0.0, 1e-3), (-1.0, 1e-3), (1.0, -1.0), (float("nan"), 0.0)]:
        with pytest.raises(afn.AFNError) as e:
            afn.kernel_matvec(X, l, mu, v)
        assert e.value.status == afn.AFN_EINVAL


# ------------------------------------------------------------------ setup pieces

def oracle_setup(X, l, mu, k, w):
    idx, _ = oracle.fps(X, k)
    return oracle.afn_build(X, l, mu, idx, w)


def gpu_csr(h):
    return h.fsai()


@pytest.fixture(scope="module")
def c1(afn):
    p = W.C1
    X, b = W.make(p)
    say("C1 setup")
    h = afn.afn_setup(dev(X), p.l, p.mu, k=p.k, w=p.w)
    A = oracle_setup(X, p.l, p.mu, p.k, p.w)
    return p, X, b, h, A


def test_c1_landmarks_bit_exact(c1):
    p, X, b, h, A = c1
    np.testing.assert_array_equal(h.landmarks(), A.perm[: p.k])


def test_c1_pattern_bit_exact(c1):
    p, X, b, h, A = c1
    rowptr, cols, _ = h.fsai()
    np.testing.assert_array_equal(rowptr, A.rowptr)
    np.testing.assert_array_equal(cols, A.cols)


def test_c1_cholesky_backward_error_and_oracle(c1):
    p, X, b, h, A = c1
    L = h.cholesky()
    Xp = X[A.perm]
    A11 = dense_K(Xp[: p.k], p.l) + p.mu * np.eye(p.k)
    assert np.all(np.triu(L, 1) == 0)
    assert np.linalg.norm(L @ L.T - A11) <= 8 * p.k * U * np.linalg.norm(A11)
    kappa = np.linalg.cond(A11)
    assert np.linalg.norm(L - A.L) <= 8 * p.k * U * kappa * np.linalg.norm(A.L)


def test_c1_fsai_invariants_and_oracle(c1):
    # Kolotilina-Yeremin conditions against the dense Schur complement, and
    # agreement with the oracle's G within the conditioning of the blocks.
    p, X, b, h, A = c1
    rowptr, cols, vals = h.fsai()
    Xp = X[A.perm]
    K = dense_K(Xp, p.l) + p.mu * np.eye(p.n)
    k = p.k
    S = K[k:, k:] - K[:k, k:].T @ np.linalg.solve(K[:k, :k], K[:k, k:])
    rng = np.random.default_rng(19)
    worst = dict(ky_diag=0.0, ky_off=0.0, rel_vs_oracle=0.0, bound=0.0)
    for q in np.concatenate([np.arange(3), rng.integers(0, p.n - k, 30)]):
        s = cols[rowptr[q]:rowptr[q + 1]]
        g = vals[rowptr[q]:rowptr[q + 1]]
        Sss = S[np.ix_(s, s)]
        r = g @ Sss
        kap = np.linalg.cond(Sss)
        assert g[-1] > 0
        ky_diag = abs(r[-1] * g[-1] - 1.0)
        ky_off = np.max(np.abs(r[:-1]), initial=0.0) / abs(r[-1])
        rel = np.linalg.norm(g - A.gval[rowptr[q]:rowptr[q + 1]]) / np.linalg.norm(g)
        bound = kap * k * 1e3 * U
        worst = {key: max(worst[key], val) for key, val in
                 dict(ky_diag=ky_diag, ky_off=ky_off, rel_vs_oracle=rel, bound=bound).items()}
        # the dense Schur complement carries cancellation error of order
        # k u kappa(K11 + mu I) relative to its entries, which enters the
        # invariants through kappa(S_ss)
        assert ky_diag <= 1e-5 and ky_off <= 1e-5
        assert rel <= max(1e-9, bound)
    say("C1 FSAI worst", worst)


def test_c1_apply_matches_oracle_and_is_symmetric(afn, c1):
    p, X, b, h, A = c1
    rng = np.random.default_rng(20)
    R = rng.standard_normal((p.n, 2))
    S = np.stack([oracle.afn_apply(A, R[:, c]) for c in range(2)], axis=1)
    Sg = np.stack([afn.afn_apply(h, dev(R[:, c])).cpu().numpy() for c in range(2)], axis=1)
    rel = np.linalg.norm(Sg - S) / np.linalg.norm(S)
    say("apply rel diff", rel)
    assert rel <= 1e-7
    assert R[:, 0] @ Sg[:, 1] == pytest.approx(R[:, 1] @ Sg[:, 0], rel=1e-9)


def _per_row_g_and_apply(afn, h, A, X, l, mu, k, w, seed):
    """Every row of G against the oracle's, each with the bound of its own
    block (kappa(S_ss) k 1e3 u, as in the sampled C1 test), and the apply
    entry by entry, each entry against the largest entry of its own group:
    the landmark entries, the first w - 1 non-landmark rows (short patterns),
    the last 64 rows of the block order and the rest.  A wrong short row or
    tail row cannot hide under the bulk."""
    n = X.shape[0]
    rowptr, cols, vals = h.fsai()
    Xp = X[A.perm]
    K = dense_K(Xp, l) + mu * np.eye(n)
    S = K[k:, k:] - (K[:k, k:].T @ np.linalg.solve(K[:k, :k], K[:k, k:]) if k > 0 else 0.0)
    worst_g = 0.0
    for q in range(n - k):
        a, b_ = rowptr[q], rowptr[q + 1]
        s_, g = cols[a:b_], vals[a:b_]
        go = A.gval[a:b_]
        kap = np.linalg.cond(S[np.ix_(s_, s_)])
        bound = max(1e-9, kap * max(k, 1) * 1e3 * U)
        rel = np.max(np.abs(g - go)) / np.max(np.abs(go))
        worst_g = max(worst_g, rel / bound)
        assert rel <= bound, (q, rel, bound)
    r = np.random.default_rng(seed).standard_normal(n)
    z = afn.afn_apply(h, dev(r)).cpu().numpy()
    zo = oracle.afn_apply(A, r)
    pos = np.empty(n, dtype=np.int64)
    pos[A.perm] = np.arange(n)           # block position of each original index
    groups = {"landmarks": pos < k, "short rows": (pos >= k) & (pos < k + w - 1),
              "last tile": pos >= n - 64}
    groups["bulk"] = ~(groups["landmarks"] | groups["short rows"] | groups["last tile"])
    worst_z = {}
    for name, m in groups.items():
        if not m.any():
            continue
        scale = np.max(np.abs(zo[m]))
        err = np.max(np.abs(z[m] - zo[m])) / scale
        worst_z[name] = err
        assert err <= 1e-9, (name, err)
    say("per-row G worst/bound", worst_g, "apply per entry", worst_z)


def test_c1_g_rows_and_apply_entries(afn, c1):
    p, X, b, h, A = c1
    _per_row_g_and_apply(afn, h, A, X, p.l, p.mu, p.k, p.w, 21)


@pytest.mark.parametrize("n,k,w,d", [(70, 3, 64, 3), (333, 17, 5, 8), (1500, 100, 40, 3), (1100, 60, 64, 5),
                                     (1500, 100, 100, 3), (900, 40, 128, 8), (300, 10, 70, 5)])
def test_ragged_g_rows_and_apply_entries(afn, n, k, w, d):
    X = W.points("normal" if d >= 5 else "uniform", n, d, 29 + n)
    l, mu = 0.7, 1e-2
    h = afn.afn_setup(dev(X), l, mu, k=k, w=w, landmarks=afn.AFN_LANDMARKS_FPS)
    A = oracle_setup(X, l, mu, k, w)
    _per_row_g_and_apply(afn, h, A, X, l, mu, k, w, 22)
    h.close()


@pytest.mark.parametrize("w", [100, 128])
def test_wide_pattern_pcg_matches_oracle(afn, w):
    """Patterns wider than one wavefront (w > 64; the paper's AFN runs use
    w = 100): single and block solves against the oracle's PCG."""
    n, d, k, l, mu = 3000, 3, 200, 0.1, 1e-4
    X = W.points("uniform", n, d, 61)
    b = np.random.default_rng(62).standard_normal(n)
    h = afn.afn_setup(dev(X), l, mu, k=k, w=w, landmarks=afn.AFN_LANDMARKS_FPS)
    A = oracle_setup(X, l, mu, k, w)
    x, info = afn.afn_pcg_solve(h, dev(b), tol=1e-10, maxit=500)
    xo, ito, *_ = oracle.pcg(A, b, 1e-10, 500)
    say(f"w={w} gpu", info["iterations"], "oracle", ito)
    assert info["converged"] and abs(info["iterations"] - ito) <= 2
    rel = np.linalg.norm(x.cpu().numpy() - xo) / np.linalg.norm(xo)
    assert rel <= 1e-6
    B = np.random.default_rng(63).standard_normal((n, 6))
    Bt = torch.tensor(B.T.copy(), device="cuda").t()
    xb, ib = afn.afn_pcg_solve(h, Bt, tol=1e-10, maxit=500)
    h.close()
    for c in (0, 5):
        xoc, *_ = oracle.pcg(A, B[:, c], 1e-10, 500)
        relc = np.linalg.norm(xb[:, c].cpu().numpy() - xoc) / np.linalg.norm(xoc)
        assert relc <= 1e-6, (c, relc)


def test_c1_pcg_matching_residual(afn, c1):
    p, X, b, h, A = c1
    x, info = afn.afn_pcg_solve(h, dev(b), tol=p.tol, maxit=p.maxit)
    x = x.cpu().numpy()
    say("C1 gpu", info)
    assert info["converged"] and info["relres"] <= p.tol
    # true residual recomputed by the oracle's FP64 matvec
    r = b - oracle.kernel_matvec(X, p.l, p.mu, x)
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 2 * p.tol
    xo, ito, rel_o, trel_o, st = oracle.pcg(A, b, p.tol, p.maxit)
    say("C1 oracle iterations", ito, "gpu", info["iterations"])
    assert abs(info["iterations"] - ito) <= 2
    # at a tightened tolerance both solutions sit within kappa * tol of the
    # exact one, so they agree to well below 1e-6
    x2, info2 = afn.afn_pcg_solve(h, dev(b), tol=1e-12, maxit=p.maxit)
    xo2, *_ = oracle.pcg(A, b, 1e-12, p.maxit)
    rel = np.linalg.norm(x2.cpu().numpy() - xo2) / np.linalg.norm(xo2)
    say("C1 solution agreement at tol 1e-12:", rel)
    assert rel <= 1e-6


def test_c1_deterministic(afn, c1):
    p, X, b, h, A = c1
    h2 = afn.afn_setup(dev(X), p.l, p.mu, k=p.k, w=p.w)
    r1, c1_, v1 = h.fsai()
    r2, c2_, v2 = h2.fsai()
    np.testing.assert_array_equal(v1, v2)
    x1, _ = afn.afn_pcg_solve(h, dev(b), tol=1e-6)
    x2, _ = afn.afn_pcg_solve(h2, dev(b), tol=1e-6)
    assert torch.equal(x1, x2)


# ------------------------------------------------------------------ exact / degenerate cases

def test_k_equals_n_is_exact(afn):
    n = 300
    X = W.points("uniform", n, 3, 21)
    b = np.random.default_rng(22).standard_normal(n)
    h = afn.afn_setup(dev(X), 0.3, 1e-2, k=n, w=8)
    x, info = afn.afn_pcg_solve(h, dev(b), tol=1e-10)
    assert info["iterations"] == 1
    xs = np.linalg.solve(dense_K(X, 0.3) + 1e-2 * np.eye(n), b)
    np.testing.assert_allclose(x.cpu().numpy(), xs, rtol=1e-6, atol=1e-8)


def test_full_pattern_is_exact(afn):
    n, k = 100, 40                       # n - k = 60 <= w = 64: every row is complete
    X = W.points("uniform", n, 3, 23)
    b = np.random.default_rng(24).standard_normal(n)
    h = afn.afn_setup(dev(X), 0.3, 1e-2, k=k, w=64)
    x, info = afn.afn_pcg_solve(h, dev(b), tol=1e-10)
    assert info["iterations"] == 1
    xs = np.linalg.solve(dense_K(X, 0.3) + 1e-2 * np.eye(n), b)
    np.testing.assert_allclose(x.cpu().numpy(), xs, rtol=1e-6, atol=1e-8)


def test_k0_w1_is_plain_cg(afn):
    n = 400
    X = W.points("uniform", n, 3, 25)
    b = np.random.default_rng(26).standard_normal(n)
    l, mu = 0.1, 1e-2
    h = afn.afn_setup(dev(X), l, mu, k=0, w=1)
    x, info = afn.afn_pcg_solve(h, dev(b), tol=1e-10)
    A = dense_K(X, l) + mu * np.eye(n)
    xk = np.zeros(n); r = b.copy(); pp = r.copy(); rr = r @ r; its = 0
    while True:
        q = A @ pp; a = rr / (pp @ q); xk += a * pp; r -= a * q; its += 1
        if np.linalg.norm(r) / np.linalg.norm(b) <= 1e-10 or its >= 500:
            break
        rn = r @ r; pp = r + rn / rr * pp; rr = rn
    assert abs(info["iterations"] - its) <= 1
    np.testing.assert_allclose(x.cpu().numpy(), xk, rtol=1e-7, atol=1e-9)


@pytest.mark.parametrize("n,k,w,d", [(1, 1, 1, 3), (5, 0, 3, 2), (70, 3, 64, 3), (333, 17, 5, 8),
                                     (129, 64, 64, 3), (200, 65, 7, 12), (150, 20, 100, 3)])
def test_small_and_ragged_shapes_match_oracle(afn, n, k, w, d):
    say(f"ragged n={n} k={k} w={w} d={d}")
    X = W.points("normal" if d == 8 else "uniform", n, d, 27 + n)
    l, mu = 0.7, 1e-2
    h = afn.afn_setup(dev(X), l, mu, k=k, w=w, landmarks=afn.AFN_LANDMARKS_FPS)
    A = oracle_setup(X, l, mu, k, w)
    np.testing.assert_array_equal(h.landmarks(), A.perm[:k])
    rowptr, cols, vals = h.fsai()
    np.testing.assert_array_equal(rowptr, A.rowptr)
    np.testing.assert_array_equal(cols, A.cols)
    if vals.size:
        assert np.linalg.norm(vals - A.gval) <= 1e-8 * np.linalg.norm(A.gval)
    r = np.random.default_rng(n).standard_normal(n)
    s = afn.afn_apply(h, dev(r)).cpu().numpy()
    so = oracle.afn_apply(A, r)
    assert np.linalg.norm(s - so) <= 1e-8 * np.linalg.norm(so)


def test_fps_with_ties_and_duplicates(afn):
    rng = np.random.default_rng(31)
    X = rng.integers(0, 5, size=(3000, 3)).astype(float)
    h = afn.afn_setup(dev(X), 0.5, 1e-2, k=100, w=16)
    idx, _ = oracle.fps(X, 100)
    np.testing.assert_array_equal(h.landmarks(), idx)


@pytest.mark.parametrize("n,d,k", [
    (2048, 8, 300),     # one workgroup, four points per thread, n d = 16384
    (2049, 3, 500),     # one workgroup, sixteen points per thread
    (8192, 2, 400),     # the largest point count of the one-workgroup form
    (8193, 2, 200),     # one launch per step
    (6741, 3, 256),     # n d = 20223: coordinates fill the LDS
    (6742, 3, 130),     # one more point: one launch per step
    (300, 3, 300),      # every point selected (the final step only reports)
    (500, 4, 1),        # the first landmark only
])
def test_fps_one_workgroup_and_per_step_forms(afn, n, d, k):
    X = W.points("mixture5", n, d, 40 + d)
    say(f"fps n={n} d={d} k={k}")
    h = afn.afn_setup(dev(X), 0.3, 1e-2, k=k, w=8, landmarks=afn.AFN_LANDMARKS_FPS)
    idx, _ = oracle.fps(X, k)
    np.testing.assert_array_equal(h.landmarks(), idx)


# ------------------------------------------------------------------ full-size setup (C2 shape)

def test_c2_fps_pattern_and_fsai_sampled(afn):
    p = W.c2(0.1)
    X = W.points(p.points, p.n, p.d, p.seed)
    k = 2000
    say("C2 setup k=2000")
    h = afn.afn_setup(dev(X), p.l, p.mu, k=k, w=p.w)
    idx, _ = oracle.fps(X, k)
    np.testing.assert_array_equal(h.landmarks(), idx)
    perm = oracle.permutation(p.n, idx)
    Xr = X[perm[k:]]
    rowptr, cols, vals = h.fsai()
    rows = np.concatenate([np.arange(3), [62, 63, 64],
                           np.random.default_rng(32).integers(0, p.n - k, 20)])
    oc, ol = oracle.knn_rows(Xr, p.w, rows)
    for s_, q in enumerate(rows):
        np.testing.assert_array_equal(cols[rowptr[q]:rowptr[q + 1]], oc[s_, :ol[s_]])
    L = oracle.landmark_cholesky(X[perm], k, p.l, p.mu)
    fc, fl, fg = oracle.fsai_rows(X, p.l, p.mu, perm, L, p.w, rows[:8])
    for s_, q in enumerate(rows[:8]):
        g = vals[rowptr[q]:rowptr[q + 1]]
        assert np.linalg.norm(g - fg[s_, :fl[s_]]) <= 1e-6 * np.linalg.norm(g)


@pytest.mark.parametrize("n,d,w,pts", [(12000, 3, 64, "mixture5"), (9000, 2, 33, "uniform"),
                                       (8000, 5, 17, "normal"), (10000, 8, 64, "normal"),
                                       (5000, 1, 8, "uniform"), (3000, 3, 1, "uniform"),
                                       (700, 4, 64, "uniform"), (6000, 3, 100, "uniform"),
                                       (5000, 8, 128, "normal"), (700, 4, 65, "mixture5"),
                                       (2500, 12, 100, "normal")])
def test_knn_pattern_full_with_tiles(afn, n, d, w, pts):
    # every row of the predecessor pattern, bit-exact, across the tile-pruned
    # search (rows p >= (n-k)/4) and the full scan (the other rows)
    X = W.points(pts, n, d, 34)
    k = 30
    say(f"knn full n={n} d={d} w={w}")
    h = afn.afn_setup(dev(X), 1.0, 1e-2, k=k, w=w)
    perm = oracle.permutation(n, h.landmarks())
    rowptr, cols, _ = h.fsai()
    orp, ocols = oracle.knn_pattern(X[perm[k:]], w)
    np.testing.assert_array_equal(rowptr, orp)
    np.testing.assert_array_equal(cols, ocols)


# ------------------------------------------------------------------ rank estimation

@pytest.mark.parametrize("l", [0.02, 0.1, 1.0])
def test_rank_estimate_matches_oracle(afn, l):
    n, m = 20000, 400
    X = W.points("mixture5", n, 3, 33)
    say(f"rank l={l}")
    h = afn.afn_setup(dev(X), l, 1e-3, k=-1, w=16, k_max=2000, m=m, seed=99)
    inf = h.info()
    ko, info = oracle.rank_estimate(X, l, 1e-3, m, kmax=2000, kswitch=2000, seed=99)
    say("gpu", inf.k, inf.rank_r, inf.rank_k_est, inf.rank_eig_count, "oracle", ko, info)
    assert inf.rank_r == info[0]
    assert inf.rank_eig_branch == info[2]
    assert inf.k == ko
    idx, _ = oracle.fps(X, ko)
    np.testing.assert_array_equal(h.landmarks(), idx)


@pytest.mark.parametrize("case", ["skipped_pivots", "ragged_last_pass"])
def test_rank_scan_edges_match_oracle(afn, case):
    # skipped_pivots: 40 points, l = 100: K is all but constant, so after the
    # first elimination every pivot is below 1e-14 m and its row and column are
    # zeroed (the error is taken after step 8).  ragged_last_pass: 61 points far
    # apart at l = 1e-3: K = I, the error sqrt((m - r) / m) stays above 0.1 to
    # the end, so r = m = 61, taken after a last pass of 29 steps whose final
    # group has 5.
    if case == "skipped_pivots":
        X = W.points("uniform", 40, 3, 71)
        l, m = 100.0, 40
    else:
        X = np.arange(61, dtype=float)[:, None] * np.ones((1, 2))
        l, m = 1e-3, 61
    n = X.shape[0]
    say(f"rank scan {case}")
    h = afn.afn_setup(dev(X), l, 1e-3, k=-1, w=4, k_max=n, m=m, seed=5, method=afn.AFN_METHOD_NYSTROM)
    inf = h.info()
    ko, info = oracle.rank_estimate(X, l, 1e-3, m, kmax=n, kswitch=2000, seed=5)
    say("gpu", inf.k, inf.rank_r, inf.rank_k_est, inf.rank_eig_count, "oracle", ko, info)
    assert inf.rank_r == info[0]
    assert inf.rank_r == (8 if case == "skipped_pivots" else 61)
    assert inf.rank_eig_branch == info[2] and inf.k == ko


@pytest.mark.parametrize("case,c,expect_r", [("stop_in_odd_chunk", 100, 104), ("stop_in_even_chunk", 150, 152),
                                             ("two_full_chunks", 128, 128)])
def test_rank_scan_fps_chunks_match_oracle(afn, case, c, expect_r):
    # The subsample's FPS order comes in 64-step chunks, each computed one
    # chunk ahead of the scan.  Clusters of c groups of nearly coincident
    # points one unit apart at l = 0.01: K is block diagonal with all-ones
    # blocks, FPS takes one point per cluster first, and after 8 j steps the
    # scan error is sqrt(remaining clusters / c), so r = 8 ceil(c / 8): the
    # scan stops inside chunk 1 or 2 with the next chunk already under way.
    # two_full_chunks: 128 points far apart at l = 1e-3 (K = I) use both
    # chunks to the end.  m = n, so no scaling and no sampling choice.
    rng = np.random.default_rng(123 + c)
    if case == "two_full_chunks":
        X = np.stack([np.arange(c, dtype=float), np.zeros(c)], axis=1)
        l = 1e-3
    else:
        per = 4 if c == 100 else 2
        centres = np.stack([np.arange(c, dtype=float), np.zeros(c)], axis=1)
        X = np.repeat(centres, per, axis=0) + 1e-6 * rng.standard_normal((c * per, 2))
        X = X[rng.permutation(X.shape[0])]
        l = 0.01
    n = X.shape[0]
    m = n
    say(f"rank scan chunks {case} n={n}")
    h = afn.afn_setup(dev(X), l, 1e-3, k=-1, w=4, k_max=n, m=m, seed=7, method=afn.AFN_METHOD_NYSTROM)
    inf = h.info()
    ko, info = oracle.rank_estimate(X, l, 1e-3, m, kmax=n, kswitch=2000, seed=7)
    say("gpu", inf.k, inf.rank_r, inf.rank_k_est, inf.rank_eig_count, "oracle", ko, info)
    assert info[0] == expect_r
    assert inf.rank_r == info[0]
    assert inf.rank_eig_branch == info[2] == 1 and inf.rank_eig_count == info[3]
    assert inf.k == ko
    idx, _ = oracle.fps(X, ko)
    np.testing.assert_array_equal(h.landmarks(), idx)


def test_rank_estimate_largest_subsample(afn):
    # m at its maximum: the tridiagonalization's LDS per launch (3 (m - j - 2)
    # doubles) exceeds 64 KB in the first steps
    n, m, l = 6000, 4096, 1.0
    X = W.points("mixture5", n, 3, 33)
    say(f"rank m={m}")
    h = afn.afn_setup(dev(X), l, 1e-3, k=-1, w=16, k_max=2000, m=m, seed=99)
    inf = h.info()
    ko, info = oracle.rank_estimate(X, l, 1e-3, m, kmax=2000, kswitch=2000, seed=99)
    say("gpu", inf.k, inf.rank_r, inf.rank_eig_count, "oracle", ko, info)
    assert inf.rank_r == info[0] and inf.rank_eig_branch == info[2] == 1
    assert inf.k == ko


# ------------------------------------------------------------------ failures

def test_setup_errors(afn):
    X = np.zeros((20, 3))
    X[10:] = 1.0
    with pytest.raises(afn.AFNError) as e:
        afn.afn_setup(dev(X), 0.5, 0.0, k=4, w=4)          # duplicate landmarks, mu = 0
    assert e.value.status == afn.AFN_ENOTSPD
    for kw in [dict(k=21, w=4), dict(k=2, w=0), dict(k=2, w=129), dict(k=-2, w=4)]:
        with pytest.raises(afn.AFNError) as e:
            afn.afn_setup(dev(W.points("uniform", 20, 3, 1)), 0.5, 1e-2, **kw)
        assert e.value.status == afn.AFN_EINVAL
    Xn = W.points("uniform", 20, 3, 1)
    Xn[3, 1] = np.nan
    with pytest.raises(afn.AFNError) as e:
        afn.afn_setup(dev(Xn), 0.5, 1e-2, k=2, w=4)
    assert e.value.status == afn.AFN_EINVAL


def test_solve_status_codes(afn):
    n = 500
    X = W.points("uniform", n, 3, 41)
    h = afn.afn_setup(dev(X), 0.1, 1e-4, k=20, w=8)
    b = np.random.default_rng(42).standard_normal(n)
    x, info = afn.afn_pcg_solve(h, dev(b), tol=1e-14, maxit=1)
    assert info["status"] == afn.AFN_ENOCONV and info["iterations"] == 1
    bn = b.copy()
    bn[7] = np.nan
    with pytest.raises(afn.AFNError) as e:
        afn.afn_pcg_solve(h, dev(bn), tol=1e-8)
    assert e.value.status == afn.AFN_EBREAKDOWN
    x, info = afn.afn_pcg_solve(h, dev(np.zeros(n)), tol=1e-8)
    assert info["iterations"] == 0 and not x.any()


# ------------------------------------------------------------------ mixed precision (FP32 inner, FP64 refinement)

def test_mixed_c1_matches_fp64_oracle(afn, c1):
    p, X, b, h, A = c1
    hm = afn.afn_setup(dev(X), p.l, p.mu, k=p.k, w=p.w, precision=afn.AFN_FP32)
    x, info = afn.afn_pcg_solve(hm, dev(b), tol=1e-12, maxit=p.maxit)
    say("C1 mixed", info)
    assert info["converged"] and info["outer_iterations"] >= 2
    xg = x.cpu().numpy()
    r = b - oracle.kernel_matvec(X, p.l, p.mu, xg)
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 2e-12
    xo, *_ = oracle.pcg(A, b, 1e-12, p.maxit)
    rel = np.linalg.norm(xg - xo) / np.linalg.norm(xo)
    say("C1 mixed vs FP64 oracle:", rel)
    assert rel <= 1e-6
    # the same factors drive the FP64 path
    np.testing.assert_array_equal(hm.landmarks(), h.landmarks())


def test_mixed_c2_shape_reaches_tolerance(afn):
    p = W.c2(0.1)
    X, b = W.make(p)
    Xt, bt = dev(X), dev(b)
    hm = afn.afn_setup(Xt, p.l, p.mu, k=p.k, w=p.w, precision=afn.AFN_FP32)
    x, info = afn.afn_pcg_solve(hm, bt, tol=1e-6, maxit=500)
    say("C2 mixed", info)
    assert info["converged"] and info["relres_true"] <= 1e-6
    r = bt - afn.kernel_matvec(Xt, p.l, p.mu, x)          # FP64 matvec (parity-tested above)
    assert (torch.linalg.norm(r) / torch.linalg.norm(bt)).item() <= 1.01e-6


def test_mixed_reports_failure_instead_of_wrong_answer(afn):
    # mu far below the FP32 operator's rounding: the rounded operator is not
    # positive definite and refinement cannot converge; the solve must end
    # with a failure status (breakdown, stagnation or no convergence), never
    # with a converged flag on a wrong answer
    n = 2000
    X = W.points("uniform", n, 3, 51)
    b = np.random.default_rng(52).standard_normal(n)
    h = afn.afn_setup(dev(X), 0.5, 1e-12, k=50, w=16, precision=afn.AFN_FP32)
    try:
        x, info = afn.afn_pcg_solve(h, dev(b), tol=1e-10, maxit=100)
    except afn.AFNError as e:
        say("mixed ill-conditioned:", e)
        assert e.status in (afn.AFN_EBREAKDOWN, afn.AFN_ESTAGNATION, afn.AFN_ENOCONV)
        return
    say("mixed ill-conditioned", info)
    if info["converged"]:
        r = b - oracle.kernel_matvec(X, 0.5, 1e-12, x.cpu().numpy())
        assert np.linalg.norm(r) <= 2e-10 * np.linalg.norm(b)
    else:
        assert info["status"] in (afn.AFN_ESTAGNATION, afn.AFN_ENOCONV)


# ------------------------------------------------------------------ many right-hand sides (MFMA tiles, block PCG)

@pytest.mark.parametrize("n,d,nrhs,prec", [(1037, 3, 16, 0), (900, 8, 64, 0), (1111, 3, 70, 0),
                                           (1037, 3, 64, 1), (700, 8, 5, 1)])
def test_kernel_matvec_many_rhs_mfma(afn, n, d, nrhs, prec):
    say(f"kmv mrhs n={n} d={d} nrhs={nrhs} prec={prec}")
    X = W.points("uniform" if d == 3 else "normal", n, d, 61)
    l = 0.15 if d == 3 else 2.0
    V = np.random.default_rng(62).standard_normal((n, nrhs))
    Vt = torch.tensor(V.T.copy(), device="cuda").t()            # column-major (n, nrhs)
    Y = afn.kernel_matvec(dev(X), l, 1e-3, Vt, precision=prec).cpu().numpy()
    for c in sorted({0, 1, nrhs // 2, nrhs - 1}):
        yo, ab = oracle.kernel_matvec_rows(X, l, 1e-3, V[:, c], np.arange(n))
        if prec == 0:
            bound = 2 * (n + 4) * U * ab
        else:
            bound = (30 * (d + 4) * math.log(2) + n + 8) * U32 * ab + 1e-13 * np.abs(V[:, c]).sum()
        assert np.all(np.abs(Y[:, c] - yo) <= bound), (c, np.max(np.abs(Y[:, c] - yo) / ab))


@pytest.fixture(scope="module")
def block_case(afn):
    n, R = 2000, 8
    X = W.points("uniform", n, 3, 71)
    B = np.random.default_rng(72).standard_normal((n, R))
    l, mu, k, w = 0.1, 1e-4, 200, 32
    h = afn.afn_setup(dev(X), l, mu, k=k, w=w, precision=afn.AFN_FP32)
    return X, B, l, mu, k, w, h


def _block_solve(afn, h, B, tol):
    Bt = torch.tensor(B.T.copy(), device="cuda").t()
    return afn.afn_pcg_solve(h, Bt, tol=tol, maxit=500)


def test_block_solve_matches_oracle_per_column(afn, block_case):
    X, B, l, mu, k, w, h = block_case
    x, info = _block_solve(afn, h, B, 1e-10)
    say("block", info)
    assert info["converged"] and info["outer_iterations"] >= 2
    x = x.cpu().numpy()
    idx, _ = oracle.fps(X, k)
    A = oracle.afn_build(X, l, mu, idx, w)
    for c in (0, 3, 7):
        r = B[:, c] - oracle.kernel_matvec(X, l, mu, x[:, c])
        assert np.linalg.norm(r) / np.linalg.norm(B[:, c]) <= 2e-10
        xo, *_ = oracle.pcg(A, B[:, c], 1e-10, 500)
        rel = np.linalg.norm(x[:, c] - xo) / np.linalg.norm(xo)
        say(f"column {c}: vs FP64 oracle {rel:.2e}")
        assert rel <= 1e-6


def test_block_solve_graph_replays_equal_eager(afn, block_case, monkeypatch):
    X, B, l, mu, k, w, h = block_case
    xg, ig = _block_solve(afn, h, B, 1e-8)
    monkeypatch.setenv("AFN_NO_GRAPH", "1")
    xe, ie = _block_solve(afn, h, B, 1e-8)
    monkeypatch.delenv("AFN_NO_GRAPH")
    xg2, ig2 = _block_solve(afn, h, B, 1e-8)
    say("graph", ig, "eager", ie)
    assert ig["iterations"] == ie["iterations"] and ig["outer_iterations"] == ie["outer_iterations"]
    assert torch.equal(xg, xe) and torch.equal(xg, xg2)


def test_block_solve_column_equals_single_solve(afn, block_case):
    X, B, l, mu, k, w, h = block_case
    xb, _ = _block_solve(afn, h, B, 1e-10)
    xs, _ = afn.afn_pcg_solve(h, dev(B[:, 5]), tol=1e-10, maxit=500)
    rel = (torch.linalg.norm(xb[:, 5] - xs) / torch.linalg.norm(xs)).item()
    say("block column vs single solve", rel)
    assert rel <= 1e-6


@pytest.fixture(scope="module")
def wide_block_case(afn):
    n = 2000
    X = W.points("uniform", n, 3, 73)
    B = np.random.default_rng(74).standard_normal((n, 70))
    l, mu, k, w = 0.1, 1e-4, 200, 32
    h = afn.afn_setup(dev(X), l, mu, k=k, w=w, precision=afn.AFN_FP32)
    idx, _ = oracle.fps(X, k)
    A = oracle.afn_build(X, l, mu, idx, w)
    return X, B, l, mu, h, A


@pytest.mark.parametrize("R", [64, 70])
def test_block_solve_wide_matches_oracle(afn, wide_block_case, R):
    """64 columns (one full block, graph-captured) and 70 (a full block plus
    a 6-column chunk): sampled columns against the FP64 oracle's solve at
    matching residual, every column's true residual below tol."""
    X, B, l, mu, h, A = wide_block_case
    tol = 1e-10
    x, info = _block_solve(afn, h, B[:, :R], tol)
    say(f"block R={R}", info)
    assert info["converged"] and info["status"] == afn.AFN_OK
    x = x.cpu().numpy()
    for c in range(R):
        r = B[:, c] - oracle.kernel_matvec(X, l, mu, x[:, c])
        assert np.linalg.norm(r) / np.linalg.norm(B[:, c]) <= 2 * tol, c
    for c in sorted({0, 31, 63, R - 1}):
        xo, *_ = oracle.pcg(A, B[:, c], tol, 500)
        rel = np.linalg.norm(x[:, c] - xo) / np.linalg.norm(xo)
        say(f"R={R} column {c}: vs FP64 oracle {rel:.2e}")
        assert rel <= 1e-6


def test_block_solve_nan_column_in_second_chunk(afn, wide_block_case):
    """A non-finite right-hand side in the second 64-column chunk: the call
    reports EBREAKDOWN, and every other column is still solved to tol."""
    X, B, l, mu, h, A = wide_block_case
    tol = 1e-8
    Bn = B.copy()
    Bn[5, 66] = np.nan
    Bt = torch.tensor(Bn.T.copy(), device="cuda").t()
    out = torch.full((70, Bn.shape[0]), 7.0, dtype=torch.float64, device="cuda").t()
    with pytest.raises(afn.AFNError) as e:
        afn.afn_pcg_solve(h, Bt, tol=tol, maxit=500, out=out)
    assert e.value.status == afn.AFN_EBREAKDOWN
    x = out.cpu().numpy()
    for c in range(70):
        if c == 66:
            continue
        r = Bn[:, c] - oracle.kernel_matvec(X, l, mu, x[:, c])
        assert np.linalg.norm(r) / np.linalg.norm(Bn[:, c]) <= 2 * tol, c


# ------------------------------------------------------------------ mixed precision: FP64 fallback

@pytest.mark.parametrize("n,l,mu,k,tol", [(4000, 0.5, 1e-8, 200, 1e-6), (2000, 0.3, 1e-6, 100, 1e-10),
                                          (3000, 1.0, 1e-6, 150, 1e-8)])
def test_mixed_falls_back_to_fp64(afn, n, l, mu, k, tol):
    """Where the FP32 corrections break down or stop reducing the residual,
    the mixed solve finishes with FP64 PCG and ends no worse than the FP64
    solve of the same system (same status; true residual within 10x)."""
    X = W.points("uniform", n, 3, 61)
    b = np.random.default_rng(62).standard_normal(n)
    res = {}
    for prec in (afn.AFN_FP32, afn.AFN_FP64):
        h = afn.afn_setup(dev(X), l, mu, k=k, w=32, precision=prec)
        x, info = afn.afn_pcg_solve(h, dev(b), tol=tol, maxit=400)
        h.close()
        xh = x.cpu().numpy()
        y, ab = oracle.kernel_matvec_rows(X, l, mu, xh, np.arange(n))
        r = b - y
        # rounding floor of any FP64 evaluation of ||b - A x|| / ||b||
        floor = 2 * (n + 4) * U * np.linalg.norm(ab) / np.linalg.norm(b)
        res[prec] = (info, np.linalg.norm(r) / np.linalg.norm(b), floor)
        say(f"fallback n={n} l={l} mu={mu} prec={prec}", info, res[prec][1:])
    (i32, t32, f32), (i64, t64, f64) = res[afn.AFN_FP32], res[afn.AFN_FP64]
    assert i32["fp64_iterations"] > 0
    assert i32["status"] == i64["status"]
    assert t32 <= max(10.0 * t64, tol)
    assert abs(i32["relres_true"] - t32) <= 1e-3 * t32 + f32


def test_pruned_pair_fraction(afn):
    # a short length-scale leaves few tile pairs above 2^-64; a long one keeps all
    X = dev(W.points("uniform", 20000, 3, 91))
    h = afn.afn_setup(X, 0.01, 1e-3, k=50, w=8)
    inf = h.info()
    h.close()
    say("kept fractions l=0.01", inf.kmv_kept_f64, inf.kmv_kept_f32, "far", inf.kmv_far_f64)
    assert 0.0 < inf.kmv_kept_f32 <= inf.kmv_kept_f64 < 0.2
    # pairs between the 2^-46 and 2^-64 cuts: FP32 exponential in the FP64 kernel
    assert 0.0 < inf.kmv_far_f64 < inf.kmv_kept_f64
    h = afn.afn_setup(X, 10.0, 1e-3, k=50, w=8)
    inf = h.info()
    h.close()
    assert inf.kmv_kept_f64 == 1.0 and inf.kmv_kept_f32 == 1.0 and inf.kmv_far_f64 == 0.0
    # d > 4: the plain tile kernel, no FP32 exponential
    h = afn.afn_setup(dev(W.points("uniform", 20000, 6, 92)), 0.05, 1e-3, k=50, w=8)
    inf = h.info()
    h.close()
    assert inf.kmv_far_f64 == 0.0


@pytest.mark.parametrize("n,d,k,lm", [(3000, 22, 300, 0), (1500, 18, 150, 0), (800, 3, 64, 2)])
def test_uniform_landmarks_match_oracle(afn, n, d, k, lm):
    # Algorithm 2: above d = 10 the landmarks are a uniform sample (the first k
    # entries of the splitmix64 Fisher-Yates shuffle, seed + 1); the rest of
    # the construction is the same as with FPS landmarks
    X = W.points("normal", n, d, 92)
    l, mu, w, seed = 3.0, 1e-2, 16, 5
    h = afn.afn_setup(dev(X), l, mu, k=k, w=w, seed=seed, landmarks=lm)
    inf = h.info()
    idx = oracle.subsample(n, k, seed + 1)
    assert inf.landmarks == afn.AFN_LANDMARKS_UNIFORM
    np.testing.assert_array_equal(h.landmarks(), idx)
    A = oracle.afn_build(X, l, mu, idx, w)
    rowptr, cols, vals = h.fsai()
    np.testing.assert_array_equal(rowptr, A.rowptr)
    np.testing.assert_array_equal(cols, A.cols)
    r = np.random.default_rng(93).standard_normal(n)
    s_ = afn.afn_apply(h, dev(r)).cpu().numpy()
    so = oracle.afn_apply(A, r)
    # entry by entry, landmark and non-landmark entries each at their own scale
    lm = np.zeros(n, dtype=bool)
    lm[A.perm[:A.k]] = True
    for m in (lm, ~lm):
        assert np.max(np.abs(s_[m] - so[m])) <= 1e-8 * np.max(np.abs(so[m]))
    x, info = afn.afn_pcg_solve(h, dev(r), tol=1e-8, maxit=500)
    h.close()
    res = r - oracle.kernel_matvec(X, l, mu, x.cpu().numpy())
    assert info["status"] == afn.AFN_OK and np.linalg.norm(res) <= 2e-8 * np.linalg.norm(r)


@pytest.mark.parametrize("n,k", [(4097, 4096), (1000, 999), (5000, 1), (70000, 4096), (3, 2)])
def test_uniform_landmark_order_edges(afn, n, k):
    # The uniform landmarks are a partial Fisher-Yates prefix, formed with all
    # draws and swaps in parallel (steps sorted by partner, chains of earlier
    # swaps resolved by pointer jumping).  With k near n nearly every step
    # meets an earlier swap; k = 4096 is the largest prefix.
    X = W.points("uniform", n, 3, 95)
    say(f"uniform landmarks n={n} k={k}")
    h = afn.afn_setup(dev(X), 0.3, 1e-2, k=k, w=4, seed=11, landmarks=afn.AFN_LANDMARKS_UNIFORM)
    got = h.landmarks()
    h.close()
    np.testing.assert_array_equal(got, oracle.subsample(n, k, 12))


def test_uniform_landmarks_limit(afn):
    X = dev(W.points("normal", 5000, 12, 94))
    with pytest.raises(afn.AFNError) as e:
        afn.afn_setup(X, 3.0, 1e-2, k=4097, w=8)
    assert e.value.status == afn.AFN_EINVAL



@pytest.mark.parametrize("n,d,k,w", [(3000, 3, 200, 32), (2500, 12, 150, 64), (4000, 12, 512, 16),
                                     (3000, 12, 200, 100)])
def test_fsai_recompute_equals_gather(afn, monkeypatch, n, d, k, w):
    # the batched mode recomputes each pattern's columns of L^{-1} K12 as a
    # product with L^{-1} (MFMA GEMM), the gather mode reads them from
    # V = L^{-1} K12 (triangular solve): same pattern, values equal to within
    # the rounding of the two products
    X = dev(W.points("uniform", n, d, 95))
    out = []
    for mode in ("0", "1"):
        monkeypatch.setenv("AFN_FSAI_RECOMPUTE", mode)
        h = afn.afn_setup(X, 0.4, 1e-3, k=k, w=w, landmarks=afn.AFN_LANDMARKS_FPS)
        out.append(h.fsai())
        h.close()
    np.testing.assert_array_equal(out[0][0], out[1][0])
    np.testing.assert_array_equal(out[0][1], out[1][1])
    rel = np.linalg.norm(out[0][2] - out[1][2]) / np.linalg.norm(out[0][2])
    say(f"recompute vs gather n={n} d={d} k={k}: rel {rel:.2e}")
    assert rel <= 1e-8
