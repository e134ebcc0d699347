"""Pins for the oracle's kernel, matvec and farthest point sampling.

Each check is tied to something other than the oracle itself: closed forms of
Eq. (1.2), the separability of the Gaussian kernel over coordinates, hand-derived
FPS worked examples (Algorithm 6), a brute-force recomputation of the FPS
definition (Section 4: x_{i+1} = argmax over X minus X_i of dist(x, X_i)), and
the properties of Theorems 4.1 and 4.3.
"""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.filterwarnings("ignore")


# --------------------------------------------------------------------------- kernel

def test_kernel_closed_form_has_no_half_factor():
    # Eq. (1.2): K(x,y) = exp(-|x-y|^2 / l^2); at distance l the value is e^-1
    # (a kernel with exp(-r^2/(2 l^2)) would give e^-1/2).
    l = 0.37
    for dist, expect in [(l, math.exp(-1.0)), (2 * l, math.exp(-4.0)), (0.0, 1.0)]:
        a = np.array([0.25])
        b = np.array([0.25 + dist])
        assert oracle.kernel(a, b, l) == pytest.approx(expect, rel=1e-15)


def test_sqdist_exact_on_integers_and_symmetric_bitwise():
    rng = np.random.default_rng(0)
    for d in (1, 3, 8):
        a = rng.integers(-50, 50, size=d).astype(float)
        b = rng.integers(-50, 50, size=d).astype(float)
        assert oracle.sqdist(a, b) == float(np.sum((a - b) ** 2))
    for _ in range(200):
        a = rng.standard_normal(8)
        b = rng.standard_normal(8)
        assert oracle.sqdist(a, b) == oracle.sqdist(b, a)


def test_matvec_two_points_closed_form():
    X = np.array([[0.0, 0.0], [0.3, 0.4]])           # distance 0.5
    l, mu = 0.5, 1e-3
    v = np.array([2.0, -3.0])
    k01 = math.exp(-1.0)
    y = oracle.kernel_matvec(X, l, mu, v)
    assert y[0] == pytest.approx((1 + mu) * 2.0 + k01 * -3.0, rel=1e-14)
    assert y[1] == pytest.approx(k01 * 2.0 + (1 + mu) * -3.0, rel=1e-14)


def test_matvec_tensor_grid_separability():
    # On a tensor grid the Gaussian kernel matrix is the Kronecker product of
    # the 1-D kernel matrices of each axis, so K (v1 x v2 x v3) factorizes.
    # A dropped coordinate, a wrong stride or a transposed index breaks this.
    ax = [np.array([0.0, 0.1, 0.35, 0.5]), np.array([0.0, 0.2, 0.25, 0.7, 0.9]),
          np.array([0.1, 0.15, 0.6])]
    l, mu = 0.3, 0.0
    X = np.array(list(itertools.product(*ax)))           # last axis fastest
    rng = np.random.default_rng(1)
    vs = [rng.standard_normal(a.size) for a in ax]
    v = np.einsum("i,j,k->ijk", *vs).ravel()
    y = oracle.kernel_matvec(X, l, mu, v)
    Ks = [np.exp(-np.subtract.outer(a, a) ** 2 / l**2) for a in ax]
    expect = np.einsum("i,j,k->ijk", *[K @ u for K, u in zip(Ks, vs)]).ravel()
    np.testing.assert_allclose(y, expect, rtol=1e-12, atol=1e-14)


def test_matvec_unit_vectors_give_symmetric_columns_with_unit_diagonal():
    rng = np.random.default_rng(2)
    X = rng.random((40, 3))
    l, mu = 0.4, 1e-2
    cols = [oracle.kernel_matvec(X, l, mu, np.eye(40)[j]) for j in (3, 17)]
    assert cols[0][3] == pytest.approx(1.0 + mu, rel=1e-15)       # K_jj = 1
    assert cols[1][17] == pytest.approx(1.0 + mu, rel=1e-15)
    assert cols[0][17] == cols[1][3]                             # K symmetric


def test_matvec_bilinear_symmetry_and_multi_rhs():
    rng = np.random.default_rng(3)
    X = rng.random((150, 3))
    l, mu = 0.2, 1e-4
    U = rng.standard_normal((150, 3))
    Y = oracle.kernel_matvec(X, l, mu, U)
    for j in range(3):
        np.testing.assert_array_equal(Y[:, j], oracle.kernel_matvec(X, l, mu, U[:, j]))
    assert U[:, 0] @ Y[:, 1] == pytest.approx(U[:, 1] @ Y[:, 0], rel=1e-12)
    rows = np.array([0, 7, 149])
    yr, ar = oracle.kernel_matvec_rows(X, l, mu, U[:, 0], rows)
    np.testing.assert_allclose(yr, Y[rows, 0], rtol=1e-13, atol=1e-15)
    assert np.all(ar >= np.abs(yr) - 1e-15)


# --------------------------------------------------------------------------- FPS

def _read_golden(path):
    rows, pts = [], None
    for line in path.read_text().splitlines():
        if not line.strip() or line.startswith("#"):
            continue
        if line.startswith("points"):
            pts = [tuple(float(c) for c in tok.split(",")) for tok in line.split()[1:]]
            continue
        i, j, dist = line.split()
        rows.append((int(i), int(j), float(dist)))
    return np.array(pts, dtype=float), rows


@pytest.mark.parametrize("name", ["fps_collinear.txt", "fps_square.txt"])
def test_fps_golden_worked_examples(golden_dir, name):
    X, rows = _read_golden(golden_dir / name)
    idx, seld = oracle.fps(X, len(rows))
    assert list(idx) == [j for _, j, _ in rows]
    assert math.isinf(seld[0])
    np.testing.assert_array_equal(seld[1:], [dd for _, _, dd in rows[1:]])


def _fps_bruteforce(X, k):
    """FPS by its definition: first = nearest to the mean (exact rational mean
    for integer data), then argmax over unselected of min squared distance to
    the selected set; ties to the smallest index.  O(k^2 n)."""
    n = X.shape[0]
    cen = [Fraction(int(s)) / n for s in X.sum(axis=0)]
    dc = [sum((Fraction(int(X[j, t])) - cen[t]) ** 2 for t in range(X.shape[1])) for j in range(n)]
    sel = [int(min(range(n), key=lambda j: (dc[j], j)))]
    D = ((X[:, None, :] - X[None, :, :]) ** 2).sum(-1)
    while len(sel) < k:
        rest = [j for j in range(n) if j not in sel]
        score = {j: min(D[j, s] for s in sel) for j in rest}
        sel.append(max(rest, key=lambda j: (score[j], -j)))
    return sel


@pytest.mark.parametrize("seed,d", [(0, 1), (1, 2), (2, 3), (3, 3), (4, 5)])
def test_fps_matches_bruteforce_on_integer_points_with_ties(seed, d):
    rng = np.random.default_rng(seed)
    X = rng.integers(0, 6, size=(60, d)).astype(float)    # many exact ties
    k = 25
    idx, _ = oracle.fps(X, k)
    assert list(idx) == _fps_bruteforce(X, k)


def test_fps_duplicates_never_reselect():
    X = np.tile(np.array([[0.5, 0.5, 0.5]]), (9, 1))
    X[4] = [0.9, 0.1, 0.5]
    idx, seld = oracle.fps(X, 9)
    assert sorted(idx) == list(range(9))
    # centroid is nearest the 8 duplicates -> index 0; then the odd one out;
    # then the remaining duplicates (distance 0) in ascending index order.
    assert list(idx) == [0, 4, 1, 2, 3, 5, 6, 7, 8]


def test_centroid_is_exact_mean_for_integer_coordinates():
    rng = np.random.default_rng(5)
    X = rng.integers(0, 1000, size=(1000, 3)).astype(float)
    c = oracle.centroid(X)
    for t in range(3):
        assert c[t] == float(Fraction(int(X[:, t].sum()), 1000))


def _fill_sep(X, idx):
    D = np.sqrt(((X[:, None, :] - X[None, :, :]) ** 2).sum(-1))
    h = D[:, idx].min(axis=1).max()
    sub = D[np.ix_(idx, idx)] + np.diag(np.full(len(idx), np.inf))
    q = sub.min()
    return h, q


def test_fps_theorem_4_3_fill_below_separation_and_monotone():
    rng = np.random.default_rng(6)
    X = rng.random((300, 3))
    idx, seld = oracle.fps(X, 120)
    assert np.all(np.diff(seld[1:]) <= 0)                  # max-min sequence non-increasing
    for k in (2, 5, 17, 60, 120):
        h, q = _fill_sep(X, idx[:k])
        assert h <= q + 1e-15                               # Theorem 4.3: h <= q
        if k < 120:   # the next selection distance is the fill distance of X_k
            assert h == pytest.approx(math.sqrt(seld[k]), rel=1e-14)


def test_fps_theorem_4_3_near_optimality_exhaustive():
    # For n <= 12, compare with the best subsets found by exhaustive search.
    rng = np.random.default_rng(7)
    for trial in range(6):
        X = rng.random((11, 2))
        for k in (2, 3, 4, 5):
            idx, _ = oracle.fps(X, k)
            h, q = _fill_sep(X, list(idx))
            hs, qs = [], []
            for S in itertools.combinations(range(11), k):
                hh, qq = _fill_sep(X, list(S))
                hs.append(hh)
                qs.append(qq)
            assert q >= 0.5 * max(qs) - 1e-12
            assert h <= 2.0 * min(hs) + 1e-12


def test_fps_theorem_4_1_packing_bound_in_unit_ball():
    rng = np.random.default_rng(8)
    for d in (2, 3):
        Z = rng.standard_normal((2000, d))
        Z *= (rng.random((2000, 1)) ** (1.0 / d)) / np.linalg.norm(Z, axis=1, keepdims=True)
        idx, _ = oracle.fps(Z, 200)
        for k in (10, 50, 200):
            _, q = _fill_sep(Z, idx[:k])
            assert q <= 6.0 * k ** (-1.0 / d)


def test_permutation_is_landmarks_then_ascending_rest():
    perm = oracle.permutation(8, [5, 2, 7])
    assert list(perm) == [5, 2, 7, 0, 1, 3, 4, 6]
    with pytest.raises(oracle.OracleError):
        oracle.permutation(8, [5, 5])
