"""A seeded sweep of kernel-matvec configurations through the C-ABI against
the oracle on sampled rows: sizes on both sides of the size from which the
matvec prunes tile pairs (n = 8192), d from 1 to 12, length scales from tiles
much wider than l to tiles much narrower, both precisions and both kernels,
one and several columns.

Bound per row i (u the unit roundoff of the precision, ab_i = sum_j |K_ij v_j|
+ mu |v_i|), each term's relative error being at most r u:
  FP64   (2 (n + 4) + r) u ab_i + 2^-64 sum_j |v_j|
  FP32   (n + 8 + r) u ab_i + (1e-13 + 2^-44) sum_j |v_j|
The last terms cover the skipped tile pairs (every value there is below 2^-64,
resp. 2^-44) and the FP64 pairs whose value is taken in FP32 (below 2^-46).
r has three parts (c the coordinate scale of the kind, xm the largest
spread max - min of a coordinate):
  - the stored coordinates (x - x0) c (1 + e), |e| <= 2 u, relative to an
    origin x0 whose every coordinate is one of the data's: each coordinate difference is off by at most 4 xm c u, so
    t by 2 sqrt(t d) 4 xm c u; the Gaussian 2^(-t) moves by ln 2 dt relative
    (t <= 64), the Matern value by at most ln 2 ds with ds <= 4 sqrt(d) xm c u;
  - t itself, direct or from norms and dot products of centred coordinates
    (centred radius^2 <= 16): 64 (d + 4) u absolute for the Gaussian, s (d + 4) / 2
    relative in s for the Matern kernel (s <= 66 in FP64, 50 in FP32);
  - the exponential and the Matern factor: 8."""
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


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def term_rel(kernel, fp64, d, xm, l):
    if kernel == 0:
        c = math.sqrt(LOG2E) / l
        return LN2 * (64 * (d + 4) + 8 * math.sqrt(64 * d) * xm * c) + 8
    c = math.sqrt(3.0) * LOG2E / l
    smax = 66 if fp64 else 50
    return LN2 * (smax * (d + 4) / 2 + 4 * math.sqrt(d) * xm * c) + 8


def spread(X):
    return float((X.max(0) - X.min(0)).max())


def cases():
    rng = np.random.default_rng(2024)
    out = []
    for i in range(24):
        n = int(rng.choice([3000, 9000, 24000]))
        d = int(rng.choice([1, 2, 3, 3, 4, 6, 8, 12]))
        kinds = ["uniform", "normal", "mixture5"] if d == 3 else ["uniform", "normal"]
        pts = str(rng.choice(kinds))
        scale = 3.0 if pts == "normal" else 1.0
        l = float(scale * 10 ** rng.uniform(-2.3, 0.3))
        kernel = int(rng.integers(0, 2))
        nrhs = int(rng.choice([1, 1, 3, 16]))
        out.append((i, n, d, pts, l, kernel, nrhs))
    return out


@pytest.mark.parametrize("i,n,d,pts,l,kernel,nrhs", cases())
def test_matvec_sweep(afn, i, n, d, pts, l, kernel, nrhs):
    print(f"sweep {i}: n={n} d={d} {pts} l={l:.3g} kernel={kernel} nrhs={nrhs}", flush=True)
    X = W.points(pts, n, d, 3000 + i)
    V = np.random.default_rng(4000 + i).standard_normal((n, nrhs))
    rows = np.concatenate([np.arange(3), np.random.default_rng(5000 + i).integers(0, n, 25), [n - 1]])
    Vd = torch.tensor(V.T.copy(), device="cuda").t()
    with oracle.use_kernel("matern32" if kernel else "gaussian"):
        ref = [oracle.kernel_matvec_rows(X, l, 1e-3, V[:, c], rows) for c in range(nrhs)]
    xm = spread(X)
    for prec in (afn.AFN_FP64, afn.AFN_FP32):
        Y = afn.kernel_matvec(dev(X), l, 1e-3, Vd, precision=prec, kernel=kernel).cpu().numpy()
        fp64 = prec == afn.AFN_FP64
        r = term_rel(kernel, fp64, d, xm, l)
        worst = 0.0
        for c in range(nrhs):
            yo, ab = ref[c]
            vs = np.abs(V[:, c]).sum()
            if fp64:
                bound = (2 * (n + 4) + r) * U * ab + 2.0 ** -64 * vs
            else:
                bound = (n + 8 + r) * U32 * ab + (1e-13 + 2.0 ** -44) * vs
            err = np.abs(Y[rows, c] - yo)
            worst = max(worst, float(np.max(err / bound)))
            assert np.all(err <= bound), (prec, c, float(np.max(err / bound)))
        print(f"  prec={prec}: worst err/bound {worst:.3f}", flush=True)


@pytest.mark.parametrize("kernel", [0, 1])
@pytest.mark.parametrize("n", [5000, 20000])
def test_matvec_far_from_origin(afn, kernel, n):
    """Points far from the origin.  The packed coordinates are relative to a
    median of the data, so the FP32 copies keep their precision (absolute coordinates
    of 3e4 at l = 0.05 would put a few percent of error into every kernel
    value), and the padding points of the last, partly filled tile must not
    break the FP64 kernel's choice of exponential."""
    d, l = 3, 0.05
    print(f"far from origin: n={n} kernel={kernel}", flush=True)
    X = W.points("mixture5", n, d, 77) + np.array([1.0e4, -3.0e4, 2.0e4])
    V = np.random.default_rng(78).standard_normal((n, 1))
    rows = np.concatenate([np.arange(3), np.random.default_rng(79).integers(0, n, 25), [n - 1]])
    with oracle.use_kernel("matern32" if kernel else "gaussian"):
        yo, ab = oracle.kernel_matvec_rows(X, l, 1e-3, V[:, 0], rows)
    for prec in (afn.AFN_FP64, afn.AFN_FP32):
        Y = afn.kernel_matvec(dev(X), l, 1e-3, dev(V), precision=prec, kernel=kernel).cpu().numpy()
        assert np.all(np.isfinite(Y))
        err = np.abs(Y[rows, 0] - yo)
        vs = np.abs(V[:, 0]).sum()
        fp64 = prec == afn.AFN_FP64
        # packed relative to a data point: the spread, not the offset,
        # sets the storage error, in both precisions
        r = term_rel(kernel, fp64, d, spread(X), l)
        if fp64:
            bound = (2 * (n + 4) + r) * U * ab + 2.0 ** -64 * vs
        else:
            bound = (n + 8 + r) * U32 * ab + (1e-13 + 2.0 ** -44) * vs
        print(f"  prec={prec}: worst err/bound {float(np.max(err / bound)):.3f}", flush=True)
        assert np.all(err <= bound)


@pytest.mark.parametrize("kernel", [0, 1])
def test_matvec_outliers(afn, kernel):
    """A mixture with 300 points moved 1e2 .. 1e6 away.  Tiles that hold both
    bulk points and outliers have boxes too wide for the FP64 kernel's
    table-driven exponential (their pairs take the clamped one), and the
    origin of the packed coordinates (a median) stays inside the bulk."""
    n, d, l = 20000, 3, 0.05
    rng = np.random.default_rng(91)
    X = W.points("mixture5", n, d, 90)
    out = rng.choice(n, 300, replace=False)
    dirs = rng.standard_normal((300, d))
    X[out] += dirs / np.linalg.norm(dirs, axis=1, keepdims=True) * 10.0 ** rng.uniform(2, 6, (300, 1))
    bulk = np.setdiff1d(np.arange(n), out)
    V = rng.standard_normal(n)
    rows = np.concatenate([rng.choice(bulk, 25, replace=False), out[:10]])
    print(f"outliers: kernel={kernel}", flush=True)
    with oracle.use_kernel("matern32" if kernel else "gaussian"):
        yo, ab = oracle.kernel_matvec_rows(X, l, 1e-3, V, rows)
    vs = np.abs(V).sum()
    xm = np.where(np.isin(rows, out), spread(X), spread(X[bulk]))
    for prec in (afn.AFN_FP64, afn.AFN_FP32):
        Y = afn.kernel_matvec(dev(X), l, 1e-3, dev(V[:, None]), precision=prec, kernel=kernel).cpu().numpy()
        assert np.all(np.isfinite(Y))
        fp64 = prec == afn.AFN_FP64
        r = np.array([term_rel(kernel, fp64, d, x, l) for x in xm])
        if fp64:
            bound = (2 * (n + 4) + r) * U * ab + 2.0 ** -64 * vs
        else:
            bound = (n + 8 + r) * U32 * ab + (1e-13 + 2.0 ** -44) * vs
        err = np.abs(Y[rows, 0] - yo)
        print(f"  prec={prec}: worst err/bound {float(np.max(err / bound)):.3f}", flush=True)
        assert np.all(err <= bound)
