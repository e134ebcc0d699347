"""Plain FP64 CPU oracle for AFN-preconditioned CG (arXiv 2304.05460).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code
with the GPU library: the AFN arithmetic lives in ``afn_oracle.c`` (plain C,
FP64, ``-ffp-contract=off``, OpenMP ``parallel for`` over independent outputs
only) and this module only marshals numpy arrays through ctypes; the Nystrom
branch of Algorithm 5 is plain numpy in ``nystrom.py``.

Every wrapper names the passage of the paper its C function follows.
"""
from __future__ import annotations

import ctypes
import os
import pathlib
import subprocess

import numpy as np

_DIR = pathlib.Path(__file__).resolve().parent
_SRC = _DIR / "afn_oracle.c"
_LIB = _DIR / "liboracle.so"
_lib = None

ORA_OK, ORA_EINVAL, ORA_ENOMEM, ORA_ENOTSPD, ORA_ENOCONV, ORA_EBREAKDOWN = range(6)


class OracleError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"oracle {where} failed with status {status}")
        self.status = status


def build() -> pathlib.Path:
    """Compile liboracle.so with gcc (always recompiles)."""
    tmp = _LIB.with_suffix(".so.tmp")
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
           "-Wall", "-o", str(tmp), str(_SRC), "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not _LIB.exists():
            build()
        _lib = ctypes.CDLL(str(_LIB))
        _declare(_lib)
    return _lib


_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I = ctypes.c_int
_D = ctypes.c_double


def _declare(L):
    L.ora_sqdist.argtypes = [_P, _P, _I]
    L.ora_sqdist.restype = _D
    L.ora_kernel.argtypes = [_P, _P, _I, _D]
    L.ora_kernel.restype = _D
    L.ora_kernel_matvec.argtypes = [_P, _I64, _I, _D, _D, _P, _I64, _P]
    L.ora_kernel_matvec_rows.argtypes = [_P, _I64, _I, _D, _D, _P, _P, _I64, _P, _P]
    L.ora_centroid.argtypes = [_P, _I64, _I, _P]
    L.ora_fps.argtypes = [_P, _I64, _I, _I64, _P, _P]
    L.ora_permutation.argtypes = [_I64, _I64, _P, _P]
    L.ora_cholesky.argtypes = [_P, _I64, _I64]
    L.ora_fwd_subst.argtypes = [_P, _I64, _P, _P]
    L.ora_bwd_subst.argtypes = [_P, _I64, _P, _P]
    L.ora_knn_pattern.argtypes = [_P, _I64, _I, _I64, _P, _P]
    L.ora_knn_rows.argtypes = [_P, _I64, _I, _I64, _P, _I64, _P, _P]
    L.ora_landmark_cholesky.argtypes = [_P, _I64, _I, _D, _D, _P]
    L.ora_afn_build.argtypes = [_P, _I64, _I, _D, _D, _I64, _P, _I64, _P, _P, _P, _P, _P]
    L.ora_fsai_rows.argtypes = [_P, _I64, _I, _D, _D, _I64, _P, _P, _I64, _P, _I64, _P, _P, _P]
    L.ora_afn_apply.argtypes = [_P, _I64, _I, _D, _I64, _P, _P, _P, _P, _P, _P, _P]
    L.ora_pcg.argtypes = [_P, _I64, _I, _D, _D, _I64, _P, _P, _P, _P, _P, _P, _D, _I64,
                          _P, _P, _P, _P]
    L.ora_splitmix64_stream.argtypes = [ctypes.c_uint64, _I64, _P]
    L.ora_subsample.argtypes = [_I64, _I64, ctypes.c_uint64, _P]
    L.ora_nystrom_scan.argtypes = [_P, _I64, _P, _I64, _D, _D, _P]
    L.ora_nystrom_scan.restype = _I64
    L.ora_count_eigs_above.argtypes = [_P, _I64, _D]
    L.ora_count_eigs_above.restype = _I64
    L.ora_rank_estimate.argtypes = [_P, _I64, _I, _D, _D, _I64, _I64, _I64, ctypes.c_uint64,
                                    _P, _P]
    L.ora_set_kernel.argtypes = [_I]


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(st: int, where: str):
    if st != ORA_OK:
        raise OracleError(st, where)


# --- kernel function and matvec (Eq. (1.1), Eq. (1.2)) -------------------------

KERNELS = {"gaussian": 0, "matern32": 1}


def set_kernel(kind: str) -> None:
    """Kernel of every later oracle call (Section 5): "gaussian" (Eq. (1.2)) or
    "matern32" ((1 + sqrt(3) r / l) exp(-sqrt(3) r / l))."""
    from . import nystrom as _nys
    _check(lib().ora_set_kernel(KERNELS[kind]), "set_kernel")
    _nys.KIND[0] = KERNELS[kind]


class use_kernel:
    """Context manager: set_kernel(kind) inside, Gaussian again on exit."""

    def __init__(self, kind: str):
        self.kind = kind

    def __enter__(self):
        set_kernel(self.kind)
        return self

    def __exit__(self, *exc):
        set_kernel("gaussian")
        return False


def sqdist(a, b) -> float:
    a, b = _f64(a), _f64(b)
    return lib().ora_sqdist(_p(a), _p(b), a.shape[0])


def kernel(a, b, l: float) -> float:
    a, b = _f64(a), _f64(b)
    return lib().ora_kernel(_p(a), _p(b), a.shape[0], l)


def kernel_matvec(X, l: float, mu: float, v) -> np.ndarray:
    """y = (K + mu I) v; v is (n,) or column-major-equivalent (n, nrhs)."""
    X = _f64(X)
    n, d = X.shape
    v = np.asarray(v, dtype=np.float64)
    vec = v.ndim == 1
    V = np.asfortranarray(v.reshape(n, -1))
    Y = np.zeros_like(V, order="F")
    _check(lib().ora_kernel_matvec(_p(X), n, d, l, mu, _p(V), V.shape[1], _p(Y)),
           "kernel_matvec")
    return Y[:, 0].copy() if vec else Y


def kernel_matvec_rows(X, l: float, mu: float, v, rows):
    """Rows of (K + mu I) v and the absolute sums sum_j |K_ij v_j| + mu |v_i|."""
    X, v = _f64(X), _f64(v)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    y = np.zeros(rows.shape[0])
    a = np.zeros(rows.shape[0])
    _check(lib().ora_kernel_matvec_rows(_p(X), X.shape[0], X.shape[1], l, mu, _p(v),
                                        _p(rows), rows.shape[0], _p(y), _p(a)),
           "kernel_matvec_rows")
    return y, a


# --- FPS (Algorithm 6) ---------------------------------------------------------

def centroid(X) -> np.ndarray:
    X = _f64(X)
    c = np.zeros(X.shape[1])
    _check(lib().ora_centroid(_p(X), X.shape[0], X.shape[1], _p(c)), "centroid")
    return c


def fps(X, k: int):
    """Landmark indices in selection order and their squared selection distances."""
    X = _f64(X)
    idx = np.zeros(max(k, 1), dtype=np.int32)
    seld = np.zeros(max(k, 1))
    _check(lib().ora_fps(_p(X), X.shape[0], X.shape[1], k, _p(idx), _p(seld)), "fps")
    return idx[:k].copy(), seld[:k].copy()


def permutation(n: int, idx) -> np.ndarray:
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    perm = np.zeros(n, dtype=np.int32)
    _check(lib().ora_permutation(n, idx.shape[0], _p(idx), _p(perm)), "permutation")
    return perm


# --- dense factorizations --------------------------------------------------------

def cholesky(A) -> np.ndarray:
    """Lower Cholesky factor (textbook, no pivoting); raises OracleError(3) if not SPD."""
    A = np.asfortranarray(np.array(A, dtype=np.float64))
    k = A.shape[0]
    _check(lib().ora_cholesky(_p(A), k, k), "cholesky")
    return A


def fwd_subst(L, b) -> np.ndarray:
    L = np.asfortranarray(L, dtype=np.float64)
    b = _f64(b)
    y = np.zeros_like(b)
    lib().ora_fwd_subst(_p(L), L.shape[0], _p(b), _p(y))
    return y


def bwd_subst(L, y) -> np.ndarray:
    L = np.asfortranarray(L, dtype=np.float64)
    y = _f64(y)
    x = np.zeros_like(y)
    lib().ora_bwd_subst(_p(L), L.shape[0], _p(y), _p(x))
    return x


def landmark_cholesky(Xp, k: int, l: float, mu: float) -> np.ndarray:
    Xp = _f64(Xp)
    L = np.zeros((max(k, 1), max(k, 1)), order="F")
    _check(lib().ora_landmark_cholesky(_p(Xp), k, Xp.shape[1], l, mu, _p(L)), "landmark_cholesky")
    return L[:k, :k].copy(order="F")


# --- FSAI pattern (Section 3.1) ---------------------------------------------------

def knn_pattern(Xr, w: int):
    Xr = _f64(Xr)
    nr = Xr.shape[0]
    rowptr = np.zeros(nr + 1, dtype=np.int64)
    cols = np.zeros(max(nr * w, 1), dtype=np.int32)
    _check(lib().ora_knn_pattern(_p(Xr), nr, Xr.shape[1], w, _p(rowptr), _p(cols)), "knn_pattern")
    return rowptr, cols[: rowptr[-1]].copy()


def knn_rows(Xr, w: int, rows):
    Xr = _f64(Xr)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.zeros((rows.shape[0], w), dtype=np.int32)
    ln = np.zeros(rows.shape[0], dtype=np.int32)
    _check(lib().ora_knn_rows(_p(Xr), Xr.shape[0], Xr.shape[1], w, _p(rows), rows.shape[0],
                              _p(out), _p(ln)), "knn_rows")
    return out, ln


# --- AFN construction / application (Algorithms 1-3) -----------------------------

class AFN:
    """Oracle AFN factors in block order (landmarks first, then X_r ascending)."""

    def __init__(self, X, l, mu, k, w, perm, L, rowptr, cols, gval):
        self.X, self.l, self.mu, self.k, self.w = X, l, mu, k, w
        self.perm, self.L, self.rowptr, self.cols, self.gval = perm, L, rowptr, cols, gval

    @property
    def n(self):
        return self.X.shape[0]

    def G_dense(self) -> np.ndarray:
        nr = self.n - self.k
        G = np.zeros((nr, nr))
        for p in range(nr):
            a, b = self.rowptr[p], self.rowptr[p + 1]
            G[p, self.cols[a:b]] = self.gval[a:b]
        return G


def afn_build(X, l: float, mu: float, idx, w: int) -> AFN:
    """Algorithm 2 on the given landmark indices (FPS order)."""
    X = _f64(X)
    n, d = X.shape
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    k = idx.shape[0]
    nr = n - k
    perm = np.zeros(n, dtype=np.int32)
    L = np.zeros((max(k, 1), max(k, 1)), order="F")
    rowptr = np.zeros(nr + 1, dtype=np.int64)
    cols = np.zeros(max(nr * w, 1), dtype=np.int32)
    gval = np.zeros(max(nr * w, 1))
    _check(lib().ora_afn_build(_p(X), n, d, l, mu, k, _p(idx), w, _p(perm), _p(L), _p(rowptr),
                               _p(cols), _p(gval)), "afn_build")
    nnz = int(rowptr[-1])
    return AFN(X, l, mu, k, w, perm, L[:k, :k].copy(order="F"), rowptr, cols[:nnz].copy(),
               gval[:nnz].copy())


def fsai_rows(X, l: float, mu: float, perm, L, w: int, rows):
    """Selected FSAI rows (positions in X_r): cols (padded -1), lengths, values."""
    X = _f64(X)
    n, d = X.shape
    perm = np.ascontiguousarray(perm, dtype=np.int32)
    k = L.shape[0] if L is not None else 0
    Lf = np.asfortranarray(L if k > 0 else np.zeros((1, 1)), dtype=np.float64)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    oc = np.zeros((rows.shape[0], w), dtype=np.int32)
    ol = np.zeros(rows.shape[0], dtype=np.int32)
    og = np.zeros((rows.shape[0], w))
    _check(lib().ora_fsai_rows(_p(X), n, d, l, mu, k, _p(perm), _p(Lf), w, _p(rows),
                               rows.shape[0], _p(oc), _p(ol), _p(og)), "fsai_rows")
    return oc, ol, og


def afn_apply(A: AFN, r) -> np.ndarray:
    """s = M^{-1} r (Algorithm 3), original point order."""
    r = _f64(r)
    s = np.zeros_like(r)
    L = A.L if A.k > 0 else np.zeros((1, 1), order="F")
    _check(lib().ora_afn_apply(_p(A.X), A.n, A.X.shape[1], A.l, A.k, _p(A.perm), _p(L),
                               _p(A.rowptr), _p(A.cols), _p(A.gval), _p(r), _p(s)), "afn_apply")
    return s


def pcg(A: AFN, b, tol: float, maxit: int = 500):
    """Textbook PCG with the AFN preconditioner; returns (x, iters, relres, true_relres, status)."""
    b = _f64(b)
    x = np.zeros_like(b)
    it = ctypes.c_int64(0)
    rr = ctypes.c_double(0)
    tr = ctypes.c_double(0)
    L = A.L if A.k > 0 else np.zeros((1, 1), order="F")
    st = lib().ora_pcg(_p(A.X), A.n, A.X.shape[1], A.l, A.mu, A.k, _p(A.perm), _p(L),
                       _p(A.rowptr), _p(A.cols), _p(A.gval), _p(b), tol, maxit, _p(x),
                       ctypes.byref(it), ctypes.byref(rr), ctypes.byref(tr))
    if st not in (ORA_OK, ORA_ENOCONV, ORA_EBREAKDOWN):
        raise OracleError(st, "pcg")
    return x, it.value, rr.value, tr.value, st


# --- rank estimation (Algorithm 4) -----------------------------------------------

def splitmix64_stream(seed: int, count: int) -> np.ndarray:
    out = np.zeros(count, dtype=np.uint64)
    lib().ora_splitmix64_stream(ctypes.c_uint64(seed), count, _p(out))
    return out


def subsample(n: int, m: int, seed: int) -> np.ndarray:
    sub = np.zeros(max(m, 1), dtype=np.int32)
    _check(lib().ora_subsample(n, m, ctypes.c_uint64(seed), _p(sub)), "subsample")
    return sub[:m].copy()


def nystrom_scan(Km, ord_, step=8, tol=0.1, pivtol=None):
    """(r, errs) for the FPS-ordered Nystrom prefixes of Km."""
    Km = np.asfortranarray(np.array(Km, dtype=np.float64))
    m = Km.shape[0]
    ord_ = np.ascontiguousarray(ord_, dtype=np.int32)
    errs = np.full(m, np.nan)
    piv = 1e-14 * m if pivtol is None else pivtol
    r = lib().ora_nystrom_scan(_p(Km), m, _p(ord_), step, tol, piv, _p(errs))
    return int(r), errs


def count_eigs_above(A, tau: float) -> int:
    A = np.asfortranarray(np.array(A, dtype=np.float64))
    return int(lib().ora_count_eigs_above(_p(A), A.shape[0], tau))


def rank_estimate(X, l: float, mu: float, m: int, kmax: int = 2000, kswitch: int = 2000,
                  seed: int = 0):
    """Algorithm 4: returns (k, info) with info = (r, k_est, eig_branch, eig_count)."""
    X = _f64(X)
    k = ctypes.c_int64(0)
    info = np.zeros(4, dtype=np.int64)
    _check(lib().ora_rank_estimate(_p(X), X.shape[0], X.shape[1], l, mu, m, kmax, kswitch,
                                   ctypes.c_uint64(seed), ctypes.byref(k), _p(info)),
           "rank_estimate")
    return int(k.value), tuple(int(v) for v in info)


# --- Algorithm 5, Nystrom branch (nystrom.py) ------------------------------------

from .nystrom import Nystrom, kernel_columns, nystrom_apply, nystrom_build, nystrom_pcg  # noqa: E402,F401


def nystrom_solve(X, l: float, mu: float, k: int, b, tol: float, maxit: int = 500):
    """FPS landmarks (Algorithm 6), the Nystrom preconditioner, textbook PCG."""
    idx, _ = fps(X, k)
    N = nystrom_build(X, l, mu, idx)
    x, it, rel, conv = nystrom_pcg(N, b, tol, maxit, lambda v: kernel_matvec(X, l, mu, v))
    return N, x, it, rel, conv

