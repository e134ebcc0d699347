"""Column-sampling Nystrom preconditioner: the else-branch of Algorithm 5.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain numpy in FP64;
library routines (Cholesky, triangular solve, SVD) serve as single steps.

Construction (Section 2, the stable form the paper recommends for both
sampling- and projection-based Nystrom, with U and Lambda built as in
Frangella, Tropp & Udell's randomized Nystrom preconditioner, here with the
column-sampling test matrix Omega = I[:, S] for the landmark set S):

    Y      = K[:, S]                         (n x k)
    nu     = eps * ||Y||_F                   (stabilizing shift)
    Y_nu   = Y + nu Omega                    (adds nu to the rows S)
    C C^T  = Omega^T Y_nu = K_SS + nu I      (Cholesky, C lower)
    B      = Y_nu C^{-T}
    U S V^T = B                              (thin SVD)
    Lambda = max(0, S^2 - nu)

so that U Lambda U^T is the sampling-based Nystrom approximation
K[:, S] K_SS^{-1} K[S, :] up to the shift.  The preconditioner is
M = U Lambda U^T + mu I, applied by the Sherman-Morrison-Woodbury form with
orthonormal U:

    M^{-1} r = U (Lambda + mu I)^{-1} U^T r + (r - U U^T r) / mu.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg

EPS = np.finfo(np.float64).eps
KIND = [0]      # 0 = Gaussian (Eq. (1.2)), 1 = Matern-3/2; set through oracle.set_kernel


def kernel_columns(X, l: float, cols) -> np.ndarray:
    """K[:, cols]: Gaussian exp(-r^2 / l^2) or Matern-3/2 (1 + sqrt(3) r / l) exp(-sqrt(3) r / l)."""
    X = np.asarray(X, dtype=np.float64)
    D = ((X[:, None, :] - X[None, np.asarray(cols), :]) ** 2).sum(-1)
    if KIND[0] == 1:
        s = np.sqrt(3.0) * np.sqrt(D) / l
        return (1.0 + s) * np.exp(-s)
    return np.exp(-D / (l * l))


@dataclasses.dataclass
class Nystrom:
    X: np.ndarray
    l: float
    mu: float
    S: np.ndarray        # landmark indices (selection order)
    U: np.ndarray        # n x k, orthonormal columns
    lam: np.ndarray      # k eigenvalues of the approximation, >= 0
    nu: float

    @property
    def k(self) -> int:
        return int(self.S.shape[0])

    def approx(self) -> np.ndarray:
        """U Lambda U^T (dense, small n only)."""
        return (self.U * self.lam) @ self.U.T


def nystrom_build(X, l: float, mu: float, S) -> Nystrom:
    X = np.asarray(X, dtype=np.float64)
    S = np.asarray(S, dtype=np.int64)
    k = S.shape[0]
    Y = kernel_columns(X, l, S)
    nu = EPS * np.linalg.norm(Y)
    Ynu = Y.copy()
    Ynu[S, np.arange(k)] += nu
    C = np.linalg.cholesky(Ynu[S, :])
    B = scipy.linalg.solve_triangular(C, Ynu.T, lower=True).T      # Y_nu C^{-T}
    U, sig, _ = np.linalg.svd(B, full_matrices=False)
    lam = np.maximum(0.0, sig * sig - nu)
    return Nystrom(X, l, mu, S, U, lam, nu)


def nystrom_apply(N: Nystrom, r) -> np.ndarray:
    """M^{-1} r by the Sherman-Morrison-Woodbury form with orthonormal U."""
    r = np.asarray(r, dtype=np.float64)
    t = N.U.T @ r
    return N.U @ (t / (N.lam + N.mu)) + (r - N.U @ t) / N.mu


def nystrom_pcg(N: Nystrom, b, tol: float, maxit: int, matvec):
    """Textbook PCG (x0 = 0, stop at ||r|| / ||b|| <= tol) with this
    preconditioner; matvec(v) = (K + mu I) v.  Returns (x, iterations,
    recurrence relres, converged)."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    r = b.copy()
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return x, 0, 0.0, True
    z = nystrom_apply(N, r)
    p = z.copy()
    rho = r @ z
    rel = 1.0
    for it in range(1, maxit + 1):
        q = matvec(p)
        pq = p @ q
        if not pq > 0.0:
            return x, it, rel, False
        alpha = rho / pq
        x += alpha * p
        r -= alpha * q
        rel = np.linalg.norm(r) / bn
        if rel <= tol:
            return x, it, rel, True
        z = nystrom_apply(N, r)
        rho_new = r @ z
        p = z + (rho_new / rho) * p
        rho = rho_new
    return x, maxit, rel, False
