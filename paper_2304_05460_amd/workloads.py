"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws random numbers (numpy ``default_rng``): it holds none of
the method's arithmetic, and it is the one piece of code that both the GPU
path's tests/benchmark and the CPU oracle consume, so both see identical bytes.

Workload family (Section 5.1): points uniform in a d-dimensional box, Gaussian
kernel, regularization mu, random right-hand sides.  The paper's cube of edge
n^{1/3} maps onto the unit cube by scaling the length-scale (Remark 4.5:
K(x/l) only depends on distances divided by l).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass(frozen=True)
class Problem:
    name: str
    n: int
    d: int
    l: float
    mu: float
    k: int          # landmarks; -1 = adaptive (rank estimation)
    w: int          # FSAI nonzeros per row including the diagonal
    tol: float
    maxit: int
    seed: int
    points: str     # "uniform" | "mixture5" | "normal"
    nrhs: int = 1
    rhs: str = "normal"   # "normal" | "uniform_half"
    k_max: int = 2000


def points(kind: str, n: int, d: int, seed: int) -> np.ndarray:
    """Row-major float64 (n, d) point cloud."""
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        return rng.random((n, d))
    if kind == "normal":
        return rng.standard_normal((n, d))
    if kind == "mixture5":
        # 5 centres uniform in the unit cube; each point picks its centre at
        # random (so index order carries no cluster structure); sigma = 0.05;
        # points outside [0,1]^d are redrawn (clipping would create ties).
        centres = rng.random((5, d))
        out = np.empty((n, d))
        todo = np.arange(n)
        while todo.size:
            c = rng.integers(0, 5, size=todo.size)
            x = centres[c] + 0.05 * rng.standard_normal((todo.size, d))
            ok = np.all((x >= 0.0) & (x <= 1.0), axis=1)
            out[todo[ok]] = x[ok]
            todo = todo[~ok]
        return out
    raise ValueError(kind)


def rhs(kind: str, n: int, nrhs: int, seed: int) -> np.ndarray:
    """Right-hand sides, column-major (n,) or (n, nrhs) float64."""
    rng = np.random.default_rng(seed + 1_000_003)
    if kind == "normal":
        b = rng.standard_normal((nrhs, n)).T
    elif kind == "uniform_half":      # Section 5: entries U[-0.5, 0.5]
        b = rng.random((nrhs, n)).T - 0.5
    else:
        raise ValueError(kind)
    b = np.asfortranarray(b)
    return b[:, 0].copy() if nrhs == 1 else b


def make(p: Problem):
    X = points(p.points, p.n, p.d, p.seed)
    b = rhs(p.rhs, p.n, p.nrhs, p.seed)
    return X, b


# Small case the oracle finishes in seconds: n=2000 uniform in [0,1]^3.
C1 = Problem("c1_uniform3d_n2000", n=2000, d=3, l=0.1, mu=1e-4, k=200, w=32,
             tol=1e-8, maxit=500, seed=1, points="uniform")


def c2(l: float, tol: float = 1e-6) -> Problem:
    """n=1e5 points of a 5-centre Gaussian mixture in [0,1]^3, adaptive k <= 2000."""
    return Problem(f"c2_mixture3d_n100000_l{l:g}", n=100_000, d=3, l=l, mu=1e-3, k=-1,
                   w=64, tol=tol, maxit=500, seed=2, points="mixture5")


# Mixed-precision case: n=2e5 standard normal points in R^8.
C3 = Problem("c3_normal8d_n200000", n=200_000, d=8, l=2.0, mu=1e-2, k=4000, w=64,
             tol=1e-6, maxit=500, seed=3, points="normal")

# Multi-RHS case: n=1.5e5 uniform in [0,1]^3, 64 right-hand sides.
C4 = Problem("c4_uniform3d_n150000_r64", n=150_000, d=3, l=0.05, mu=1e-4, k=3000, w=64,
             tol=1e-6, maxit=500, seed=4, points="uniform", nrhs=64)


# High-dimensional case shaped like the paper's 22-feature dataset (n = 49990,
# mu = n 1e-6, l = 1); synthetic points uniform in [0,1]^22 stand in for it.
HIGHD = Problem("highd_uniform22d_n49990", n=49_990, d=22, l=1.0, mu=49_990e-6, k=-1, w=64,
                tol=1e-6, maxit=500, seed=9, points="uniform")


def paper_table1a(l2_paper: float, n: int = 160_000) -> Problem:
    """Table 1a workload mapped to the unit cube: l = sqrt(l2)/n^{1/3}."""
    l = math.sqrt(l2_paper) / n ** (1.0 / 3.0)
    return Problem(f"table1a_l2_{l2_paper:g}", n=n, d=3, l=l, mu=1e-4, k=-1, w=100,
                   tol=1e-4, maxit=500, seed=6, points="uniform", rhs="uniform_half")


def serving_requests(count: int = 256, seed: int = 5, n_lo: float = 5e3, n_hi: float = 2e5):
    """Mixed-size request stream: n log-uniform in [n_lo, n_hi] (default
    [5e3, 2e5]), d in {3, 8}, l log-uniform in [0.01, 2], mu in {1e-4, 1e-2};
    one right-hand side each."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        d = int(rng.choice([3, 8]))
        l = float(math.exp(rng.uniform(math.log(0.01), math.log(2.0))))
        mu = float(rng.choice([1e-4, 1e-2]))
        out.append(Problem(f"req{i}", n=n, d=d, l=l, mu=mu, k=-1, w=64, tol=1e-6,
                           maxit=500, seed=10_000 + i,
                           points="uniform" if d == 3 else "normal"))
    return out


def poisson_arrivals(count: int, rate_hz: float, seed: int = 7) -> np.ndarray:
    """Arrival times (seconds) of a Poisson stream: exponential gaps of mean 1/rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_hz, size=count))
