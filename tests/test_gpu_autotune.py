"""The autotuner's candidates agree: every candidate of every tunable (forced
in turn) gives a kernel matvec within the oracle's bound and solves that meet
tol and agree with each other; tuning on records its decisions and the cache
file round-trips them."""
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
    yield mod
    mod.tune_config(mod.AFN_TUNE_OFF)


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def test_every_candidate_agrees(afn):
    n, d, l, mu = 20000, 8, 2.0, 1e-2
    X = W.points("normal", n, d, 81)
    v = np.random.default_rng(82).standard_normal(n)
    rows = np.random.default_rng(83).integers(0, n, 40)
    yo, ab = oracle.kernel_matvec_rows(X, l, mu, v, rows)
    # a handle whose setup and solves run the GEMVs and, with 8 columns,
    # the split-K GEMMs of the block apply
    Xs = W.points("uniform", 4000, 3, 84)
    B = np.random.default_rng(85).standard_normal((4000, 8))
    Bt = torch.tensor(B.T.copy(), device="cuda").t()
    sols = []
    for idx in range(3):
        afn.tune_config(afn.AFN_TUNE_FORCE, idx)
        for prec in (afn.AFN_FP64, afn.AFN_FP32):
            y = afn.kernel_matvec(dev(X), l, mu, dev(v), precision=prec).cpu().numpy()
            if prec == afn.AFN_FP64:
                bound = 2 * (n + 4) * U * ab
            else:
                bound = (30 * (d + 4) * math.log(2) + n + 8) * U32 * ab + 1e-13 * np.abs(v).sum()
            assert np.all(np.abs(y[rows] - yo) <= bound), (idx, prec)
        h = afn.afn_setup(dev(Xs), 0.1, 1e-3, k=200, w=32, precision=afn.AFN_FP32, nrhs_max=8)
        x, info = afn.afn_pcg_solve(h, Bt, tol=1e-8, maxit=500)
        h.close()
        print(f"candidate {idx}:", info, flush=True)
        assert info["converged"]
        sols.append(x.cpu().numpy())
    for s in sols[1:]:
        assert np.linalg.norm(s - sols[0]) <= 1e-6 * np.linalg.norm(sols[0])


def test_tuning_records_decisions_and_cache_round_trips(afn, tmp_path):
    path = tmp_path / "tune.txt"
    afn.tune_config(afn.AFN_TUNE_ON, 0, str(path))
    n, d = 20000, 8
    X = dev(W.points("normal", n, d, 86))
    v = dev(np.random.default_rng(87).standard_normal(n))
    afn.kernel_matvec(X, 2.0, 1e-2, v, precision=afn.AFN_FP32)
    h = afn.afn_setup(dev(W.points("uniform", 3000, 3, 88)), 0.1, 1e-3, k=150, w=32)
    afn.afn_pcg_solve(h, dev(np.ones(3000)), tol=1e-6)
    h.close()
    rep = afn.tune_report()
    print(rep, flush=True)
    assert "kmv_tile|d8_n20000_f32" in rep and "gemv_n_splits|" in rep
    lines = [ln.split() for ln in rep.strip().splitlines()]
    for ln in lines:
        if len(ln) > 2:        # timed here: choice is the fastest candidate
            ms = [float(t) for t in ln[2:]]
            assert ms[int(ln[1])] == min(ms)
    saved = path.read_text().split("\n")
    afn.tune_config(afn.AFN_TUNE_OFF)
    afn.tune_config(afn.AFN_TUNE_ON, 0, str(path))
    rep2 = afn.tune_report()
    for ln in saved:
        if ln:
            assert ln in rep2
    afn.tune_config(afn.AFN_TUNE_OFF)
