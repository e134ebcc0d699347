"""Continuous batching in afn_pcg_step_many: the inner iterations of like
mixed-precision solves (same d, kernel, precision, method, pattern width, n
within a factor of 2) advance in grouped launches (one ragged launch per
kernel over all of them).  Each solve's arithmetic is that of its own
launches, so every solution must equal the one afn_pcg_solve gives alone,
bit for bit, and the like solves must report grouped units."""
import numpy as np
import pytest
import torch

from paper_2304_05460_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def afn():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2304_05460_amd import afn as mod
    mod.lib()
    return mod


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), device="cuda")


# (label, n, d, points, l, mu, setup params, tol, groupable)
CASES = [
    ("afn32 d3 a", 2100, 3, "uniform", 0.3, 1e-3, dict(k=120, w=32, precision=1, nrhs_max=0), 1e-6, True),
    ("afn32 d3 b", 2600, 3, "uniform", 0.4, 1e-3, dict(k=150, w=32, precision=1, nrhs_max=0), 1e-6, True),
    ("afn32 d3 c", 3000, 3, "mixture5", 0.2, 1e-3, dict(k=200, w=16, precision=1, nrhs_max=0), 1e-6, True),
    ("afn32 d3 d", 3900, 3, "uniform", 0.3, 1e-3, dict(k=100, w=64, precision=1, nrhs_max=0), 1e-6, True),
    ("afn32 d8 a", 2200, 8, "normal", 2.0, 1e-2, dict(k=150, w=16, precision=1, nrhs_max=0), 1e-6, True),
    ("afn32 d8 b", 3300, 8, "normal", 1.5, 1e-2, dict(k=200, w=24, precision=1, nrhs_max=0), 1e-6, True),
    ("nys32 a", 2500, 3, "uniform", 0.5, 1e-2, dict(k=150, method=1, precision=1, nrhs_max=0), 1e-6, True),
    ("nys32 b", 3100, 3, "uniform", 0.6, 1e-2, dict(k=180, method=1, precision=1, nrhs_max=0), 1e-6, True),
    ("bf16 a", 2300, 3, "uniform", 0.3, 1e-3, dict(k=120, w=32, precision=2, nrhs_max=0), 1e-6, True),
    ("bf16 b", 2900, 3, "uniform", 0.3, 1e-3, dict(k=160, w=32, precision=2, nrhs_max=0), 1e-6, True),
    ("matern a", 2400, 3, "uniform", 0.2, 1e-3, dict(k=120, w=32, precision=1, nrhs_max=0, kernel=1), 1e-6, True),
    ("matern b", 3500, 3, "uniform", 0.2, 1e-3, dict(k=150, w=32, precision=1, nrhs_max=0, kernel=1), 1e-6, True),
    ("fp64", 2700, 3, "uniform", 0.3, 1e-3, dict(k=120, w=32), 1e-8, False),
    ("afn32 large", 9000, 3, "uniform", 0.3, 1e-3, dict(k=200, w=32, precision=1, nrhs_max=0), 1e-6, False),
]


def test_grouped_step_many_equals_solves_alone(afn):
    handles, bs, refs = [], [], []
    for i, (lab, n, d, pts, l, mu, prm, tol, _) in enumerate(CASES):
        h = afn.afn_setup(dev(W.points(pts, n, d, 300 + i)), l, mu, **prm)
        b = dev(np.random.default_rng(400 + i).standard_normal(n))
        x, info = afn.afn_pcg_solve(h, b, tol=tol, maxit=400)
        assert info["status"] == afn.AFN_OK, (lab, info)
        assert info["grouped_units"] == 0
        handles.append(h)
        bs.append(b)
        refs.append((x.clone(), info))
        print(f"{lab}: n={n} {info['iterations']} its, {info['outer_iterations']} outer", flush=True)
    states = [afn.afn_pcg_begin(h, b, tol=CASES[i][7], maxit=400) for i, (h, b) in enumerate(zip(handles, bs))]
    rounds = 0
    while not all(s.query()[0] for s in states):
        afn.afn_pcg_step_many(states, iters=1)
        rounds += 1
        assert rounds < 5000
    torch.cuda.synchronize()
    for i, s in enumerate(states):
        lab, groupable = CASES[i][0], CASES[i][8]
        done, info = s.query()
        x0, i0 = refs[i]
        print(f"{lab}: grouped units {info['grouped_units']} of {info['iterations']}", flush=True)
        assert done and info["status"] == i0["status"]
        assert torch.equal(s.x, x0), lab
        assert info["iterations"] == i0["iterations"] and info["outer_iterations"] == i0["outer_iterations"]
        assert info["relres_true"] == i0["relres_true"]
        if groupable:
            assert info["grouped_units"] > info["iterations"] // 4, lab
        else:
            assert info["grouped_units"] == 0, lab
        s.end()
    for h in handles:
        h.close()


def test_grouped_step_many_on_one_stream(afn):
    # every state on one caller stream: the same bits, and the like solves grouped
    cases = [c for c in CASES if c[0].startswith("afn32 d3")]
    handles, bs, refs = [], [], []
    for i, (lab, n, d, pts, l, mu, prm, tol, _) in enumerate(cases):
        h = afn.afn_setup(dev(W.points(pts, n, d, 500 + i)), l, mu, **prm)
        b = dev(np.random.default_rng(600 + i).standard_normal(n))
        x, info = afn.afn_pcg_solve(h, b, tol=tol, maxit=400)
        handles.append(h)
        bs.append(b)
        refs.append(x.clone())
    stream = torch.cuda.Stream()
    states = [afn.afn_pcg_begin(h, b, tol=1e-6, maxit=400, stream=stream) for h, b in zip(handles, bs)]
    while not all(s.query()[0] for s in states):
        afn.afn_pcg_step_many(states, iters=3, stream=stream)
    torch.cuda.synchronize()
    for i, s in enumerate(states):
        done, info = s.query()
        assert done and torch.equal(s.x, refs[i]) and info["grouped_units"] > 0, cases[i][0]
        s.end()
    for h in handles:
        h.close()
