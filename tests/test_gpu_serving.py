"""Continuous-batching loop: admission, latency bookkeeping, and the result of
each request independent of which requests share the GPU with it."""
import numpy as np
import pytest
import torch

from paper_2304_05460_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    from paper_2304_05460_amd import afn, serving
    afn.lib()
    return afn, serving


def _requests(serving, count=10, seed=11):
    rng = np.random.default_rng(seed)
    arr = W.poisson_arrivals(count, rate_hz=200.0, seed=seed)
    out = []
    for i in range(count):
        n = int(rng.integers(1500, 9000))
        d = int(rng.choice([3, 8]))
        p = W.Problem(f"s{i}", n=n, d=d, l=float(rng.choice([0.05, 0.2, 1.0])),
                      mu=float(rng.choice([1e-3, 1e-2])), k=-1, w=32, tol=1e-6,
                      maxit=400, seed=500 + i, points="uniform" if d == 3 else "normal",
                      k_max=400)
        X, b = W.make(p)
        out.append(serving.Request(i, X, b, p.l, p.mu, arrival=float(arr[i]), k=-1, w=p.w,
                                   k_max=p.k_max, tol=p.tol, maxit=p.maxit))
    return out


def _alone(afn, r, precision):
    X = torch.from_numpy(r.X).cuda()
    b = torch.from_numpy(r.b).cuda()
    h = afn.afn_setup(X, r.l, r.mu, k=r.k, w=r.w, k_max=r.k_max, precision=precision)
    try:
        x, info = afn.afn_pcg_solve(h, b, tol=r.tol, maxit=r.maxit)
    except afn.AFNError as e:
        return None, {"status": e.status, "iterations": 0}
    finally:
        h.close()
    return x.cpu(), info


@pytest.mark.parametrize("prec", [0, 1])
def test_serving_results_equal_alone_and_in_mix(mods, prec):
    afn, serving = mods
    reqs = _requests(serving)
    srv = serving.Server(slots=4, precision=prec, keep_x="host")
    res = srv.run(reqs)
    summ = serving.summarize(res)
    print("serving", prec, summ, flush=True)
    assert summ["rejected"] == 0
    for q, r in zip(reqs, res):
        assert r.rid == q.rid
        assert r.admitted >= q.arrival - 1e-9 and r.done >= r.admitted
        xa, ia = _alone(afn, q, prec)
        assert r.status == ia["status"], (q.rid, r.error)
        assert r.iterations == ia["iterations"]
        if xa is not None:
            assert torch.equal(r.x, xa), f"request {q.rid}: result differs in the mix"
    assert summ["completed"] + summ["failed"] == len(reqs)
    assert np.isfinite(summ["p50_s"]) and summ["p99_s"] >= summ["p50_s"]


def test_serving_admission_by_footprint(mods):
    afn, serving = mods
    reqs = _requests(serving, count=6, seed=12)
    fps = [serving.Server(slots=1, hbm_budget=1 << 40).footprint(q) for q in reqs]
    # the largest request fits alone, but not beside the third largest
    big = sorted(fps)[-3:]
    budget = max(fps) + min(big) - 1
    srv = serving.Server(slots=6, hbm_budget=budget, keep_x=False)
    res = srv.run(reqs)
    assert all(r.status == afn.AFN_OK for r in res), [r.error for r in res]
    assert srv.peak_committed <= budget
    # a request larger than the whole budget is rejected, the rest still run
    srv2 = serving.Server(slots=2, hbm_budget=sorted(fps)[-2], keep_x=False)
    res2 = srv2.run(reqs)
    rej = [r.rid for r in res2 if r.status == serving.REJECTED]
    assert rej == [int(np.argmax(fps))]


def _factors(afn, r, precision, k, stream=None):
    X = torch.from_numpy(r.X).cuda()
    h = afn.afn_setup(X, r.l, r.mu, k=k, w=r.w, k_max=r.k_max, precision=precision,
                      nrhs_max=0, stream=stream)
    try:
        (stream.synchronize if stream is not None else torch.cuda.synchronize)()
        si = h.info()
        out = {"k": si.k, "method": si.method, "lm": h.landmarks()}
        if si.k > 0:
            out["L"] = h.cholesky()
        if si.method == 0 and si.n > si.k:
            out["G"] = h.fsai()
        return out
    finally:
        h.close()


@pytest.mark.parametrize("kfix", [False, True], ids=["rank_estimate", "k400"])
def test_setups_on_concurrent_streams_match_solo(mods, kfix):
    """Setups running at once on four streams give the landmarks, the landmark
    Cholesky factor and the FSAI factor of the same setup run alone, bit for
    bit: no kernel of the setup may depend on what else shares the GPU."""
    import concurrent.futures as cf
    afn, serving = mods
    reqs = _requests(serving)
    ks = [min(400, q.X.shape[0]) if kfix else q.k for q in reqs]
    solo = [_factors(afn, q, 1, k) for q, k in zip(reqs, ks)]
    streams = [torch.cuda.Stream() for _ in range(4)]

    def job(i):
        s = streams[i % 4]
        with torch.cuda.stream(s):
            return _factors(afn, reqs[i], 1, ks[i], stream=s)

    for rep in range(3):
        with cf.ThreadPoolExecutor(4) as ex:
            got = list(ex.map(job, range(len(reqs))))
        for i, (a, b) in enumerate(zip(solo, got)):
            assert (a["k"], a["method"]) == (b["k"], b["method"]), (rep, i)
            assert np.array_equal(a["lm"], b["lm"]), (rep, i, "landmarks")
            if "L" in a:
                assert np.array_equal(a["L"], b["L"]), (rep, i, "cholesky")
            if "G" in a:
                for name, p, q in zip(("rowptr", "cols", "vals"), a["G"], b["G"]):
                    assert np.array_equal(p, q), (rep, i, "fsai " + name)
