"""Continuous-batching request loop for AFN-PCG solves on one GPU.

Requests (points, right-hand side, l, mu) arrive over time.  A request is
admitted -- first come, first served -- as soon as a slot is free and its
device footprint (afn_workspace_size, the one workspace its handle lives in,
plus its inputs and solution) fits in the HBM budget next to the requests
already admitted; a request whose footprint exceeds the whole budget is
rejected.  An admitted request is set up (Algorithm 4/5 and the
preconditioner) on a setup thread, on a stream of its own, while the
requests already set up keep iterating.  All running solves are advanced
together by afn_pcg_step_many: each keeps one PCG iteration (or refinement
step) in flight on its own stream -- so their kernels overlap on the device
-- and the host takes each stopping decision as soon as that request's
iteration is done.  A finished solve leaves the batch at once (the call
returns) and its slot and memory go to the next request, so requests join
and leave between iterations.  The step API runs the same launches as afn_pcg_solve,
so a request's result does not depend on which other requests share the GPU.
"""
from __future__ import annotations

import collections
import concurrent.futures as cf
import dataclasses
import time

import numpy as np
import torch

from . import afn

REJECTED = -1


@dataclasses.dataclass
class Request:
    rid: int
    X: np.ndarray            # (n, d) float64
    b: np.ndarray            # (n,) float64
    l: float
    mu: float
    arrival: float = 0.0     # seconds after the start of the run
    k: int = -1
    w: int = 64
    k_max: int = 2000
    tol: float = 1e-6
    method: int = afn.AFN_METHOD_AFN
    maxit: int = 500
    kernel: int = afn.AFN_KERNEL_GAUSSIAN


@dataclasses.dataclass
class Result:
    rid: int
    status: int
    n: int
    d: int
    footprint: int
    arrival: float
    admitted: float = float("nan")
    done: float = float("nan")
    iterations: int = 0
    outer_iterations: int = 0
    relres_true: float = float("nan")
    k: int = 0
    method: int = -1
    fp64_iterations: int = 0
    grouped_units: int = 0       # iterations advanced in launches shared with other requests
    setup_s: float = float("nan")   # afn_setup on the setup thread, inputs copied in
    x: torch.Tensor | None = None
    error: str = ""

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclasses.dataclass
class Job:
    """A request that is set up: its handle, device inputs and PCG state."""
    req: Request
    res: Result
    slot: int
    stream: object = None
    handle: object = None
    X: object = None
    b: object = None
    state: object = None


class Server:
    """slots: requests admitted at once (set up or iterating); hbm_budget:
    bytes for all of them together (default: 90% of the free device memory
    at start); iters: products per request and afn_pcg_step_many call at most
    (the call also returns as soon as a request finishes);
    setup_workers: setups that may run at once."""

    def __init__(self, slots: int = 8, hbm_budget: int | None = None,
                 precision: int = afn.AFN_FP32, keep_x: bool | str = False, device: str = "cuda",
                 iters: int = 8, setup_workers: int = 2):
        self.slots = slots
        self.precision = precision
        self.keep_x = keep_x
        self.device = torch.device(device)
        self.iters = iters
        self.setup_workers = setup_workers
        self.peak_active = 0
        if hbm_budget is None:
            free, _ = torch.cuda.mem_get_info(self.device)
            hbm_budget = int(0.9 * free)
        self.hbm_budget = hbm_budget
        self.peak_committed = 0
        self.peak_batch = 0

    def footprint(self, r: Request) -> int:
        n, d = r.X.shape
        fp = afn.afn_workspace_size(n, d, k=r.k, w=r.w, k_max=r.k_max, precision=self.precision,
                                    method=r.method, kernel=r.kernel, nrhs_max=0)
        return fp + 8 * n * (d + 2) + (1 << 20)     # inputs, solution, allocator slack

    def _make_stream(self):
        return torch.cuda.Stream(device=self.device)

    # -- the three steps of a request; a test may replace them ------------------
    def _prepare(self, job: Job) -> None:
        """Setup thread: inputs to the device and afn_setup on the job's stream."""
        r = job.req
        t_setup = time.perf_counter()
        with torch.cuda.stream(job.stream):
            job.X = torch.from_numpy(np.ascontiguousarray(r.X)).to(self.device)
            job.b = torch.from_numpy(np.ascontiguousarray(r.b)).to(self.device)
            job.handle = afn.afn_setup(job.X, r.l, r.mu, k=r.k, w=r.w, k_max=r.k_max,
                                       precision=self.precision, method=r.method, kernel=r.kernel,
                                       nrhs_max=0, stream=job.stream)
        si = job.handle.info()
        job.res.k, job.res.method = si.k, si.method
        job.res.setup_s = time.perf_counter() - t_setup

    def _begin(self, job: Job) -> None:
        job.state = afn.afn_pcg_begin(job.handle, job.b, tol=job.req.tol, maxit=job.req.maxit,
                                      stream=job.stream)

    def _step(self, jobs: list[Job]) -> list[Job]:
        """One batch of rounds over every running solve; returns those that finished."""
        afn.afn_pcg_step_many([j.state for j in jobs], iters=self.iters, stream=None)
        done = []
        for j in jobs:
            fin, info = j.state.query()
            if not fin:
                continue
            res = j.res
            res.status = info["status"]
            res.iterations = info["iterations"]
            res.outer_iterations = info["outer_iterations"]
            res.fp64_iterations = info["fp64_iterations"]
            res.grouped_units = info["grouped_units"]
            res.relres_true = info["relres_true"]
            if self.keep_x:
                res.x = j.state.x.cpu() if self.keep_x == "host" else j.state.x
            done.append(j)
        return done

    def _release(self, job: Job) -> None:
        if job.state is not None:
            job.state.end()
        if job.handle is not None:
            job.handle.close()
        job.state = job.handle = job.X = job.b = None

    def run(self, requests: list[Request], on_done=None) -> list[Result]:
        """Serve the requests (arrival times relative to the call); on_done(result)
        runs after each request finishes."""
        order = sorted(requests, key=lambda q: (q.arrival, q.rid))
        results = {q.rid: Result(q.rid, 0, q.X.shape[0], q.X.shape[1], self.footprint(q),
                                 q.arrival) for q in order}
        arrivals = collections.deque(order)
        ready: collections.deque = collections.deque()
        streams = [self._make_stream() for _ in range(self.slots)]
        free_slots = list(range(self.slots))
        committed = 0
        pending: dict = {}       # setup future -> job
        running: list[Job] = []
        t0 = time.perf_counter()

        def close(job: Job):
            nonlocal committed
            self._release(job)
            job.res.done = time.perf_counter() - t0
            committed -= job.res.footprint
            free_slots.append(job.slot)
            if on_done is not None:
                on_done(job.res)

        with cf.ThreadPoolExecutor(max_workers=max(1, self.setup_workers)) as pool:
            while arrivals or ready or pending or running:
                now = time.perf_counter() - t0
                while arrivals and arrivals[0].arrival <= now:
                    ready.append(arrivals.popleft())
                # reject what can never fit
                while ready and results[ready[0].rid].footprint > self.hbm_budget:
                    q = ready.popleft()
                    res = results[q.rid]
                    res.status = REJECTED
                    res.admitted = res.done = now
                    res.error = "footprint exceeds the HBM budget"
                # admit in arrival order while a slot and the memory are free
                while ready and free_slots and committed + results[ready[0].rid].footprint <= self.hbm_budget:
                    q = ready.popleft()
                    res = results[q.rid]
                    res.admitted = time.perf_counter() - t0
                    committed += res.footprint
                    slot = free_slots.pop()
                    job = Job(q, res, slot, streams[slot])
                    pending[pool.submit(self._prepare, job)] = job
                    self.peak_committed = max(self.peak_committed, committed)
                    self.peak_active = max(self.peak_active, self.slots - len(free_slots))
                # set-up requests join the batch
                for fut in [f for f in pending if f.done()]:
                    job = pending.pop(fut)
                    try:
                        fut.result()
                        self._begin(job)
                        running.append(job)
                    except afn.AFNError as e:
                        job.res.status, job.res.error = e.status, str(e)
                        close(job)
                    except Exception as e:  # noqa: BLE001  (reported per request)
                        job.res.status, job.res.error = afn.AFN_EDEVICE, repr(e)
                        close(job)
                if running:
                    self.peak_batch = max(self.peak_batch, len(running))
                    for job in self._step(running):
                        running.remove(job)
                        close(job)
                    continue
                # nothing to iterate: wait for a setup or the next arrival
                timeout = 1.0
                if arrivals:
                    timeout = max(0.0, arrivals[0].arrival - (time.perf_counter() - t0))
                if pending:
                    cf.wait(list(pending), timeout=timeout, return_when=cf.FIRST_COMPLETED)
                elif arrivals:
                    time.sleep(timeout)
        return [results[q.rid] for q in requests]


def _mean(v) -> float:
    v = [x for x in v if x == x]
    return float(np.mean(v)) if v else float("nan")


def summarize(results: list[Result]) -> dict:
    """Throughput of converged requests; latency percentiles (nearest rank)
    over every request that ran, converged or not."""
    ok = [r for r in results if r.status in (afn.AFN_OK,)]
    lat = sorted(r.latency for r in results if r.status != REJECTED)

    def pct(p):
        if not lat:
            return float("nan")
        i = max(0, min(len(lat) - 1, int(np.ceil(p / 100.0 * len(lat))) - 1))
        return lat[i]

    span = max((r.done for r in results if r.done == r.done), default=float("nan"))
    first = min((r.arrival for r in results), default=0.0)
    return {
        "requests": len(results),
        "completed": len(ok),
        "failed": sum(1 for r in results if r.status not in (afn.AFN_OK, REJECTED)),
        "rejected": sum(1 for r in results if r.status == REJECTED),
        "solves_per_s": len(ok) / (span - first) if ok else 0.0,
        "p50_s": pct(50),
        "p99_s": pct(99),
        "max_relres_true": max((r.relres_true for r in ok), default=float("nan")),
        # share of the iterations advanced in launches shared with other requests
        "grouped_frac": (sum(r.grouped_units for r in results) /
                         max(1, sum(r.iterations for r in results))),
        # mean setup time (setup thread) and mean time from setup to done
        "mean_setup_s": _mean([r.setup_s for r in ok]),
        "mean_solve_s": _mean([r.done - r.admitted - r.setup_s for r in ok]),
    }
