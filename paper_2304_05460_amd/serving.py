"""Continuous-batching request loop for AFN-PCG solves on one GPU.

Requests (points, right-hand side, l, mu) arrive over time.  A request is
admitted -- first come, first served -- as soon as a slot is free and its
device footprint (afn_footprint_bytes: an upper bound of what afn_setup
allocates, plus its inputs and solution) fits in the HBM budget next to the
requests already running.  Every admitted request runs setup and solve on a
stream of its own, so the kernels of different requests overlap on the
device; when it finishes, its handle and buffers are released and the next
request is admitted.  A request whose footprint exceeds the whole budget is
rejected.  Every kernel of the library reduces in a fixed order, so a
request's result does not depend on which other requests share the GPU.

The scheduler and the workers are Python threads; every device call goes
through the C-ABI (ctypes releases the interpreter lock during the call).
"""
from __future__ import annotations

import collections
import dataclasses
import threading
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
    x: torch.Tensor | None = None
    error: str = ""

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class Server:
    """slots: requests running at once; hbm_budget: bytes for all running
    requests together (default: 90% of the free device memory at start)."""

    def __init__(self, slots: int = 8, hbm_budget: int | None = None,
                 precision: int = afn.AFN_FP32, keep_x: bool = False, device: str = "cuda"):
        self.slots = slots
        self.precision = precision
        self.keep_x = keep_x
        self.device = torch.device(device)
        self.peak_active = 0
        if hbm_budget is None:
            free, _ = torch.cuda.mem_get_info(self.device)
            hbm_budget = int(0.9 * free)
        self.hbm_budget = hbm_budget
        self.peak_committed = 0

    def footprint(self, r: Request) -> int:
        n, d = r.X.shape
        fp = afn.afn_footprint_bytes(n, d, k=r.k, w=r.w, k_max=r.k_max,
                                     precision=self.precision, method=r.method)
        return fp + 8 * n * (d + 2) + (1 << 20)     # inputs, solution, allocator slack

    def _make_stream(self):
        return torch.cuda.Stream(device=self.device)

    def _work(self, r: Request, res: Result, stream: torch.cuda.Stream):
        try:
            with torch.cuda.stream(stream):
                X = torch.from_numpy(np.ascontiguousarray(r.X)).to(self.device, non_blocking=False)
                b = torch.from_numpy(np.ascontiguousarray(r.b)).to(self.device, non_blocking=False)
                h = afn.afn_setup(X, r.l, r.mu, k=r.k, w=r.w, k_max=r.k_max,
                                  precision=self.precision, method=r.method, kernel=r.kernel,
                                  stream=stream)
                try:
                    x, info = afn.afn_pcg_solve(h, b, tol=r.tol, maxit=r.maxit, stream=stream)
                    si = h.info()
                    res.k, res.method = si.k, si.method
                finally:
                    h.close()
                res.status = info["status"]
                res.iterations = info["iterations"]
                res.outer_iterations = info["outer_iterations"]
                res.fp64_iterations = info["fp64_iterations"]
                res.relres_true = info["relres_true"]
                if self.keep_x:
                    res.x = x.cpu() if self.keep_x == "host" else x
                stream.synchronize()
        except afn.AFNError as e:
            res.status = e.status
            res.error = str(e)
        except Exception as e:  # noqa: BLE001  (reported per request)
            res.status = afn.AFN_EDEVICE
            res.error = repr(e)

    def run(self, requests: list[Request], on_done=None) -> list[Result]:
        """Serve the requests (arrival times relative to the call); on_done(result)
        runs on the worker thread after each request finishes."""
        order = sorted(requests, key=lambda q: (q.arrival, q.rid))
        results = {q.rid: Result(q.rid, 0, q.X.shape[0], q.X.shape[1], self.footprint(q),
                                 q.arrival) for q in order}
        arrivals = collections.deque(order)
        ready: collections.deque = collections.deque()
        cv = threading.Condition()
        state = {"active": 0, "committed": 0}
        streams = [self._make_stream() for _ in range(self.slots)]
        free_streams = list(range(self.slots))
        t0 = time.perf_counter()

        def finish(q: Request, res: Result, sidx: int):
            res.done = time.perf_counter() - t0
            with cv:
                state["active"] -= 1
                state["committed"] -= res.footprint
                free_streams.append(sidx)
                cv.notify_all()

        def runner(q: Request, res: Result, sidx: int):
            try:
                self._work(q, res, streams[sidx])
            finally:
                finish(q, res, sidx)
                if on_done is not None:
                    on_done(res)

        threads = []
        with cv:
            while arrivals or ready or state["active"]:
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
                while (ready and state["active"] < self.slots and
                       state["committed"] + results[ready[0].rid].footprint <= self.hbm_budget):
                    q = ready.popleft()
                    res = results[q.rid]
                    res.admitted = time.perf_counter() - t0
                    state["active"] += 1
                    state["committed"] += res.footprint
                    self.peak_committed = max(self.peak_committed, state["committed"])
                    self.peak_active = max(self.peak_active, state["active"])
                    sidx = free_streams.pop()
                    th = threading.Thread(target=runner, args=(q, res, sidx), daemon=True)
                    threads.append(th)
                    th.start()
                timeout = None
                if arrivals:
                    timeout = max(0.0, arrivals[0].arrival - (time.perf_counter() - t0))
                if arrivals or ready or state["active"]:
                    cv.wait(timeout=timeout if timeout is not None else 1.0)
        for th in threads:
            th.join()
        return [results[q.rid] for q in requests]


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
    }
