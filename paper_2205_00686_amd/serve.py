"""Continuous-batching server for phase-change solves.

Requests (a workload: parameters, initial fields, step count) arrive over time.  The server admits
a queued request as soon as a slot is free and its device footprint (lbm_footprint_bytes) fits in
the HBM budget next to the running ones; its state then stays on the device until it finishes.
All running simulations advance together, `chunk` steps at a time, in one batched kernel launch
per step (graph-replayed), each stopping at its own step count; between chunks finished requests
are read back and retired and newly arrived ones join.  A request's result is bit-identical to
running it alone (the batched launch executes the same kernel on every node).

Admission order: "arrival" (the default) admits queued requests strictly in arrival order, so a
request that does not fit holds back the ones behind it.  "shortest" admits, among the queued
requests whose fields are ready, the one with the least work (nodes x steps) first, and lets a
smaller one pass a larger one that does not fit yet; once the oldest queued request has waited
`max_wait` seconds it is admitted next regardless of its size, which bounds how long the largest
requests can be passed over.

`fifo()` is the baseline: one request at a time, in arrival order, each with its own plain
lbm_step launches.
"""
from __future__ import annotations

import concurrent.futures as cf
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import LBM_FP32, Batch, Solver, footprint_bytes


@dataclass
class Request:
    rid: int
    arrival: float           # seconds after the start of the run
    steps: int
    make: object             # callable returning a workloads.Workload (initial fields built on demand)
    nodes: int = 0
    footprint: int = 0
    t_arrive: float = float("nan")   # when the request counts as arrived (its arrival, or 0 without realtime)
    t_admit: float = float("nan")
    t_done: float = float("nan")
    result: tuple = None
    error: str = None
    meta: dict = field(default_factory=dict)

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrive


def _percentile(v, q):
    return float(np.percentile(np.asarray(v, dtype=np.float64), q)) if len(v) else float("nan")


def summarize(reqs, t0, t1):
    done = [r for r in reqs if r.error is None and r.t_done == r.t_done]
    lat = [r.latency for r in done]
    lu = sum(r.nodes * r.steps for r in done)
    span = t1 - t0
    return {"requests": len(reqs), "completed": len(done), "failed": sum(r.error is not None for r in reqs),
            "latency_p50_s": _percentile(lat, 50), "latency_p99_s": _percentile(lat, 99),
            "latency_mean_s": float(np.mean(lat)) if lat else float("nan"),
            "makespan_s": span, "node_updates": lu, "aggregate_mlups": lu / span / 1e6 if span > 0 else 0.0}


class Server:
    def __init__(self, hbm_budget: int, max_slots: int = 64, chunk: int = 512, precision: int = LBM_FP32,
                 keep_results: bool = True, prepare_workers: int = 4, streams: int = 4, policy: str = "arrival",
                 max_wait: float = 5.0):
        if policy not in ("arrival", "shortest"):
            raise ValueError(f"unknown admission policy {policy!r}")
        self.policy = policy
        self.max_wait = float(max_wait)
        self.hbm_budget = int(hbm_budget)
        self.max_slots = int(max_slots)
        self.chunk = int(chunk)
        self.precision = precision
        self.keep_results = keep_results
        self.pool = cf.ThreadPoolExecutor(max_workers=prepare_workers)
        self.n_streams = int(streams)

    def run(self, requests, realtime: bool = True, log=None):
        """Serve `requests` (sorted by arrival).  With realtime=False every request is considered
        arrived at t=0 (pure throughput run).  Returns (requests, summary).

        The host work of a round overlaps the GPU work of the chunk in flight: the batch runs on
        a stream of its own and every request on one of a few request streams, so while chunk k
        runs the server reads back the requests that finished with chunk k-1 and initialises the
        ones admitted for chunk k+1."""
        import torch

        batch_stream = _new_stream()
        req_streams = [_new_stream() for _ in range(self.n_streams)]
        reqs = sorted(requests, key=lambda r: r.arrival)
        arriving = deque(reqs)
        queued = deque()
        prep = {}
        running = {}       # rid -> (request, solver): members of the batch
        remaining = {}
        ready = []         # admitted and initialised, joining at the next launch
        finishing = []     # finished with the last synced chunk, results not read yet
        batch, members = None, ()
        inflight = False
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0  # noqa: E731
        used = 0
        admitted = 0
        while arriving or queued or running or ready or finishing or inflight:
            # ---- host work, overlapping the chunk in flight
            while arriving and (not realtime or arriving[0].arrival <= now()):
                r = arriving.popleft()
                r.t_arrive = r.arrival if realtime else 0.0
                prep[r.rid] = self.pool.submit(r.make)
                queued.append(r)
            for r, sol in finishing:
                if r.error is None:
                    fields = sol.fields()
                    if self.keep_results:
                        r.result = fields
                r.t_done = now()
                used -= r.footprint
                sol.close()
                if log:
                    log(r)
            finishing = []
            while queued and len(running) + len(ready) < self.max_slots:
                r = self._next(queued, prep, now())
                if r is None:
                    break
                try:
                    w = prep[r.rid].result()
                    need = footprint_bytes(w.params, self.precision)
                except Exception as e:  # noqa: BLE001 -- a request that cannot be prepared fails alone
                    queued.remove(r)
                    del prep[r.rid]
                    r.error = f"preparing the request failed: {e}"
                    r.t_done = now()
                    continue
                if need > self.hbm_budget:  # can never fit: reject it now instead of blocking the queue
                    queued.remove(r)
                    del prep[r.rid]
                    r.error = "footprint exceeds the HBM budget"
                    r.t_done = now()
                    continue
                if used + need > self.hbm_budget:
                    break  # wait for room (under "shortest" nothing smaller is ready either)
                queued.remove(r)
                del prep[r.rid]
                try:
                    st = req_streams[admitted % len(req_streams)]
                    sol = Solver(w.params, precision=self.precision, stream=st).init(w.rho, w.ux, w.uy, w.T)
                except Exception as e:  # noqa: BLE001 -- a bad request must not stop the others
                    r.error = str(e)
                    r.t_done = now()
                    continue
                admitted += 1
                r.nodes, r.footprint, r.t_admit = w.nodes, need, now()
                used += need
                ready.append((r, sol))
            # ---- the chunk in flight ends: finished and failed members leave the batch
            if inflight:
                status = batch.sync()
                inflight = False
                for j, i in enumerate(members):
                    r, sol = running[i]
                    remaining[i] -= min(self.chunk, remaining[i])
                    if status[j] != 0:
                        r.error = "numerical failure"
                    if remaining[i] == 0 or r.error is not None:
                        finishing.append((r, sol))
                        del running[i], remaining[i]
            for r, sol in ready:
                running[r.rid] = (r, sol)
                remaining[r.rid] = r.steps
            ready = []
            if not running:
                if batch is not None:  # no member left: release it before its members go
                    batch.close()
                    batch, members = None, ()
                if not (finishing or queued or arriving):
                    continue
                if not finishing:
                    # idle: wait for the next arrival or a field preparation
                    if queued:
                        cf.wait([prep[queued[0].rid]], timeout=0.05)
                    elif arriving and realtime:
                        time.sleep(max(0.0, min(0.05, arriving[0].arrival - now())))
                continue
            ids = tuple(sorted(running))
            if ids != members:
                if batch is not None:
                    batch.close()
                batch = Batch([running[i][1] for i in ids], stream=batch_stream)
                members = ids
            for j, i in enumerate(ids):
                batch.set_budget(j, min(self.chunk, remaining[i]))
            batch.step(self.chunk)
            inflight = True
        if batch is not None:
            batch.close()
        torch.cuda.synchronize()
        return reqs, summarize(reqs, 0.0, now())


    def _next(self, queued, prep, t):
        """The queued request to admit next, or None while its fields are still being prepared."""
        if self.policy == "arrival":
            r = queued[0]
            return r if prep[r.rid].done() else None
        # shortest: a request that has waited max_wait seconds goes first (in arrival order)
        head = queued[0]
        if t - head.t_arrive >= self.max_wait:
            return head if prep[head.rid].done() else None
        best, work = None, None
        for r in queued:
            fut = prep[r.rid]
            if not fut.done():
                continue
            if fut.exception() is not None:
                return r  # the caller records its failure and removes it
            w = fut.result()
            wk = w.nodes * r.steps
            if best is None or wk < work:
                best, work = r, wk
        return best


def _new_stream():
    """A stream of default priority on the current device."""
    import torch
    return torch.cuda.Stream()


def fifo(requests, precision: int = LBM_FP32, realtime: bool = True, keep_results: bool = True, log=None,
         prepare_workers: int = 4):
    """Baseline: one request at a time in arrival order, plain lbm_step launches.  Initial fields
    of requests that have arrived are prepared in the background meanwhile, as in Server.run."""
    import torch

    reqs = sorted(requests, key=lambda r: r.arrival)
    pool = cf.ThreadPoolExecutor(max_workers=prepare_workers)
    t0 = time.perf_counter()
    now = lambda: time.perf_counter() - t0  # noqa: E731
    futs = {}

    def submit_arrived():
        for q in reqs:
            if q.rid not in futs and (not realtime or q.arrival <= now()):
                futs[q.rid] = pool.submit(q.make)

    for r in reqs:
        r.t_arrive = r.arrival if realtime else 0.0
    for r in reqs:
        while realtime and r.arrival > now():
            time.sleep(min(0.05, r.arrival - now()))
        submit_arrived()
        r.t_admit = now()
        try:
            w = futs[r.rid].result()
            s = Solver(w.params, precision=precision).init(w.rho, w.ux, w.uy, w.T)
            r.nodes = w.nodes
            s.step(r.steps)
            fields = s.fields()
            if keep_results:
                r.result = fields
            s.close()
        except Exception as e:  # noqa: BLE001 -- a bad request must not stop the others
            r.error = str(e)
        futs[r.rid] = None
        r.t_done = now()
        submit_arrived()
        if log:
            log(r)
    torch.cuda.synchronize()
    return reqs, summarize(reqs, 0.0, now())
