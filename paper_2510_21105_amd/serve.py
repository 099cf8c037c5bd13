"""Serving loops for population-annealing requests on one GPU.

``PoolServer`` batches continuously: admitted requests share each
iteration's kernel launches (one step of every request per iteration) inside
a resident device pool. ``Server`` runs each request on its own stream.

Requests (a graph and its run parameters) arrive over time. ``Server`` admits
them in arrival order whenever a stream is free and the device workspaces of
the runs in flight, plus the new one (``pa_workspace_bytes``), fit an HBM
budget; each admitted run is enqueued with ``pa_run`` on its own HIP stream,
and its completion is detected with an event. Every result is the result of
the same run alone (runs are pure functions of their inputs), whatever the mix
it was served in. Requests still waiting can be cancelled. Argument
marshalling and scheduling only: all annealing work runs in the library's
kernels.

The admission policy (``Admission``) is plain Python with no device calls, so
its paths (queueing under the budget, refusal of requests larger than the
budget, cancellation) are testable without a GPU.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

from . import pa


@dataclass
class Request:
    rid: int
    graph: object
    params: pa.RunParams
    arrival: float = 0.0          # seconds after the start of serving


@dataclass
class Result:
    rid: int
    arrival: float
    start: float
    finish: float
    best_cut: int
    best_E: int
    workspace_bytes: int
    cancelled: bool = False
    best_info: dict | None = None     # {E, step, sweep, replica} of the best
    best_x: object = None             # best configuration (n int8, +-1)
    stats: object = None              # per-step statistics (K x PA_STAT_FIELDS int64)

    @property
    def latency(self) -> float:
        return self.finish - self.arrival


class Admission:
    """Arrival-order admission under a byte budget and a number of slots.

    ``arrive(rid, nbytes)`` queues a request (ValueError if it can never fit);
    ``cancel(rid)`` drops a waiting request (False if it was already admitted
    or unknown); ``admit()`` returns the rids that start now, oldest first,
    stopping at the first that does not fit (no overtaking); ``finish(rid)``
    returns a running request's bytes and slot.
    """

    def __init__(self, budget: int, slots: int):
        if budget < 1 or slots < 1:
            raise ValueError("budget and slots must be positive")
        self.budget, self.slots = int(budget), int(slots)
        self.used = 0
        self.waiting: deque = deque()       # (rid, nbytes)
        self.running: dict = {}             # rid -> nbytes

    def arrive(self, rid, nbytes: int) -> None:
        if nbytes > self.budget:
            raise ValueError(f"request {rid} needs {nbytes} workspace bytes, more than the "
                             f"budget {self.budget}")
        self.waiting.append((rid, int(nbytes)))

    def cancel(self, rid) -> bool:
        for q, (r, _) in enumerate(self.waiting):
            if r == rid:
                del self.waiting[q]
                return True
        return False

    def admit(self) -> list:
        out = []
        while self.waiting and len(self.running) < self.slots:
            rid, nb = self.waiting[0]
            if self.used + nb > self.budget:
                break
            self.waiting.popleft()
            self.running[rid] = nb
            self.used += nb
            out.append(rid)
        return out

    def finish(self, rid) -> None:
        self.used -= self.running.pop(rid)

    def idle(self) -> bool:
        return not self.waiting and not self.running


@dataclass
class _Flight:
    req: Request
    solver: pa.Solver
    stream: object
    event: object
    start: float
    nbytes: int


@dataclass
class Server:
    """``hbm_budget``: device bytes the workspaces of concurrent runs may use;
    ``n_streams``: concurrent runs at most (one HIP stream each)."""
    hbm_budget: int
    n_streams: int = 8
    poll_s: float = 2e-4
    _streams: list = field(default_factory=list)

    def __post_init__(self):
        import torch
        if self.n_streams < 1:
            raise ValueError("n_streams must be >= 1")
        self._streams = [torch.cuda.Stream() for _ in range(self.n_streams)]

    def serve(self, requests, realtime: bool = True, cancel=()) -> list:
        """Serve ``requests`` (arrival times honoured when ``realtime``, else all
        present at once); return one Result per request in completion order.
        ``cancel`` holds (time, rid) pairs: at that time the request is dropped
        if it is still waiting (reported with ``cancelled``), else it runs."""
        import torch
        pending = deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        cancels = deque(sorted(cancel))
        adm = Admission(self.hbm_budget, self.n_streams)
        free = list(self._streams)
        flights = {}
        prepared = {}       # rid -> (request, solver, workspace bytes), made once on arrival
        results = []
        t0 = time.perf_counter()
        while pending or not adm.idle():
            now = time.perf_counter() - t0
            while pending and (not realtime or pending[0].arrival <= now):
                req = pending.popleft()
                solver = pa.Solver(req.graph)
                need = solver.workspace_bytes(req.params) + 256
                adm.arrive(req.rid, need)
                prepared[req.rid] = (req, solver, need)
            while cancels and (not realtime or cancels[0][0] <= now):
                _, rid = cancels.popleft()
                if rid in prepared and adm.cancel(rid):
                    req, solver, need = prepared.pop(rid)
                    solver.close()
                    t = time.perf_counter() - t0
                    results.append(Result(rid, req.arrival, t, t, 0, 0, need, cancelled=True))
            # completions
            for rid, f in list(flights.items()):
                if f.event.query():
                    t = time.perf_counter() - t0
                    cut = f.solver.best_cut()
                    info = f.solver.best_info()
                    results.append(Result(rid, f.req.arrival, f.start, t, cut, info["E"], f.nbytes,
                                          best_info=info, best_x=f.solver.best_config(),
                                          stats=f.solver.step_stats()))
                    adm.finish(rid)
                    free.append(f.stream)
                    f.solver.close()
                    del flights[rid]
            # admissions, in arrival order
            started = adm.admit()
            for rid in started:
                req, solver, need = prepared.pop(rid)
                stream = free.pop()
                ws = torch.empty(need, dtype=torch.uint8, device="cuda")
                start = time.perf_counter() - t0
                solver.run(req.params, stream=stream, workspace=ws)
                ev = torch.cuda.Event()
                ev.record(stream)
                flights[rid] = _Flight(req, solver, stream, ev, start, need)
            if not started:
                time.sleep(self.poll_s)
        return results


@dataclass
class PoolServer:
    """Continuous batching: requests join a resident pool (``pa_pool_*``)
    whose device region is ``hbm_budget`` bytes; each iteration advances
    every admitted request by one temperature step in shared launches, and a
    request that finishes leaves, freeing its memory for the next in arrival
    order. One stream for the pool; argument marshalling and scheduling only
    -- all annealing work runs in the library's kernels."""
    hbm_budget: int
    poll_s: float = 2e-4
    iterations: int = 8       # iterations enqueued per advance call (two calls in flight)

    def serve(self, requests, realtime: bool = True, cancel=()) -> list:
        """Serve ``requests`` (arrival times honoured when ``realtime``, else
        all present at once); return one Result per request in completion
        order. ``cancel`` holds (time, rid) pairs: a request still waiting at
        that time is dropped (reported with ``cancelled``)."""
        import torch
        pool = pa.Pool(self.hbm_budget)
        stream = torch.cuda.Stream()
        pending = deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        cancels = deque(sorted(cancel))
        live = {}           # ticket -> (request, solver, submit time)
        waiting = {}        # rid -> ticket, until admitted or finished
        results = []
        t0 = time.perf_counter()
        try:
            while pending or live:
                now = time.perf_counter() - t0
                while pending and (not realtime or pending[0].arrival <= now):
                    req = pending.popleft()
                    solver = pa.Solver(req.graph)
                    t = pool.submit(solver, req.params)
                    live[t] = (req, solver, now)
                    waiting[req.rid] = t
                while cancels and (not realtime or cancels[0][0] <= now):
                    _, rid = cancels.popleft()
                    t = waiting.get(rid)
                    if t is None:
                        continue
                    try:
                        pool.cancel(t)
                    except pa.PAError:
                        continue            # already admitted: it runs
                    req, solver, ts = live.pop(t)
                    del waiting[rid]
                    tc = time.perf_counter() - t0
                    results.append(Result(req.rid, req.arrival, ts, tc, 0, 0, 0, cancelled=True))
                stepped = pool.advance(stream, self.iterations)
                for t in pool.poll():
                    req, solver, ts = live.pop(t)
                    waiting.pop(req.rid, None)
                    info = solver.best_info()
                    tf = time.perf_counter() - t0
                    results.append(Result(req.rid, req.arrival, ts, tf, solver.best_cut(), info["E"],
                                          0, best_info=info, best_x=solver.best_config(),
                                          stats=solver.step_stats()))
                    pool.release(t)
                if stepped == 0:
                    time.sleep(self.poll_s)
            torch.cuda.synchronize()
        finally:
            pool.close()
        return results


def percentile(values, q: float) -> float:
    v = sorted(values)
    if not v:
        return float("nan")
    k = min(len(v) - 1, max(0, int(round(q / 100.0 * (len(v) - 1)))))
    return v[k]
