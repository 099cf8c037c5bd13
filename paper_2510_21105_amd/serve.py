"""Serving loop for population-annealing requests on one GPU.

Requests (a graph and its run parameters) arrive over time. The server admits
them in arrival order whenever a stream is free and the device workspaces of
the runs in flight, plus the new one (``pa_workspace_bytes``), fit an HBM
budget; each admitted run is enqueued with ``pa_run`` on its own HIP stream,
and its completion is detected with an event. Every result is the result of
the same run alone (runs are pure functions of their inputs), whatever the mix
it was served in. Argument marshalling and scheduling only: all annealing work
runs in the library's kernels.
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

    @property
    def latency(self) -> float:
        return self.finish - self.arrival


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

    def serve(self, requests, realtime: bool = True) -> list:
        """Serve ``requests`` (arrival times honoured when ``realtime``, else all
        present at once); return one Result per request in completion order."""
        import torch
        pending = deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        waiting: deque = deque()
        flights: list = []
        free = list(self._streams)
        used = 0
        results = []
        t0 = time.perf_counter()
        prepared = {}       # rid -> (solver, workspace bytes), made once on arrival
        while pending or waiting or flights:
            now = time.perf_counter() - t0
            while pending and (not realtime or pending[0].arrival <= now):
                req = pending.popleft()
                solver = pa.Solver(req.graph)
                need = solver.workspace_bytes(req.params) + 256
                if need > self.hbm_budget:
                    raise ValueError(f"request {req.rid} needs {need} workspace bytes, "
                                     f"more than the budget {self.hbm_budget}")
                prepared[req.rid] = (solver, need)
                waiting.append(req)
            # completions
            still = []
            for f in flights:
                if f.event.query():
                    t = time.perf_counter() - t0
                    cut = f.solver.best_cut()
                    info = f.solver.best_info()
                    results.append(Result(f.req.rid, f.req.arrival, f.start, t, cut, info["E"],
                                          f.nbytes))
                    used -= f.nbytes
                    free.append(f.stream)
                    f.solver.close()
                else:
                    still.append(f)
            flights = still
            # admissions, in arrival order
            admitted = False
            while waiting and free:
                req = waiting[0]
                solver, need = prepared[req.rid]
                if used + need > self.hbm_budget:
                    break
                waiting.popleft()
                del prepared[req.rid]
                admitted = True
                stream = free.pop()
                ws = torch.empty(need, dtype=torch.uint8, device="cuda")
                start = time.perf_counter() - t0
                solver.run(req.params, stream=stream, workspace=ws)
                ev = torch.cuda.Event()
                ev.record(stream)
                flights.append(_Flight(req, solver, stream, ev, start, need))
                used += need
            if not admitted:
                time.sleep(self.poll_s)
        return results


def percentile(values, q: float) -> float:
    v = sorted(values)
    if not v:
        return float("nan")
    k = min(len(v) - 1, max(0, int(round(q / 100.0 * (len(v) - 1)))))
    return v[k]
