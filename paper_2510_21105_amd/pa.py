"""Python binding of the C ABI in ``include/pa.h`` (argument marshalling only).

Every step of the annealing runs in the HIP kernels of ``libpa.so``; PyTorch
only supplies the device workspace (a uint8 tensor) and the HIP stream. There
is no CPU fallback: if the library is missing this module raises on import
of the library.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, fields

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpa.so")
STAT_FIELDS = 10
STAT_NAMES = ("E_min", "E_sum", "uphill_attempts", "uphill_accepts", "level",
              "best_E", "parents", "weight_sum", "grid_index", "jump")

PA_OK, PA_EINVAL, PA_ERANGE, PA_EWORKSPACE, PA_EDEVICE, PA_ESTATE, PA_EABORTED = 0, -1, -2, -3, -4, -5, -6
_STATUS = {PA_EINVAL: "PA_EINVAL", PA_ERANGE: "PA_ERANGE", PA_EWORKSPACE: "PA_EWORKSPACE",
           PA_EDEVICE: "PA_EDEVICE", PA_ESTATE: "PA_ESTATE", PA_EABORTED: "PA_EABORTED"}

EXPORTS = ("pa_last_error", "pa_create", "pa_destroy", "pa_graph_info", "pa_workspace_bytes",
           "pa_run", "pa_run_batch", "pa_build_tables", "pa_best_cut", "pa_best_info", "pa_best_config", "pa_best_config_hex",
           "pa_get_population", "pa_get_initial_population", "pa_get_step_stats",
           "pa_get_counts", "pa_get_launch_info", "pa_set_timing", "pa_get_sweep_time",
           "pa_run_steps", "pa_checkpoint_bytes", "pa_checkpoint_save", "pa_checkpoint_load",
           "pa_run_static", "pa_fused_create", "pa_fused_workspace_bytes", "pa_fused_tune",
           "pa_fused_run", "pa_fused_set_graph", "pa_fused_info", "pa_fused_destroy",
           "pa_pool_create", "pa_pool_submit", "pa_pool_cancel", "pa_pool_advance", "pa_pool_poll",
           "pa_pool_release", "pa_pool_info", "pa_pool_destroy", "pa_set_fault_step")
STATIC_SCRATCH_BYTES = 64 << 20     # PA_STATIC_SCRATCH_BYTES


class PAError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class Schedule(ctypes.Structure):
    _fields_ = [
        ("n_steps", ctypes.c_int32),
        ("beta", ctypes.POINTER(ctypes.c_double)),
        ("sweeps_per_step", ctypes.c_int32),
        ("order", ctypes.POINTER(ctypes.c_int32)),
        ("as_enable", ctypes.c_int32),
        ("as_stall_steps", ctypes.c_int32),
        ("as_max_level", ctypes.c_int32),
        ("as_frozen_inv", ctypes.c_int32),
        ("as_gamma", ctypes.c_double),
        ("nl_period", ctypes.c_int32),
        ("sweep_kernel", ctypes.c_int32),
        ("tile_replicas", ctypes.c_int32),
        ("wg_threads", ctypes.c_int32),
        ("record", ctypes.c_int32),
        ("nl_kind", ctypes.c_int32),
        ("beta_adapt", ctypes.c_int32),
        ("adapt_jump", ctypes.c_int32),
        ("adapt_num", ctypes.c_int32),
        ("adapt_den", ctypes.c_int32),
        ("field_bits", ctypes.c_int32),
    ]


class BatchRun(ctypes.Structure):
    _fields_ = [
        ("solver", ctypes.c_void_p),
        ("schedule", ctypes.POINTER(Schedule)),
        ("R", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("instance", ctypes.c_uint32),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t),
    ]


class FusedEntry(ctypes.Structure):
    _fields_ = [
        ("solver", ctypes.c_void_p),
        ("schedule", ctypes.POINTER(Schedule)),
        ("R", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("instance", ctypes.c_uint32),
    ]


_lib = None


def lib():
    """Load ``libpa.so``; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2510_21105_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, u32, u64 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                 ctypes.c_uint32, ctypes.c_uint64)
        L.pa_last_error.restype = ctypes.c_char_p
        L.pa_last_error.argtypes = []
        sigs = {
            "pa_create": [ctypes.POINTER(P), i32, P, P, P],
            "pa_destroy": [P],
            "pa_graph_info": [P, P],
            "pa_workspace_bytes": [P, ctypes.POINTER(Schedule), i32, ctypes.POINTER(ctypes.c_size_t)],
            "pa_run": [P, ctypes.POINTER(Schedule), i32, u64, u32, P, ctypes.c_size_t, P],
            "pa_run_batch": [ctypes.POINTER(BatchRun), i32, ctypes.POINTER(P), i32],
            "pa_run_static": [P, ctypes.POINTER(Schedule), i32, u64, u32, P],
            "pa_fused_create": [ctypes.POINTER(P), ctypes.POINTER(FusedEntry), i32],
            "pa_fused_workspace_bytes": [P, ctypes.POINTER(ctypes.c_size_t)],
            "pa_fused_tune": [P, P, ctypes.c_size_t, P, i32],
            "pa_fused_run": [P, P, ctypes.c_size_t, P],
            "pa_fused_set_graph": [P, i32],
            "pa_fused_info": [P, P, i32, ctypes.POINTER(i32)],
            "pa_fused_destroy": [P],
            "pa_pool_create": [ctypes.POINTER(P), P, ctypes.c_size_t],
            "pa_pool_submit": [P, ctypes.POINTER(FusedEntry), ctypes.POINTER(i64)],
            "pa_pool_cancel": [P, i64],
            "pa_pool_advance": [P, P, i32, ctypes.POINTER(i32)],
            "pa_pool_poll": [P, P, i32, ctypes.POINTER(i32)],
            "pa_pool_release": [P, i64],
            "pa_pool_info": [P, P],
            "pa_pool_destroy": [P],
            "pa_build_tables": [ctypes.POINTER(Schedule), i32, i32, P, ctypes.POINTER(ctypes.c_size_t)],
            "pa_best_cut": [P, ctypes.POINTER(i64), ctypes.POINTER(i32)],
            "pa_best_info": [P, P],
            "pa_best_config": [P, P],
            "pa_best_config_hex": [P, ctypes.c_char_p, ctypes.c_size_t],
            "pa_get_population": [P, P, P, P],
            "pa_get_initial_population": [P, P],
            "pa_get_step_stats": [P, P],
            "pa_get_counts": [P, P],
            "pa_get_launch_info": [P, P],
            "pa_set_timing": [P, i32],
            "pa_set_fault_step": [P, i32],
            "pa_get_sweep_time": [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)],
            "pa_run_steps": [P, ctypes.POINTER(Schedule), i32, u64, u32, i32, i32, P, ctypes.c_size_t, P],
            "pa_checkpoint_bytes": [P, ctypes.POINTER(ctypes.c_size_t)],
            "pa_checkpoint_save": [P, P, ctypes.c_size_t],
            "pa_checkpoint_load": [P, ctypes.POINTER(Schedule), i32, u64, u32, P, ctypes.c_size_t, P,
                                   ctypes.c_size_t, P],
        }
        for name, args in sigs.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        _lib = L
    return _lib


def _check(st: int):
    if st != PA_OK:
        raise PAError(st, lib().pa_last_error().decode(errors="replace"))


def _p(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


@dataclass
class RunParams:
    betas: np.ndarray
    sweeps: int
    R: int
    seed: int
    inst: int = 0
    order: np.ndarray | None = None
    as_enable: int = 0
    as_stall_steps: int = 20
    as_max_level: int = 4
    as_frozen_inv: int = 256
    as_gamma: float = 0.8
    nl_period: int = 0
    sweep_kernel: int = 0
    tile_replicas: int = 0
    wg_threads: int = 0
    record: int = 0
    nl_kind: int = 0              # 0: pair cluster moves; 1: single-replica Wolff updates
    beta_adapt: int = 0           # 1: betas is a grid walked by adaptive jumps
    adapt_jump: int = 8
    adapt_num: int = 1
    adapt_den: int = 2
    field_bits: int = 0           # 8 or 16: refuse graphs whose local fields do not fit


def _params_key(p: RunParams):
    """Hashable form of a RunParams (arrays by their bytes)."""
    out = []
    for f in fields(p):
        v = getattr(p, f.name)
        if isinstance(v, (list, tuple)):
            v = np.asarray(v)
        if isinstance(v, np.ndarray):
            v = (str(v.dtype), v.shape, v.tobytes())
        out.append(v)
    return tuple(out)


class Solver:
    """One validated graph; runs population annealing on the current HIP device."""

    def __init__(self, graph):
        self.graph = graph
        self.n = int(graph.n)
        self._row_ptr = np.ascontiguousarray(graph.row_ptr, dtype=np.int32)
        self._col = np.ascontiguousarray(graph.col, dtype=np.int32)
        self._w = np.ascontiguousarray(graph.w, dtype=np.int8)
        h = ctypes.c_void_p()
        _check(lib().pa_create(ctypes.byref(h), self.n, _p(self._row_ptr), _p(self._col), _p(self._w)))
        self._h = h
        self._workspace = None
        self._need = {}
        self._keep = None
        self._R = 0
        self._K = 0

    def close(self):
        if getattr(self, "_h", None):
            lib().pa_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        out = np.zeros(4, dtype=np.int64)
        _check(lib().pa_graph_info(self._h, _p(out)))
        return dict(n=int(out[0]), nnz=int(out[1]), w_tot=int(out[2]), dmax=int(out[3]))

    @staticmethod
    def _schedule(p: RunParams):
        betas = np.ascontiguousarray(p.betas, dtype=np.float64)
        order = None if p.order is None else np.ascontiguousarray(p.order, dtype=np.int32)
        sch = Schedule()
        sch.n_steps = betas.shape[0]
        sch.beta = betas.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        sch.sweeps_per_step = p.sweeps
        sch.order = (order.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if order is not None
                     else ctypes.POINTER(ctypes.c_int32)())
        sch.as_enable = p.as_enable
        sch.as_stall_steps = p.as_stall_steps
        sch.as_max_level = p.as_max_level
        sch.as_frozen_inv = p.as_frozen_inv
        sch.as_gamma = p.as_gamma
        sch.nl_period = p.nl_period
        sch.sweep_kernel = p.sweep_kernel
        sch.tile_replicas = p.tile_replicas
        sch.wg_threads = p.wg_threads
        sch.record = p.record
        sch.nl_kind = p.nl_kind
        sch.beta_adapt = p.beta_adapt
        sch.adapt_jump = p.adapt_jump
        sch.adapt_num = p.adapt_num
        sch.adapt_den = p.adapt_den
        sch.field_bits = p.field_bits
        return sch, (betas, order)

    def workspace_bytes(self, p: RunParams) -> int:
        sch, keep = self._schedule(p)
        b = ctypes.c_size_t()
        _check(lib().pa_workspace_bytes(self._h, ctypes.byref(sch), p.R, ctypes.byref(b)))
        return int(b.value)

    def _prepare(self, p: RunParams, workspace=None):
        """Schedule struct (with the arrays it points to) and an aligned workspace."""
        import torch
        sch, keep = self._schedule(p)
        # The size is a pure function of the graph and the run's arguments:
        # asked once per distinct arguments (the library plans the run again
        # when it starts it).
        key = _params_key(p)
        need = self._need.get(key)
        if need is None:
            need = self._need[key] = self.workspace_bytes(p)
        if workspace is None:
            if self._workspace is None or self._workspace.numel() < need + 256:
                self._workspace = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
            workspace = self._workspace
        base = workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        avail = workspace.numel() - (aligned - base)
        return sch, keep, workspace, aligned, avail

    def _started(self, p: RunParams, sch, keep, workspace, stream=None):
        # The workspace may be dropped (replaced by a larger one) while the run
        # still executes on its stream: the allocator must not hand the memory
        # out again before that stream's queued work is done.
        if workspace is not None and stream is not None:
            workspace.record_stream(stream)
        self._keep = (keep, workspace, sch)
        self._R = p.R
        self._K = int(sch.n_steps)

    def _enqueued(self, st: int, p: RunParams, sch, keep, workspace, stream=None):
        """Record the run a call started; a run stopped by the fault hook
        (PA_EABORTED) still holds its workspace and can continue."""
        if st in (PA_OK, PA_EABORTED):
            self._started(p, sch, keep, workspace, stream)
        _check(st)
        return self

    def run(self, p: RunParams, stream=None, workspace=None):
        """Enqueue a run on ``stream`` (torch.cuda stream; current one by default)."""
        import torch
        sch, keep, workspace, aligned, avail = self._prepare(p, workspace)
        st = torch.cuda.current_stream() if stream is None else stream
        return self._enqueued(lib().pa_run(self._h, ctypes.byref(sch), p.R, p.seed, p.inst,
                                           ctypes.c_void_p(aligned), avail, ctypes.c_void_p(st.cuda_stream)),
                              p, sch, keep, workspace, st)

    def run_static(self, p: RunParams, stream=None):
        """Enqueue a run inside the library's static device workspace
        (pa_run_static: no device allocation; results valid until the next
        such run on this GPU)."""
        import torch
        sch, keep = self._schedule(p)
        st = torch.cuda.current_stream() if stream is None else stream
        return self._enqueued(lib().pa_run_static(self._h, ctypes.byref(sch), p.R, p.seed, p.inst,
                                                  ctypes.c_void_p(st.cuda_stream)),
                              p, sch, keep, None)

    def run_steps(self, p: RunParams, k_begin: int, k_end: int, stream=None, workspace=None):
        """Enqueue steps [k_begin, k_end) of the run (k_begin > 0 continues the
        run this solver holds, in the same workspace)."""
        import torch
        if k_begin > 0 and workspace is None and self._keep is not None:
            workspace = self._keep[1]
        sch, keep, workspace, aligned, avail = self._prepare(p, workspace)
        st = torch.cuda.current_stream() if stream is None else stream
        return self._enqueued(lib().pa_run_steps(self._h, ctypes.byref(sch), p.R, p.seed, p.inst, k_begin,
                                                 k_end, ctypes.c_void_p(aligned), avail,
                                                 ctypes.c_void_p(st.cuda_stream)),
                              p, sch, keep, workspace, st)

    def checkpoint(self) -> bytes:
        """The run's state between steps as bytes (synchronises its stream)."""
        n = ctypes.c_size_t()
        _check(lib().pa_checkpoint_bytes(self._h, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        _check(lib().pa_checkpoint_save(self._h, buf, n.value))
        return buf.raw

    def restore(self, p: RunParams, blob: bytes, stream=None, workspace=None):
        """Prepare a run of ``p`` and load the state saved by ``checkpoint``;
        continue with ``run_steps(p, k, K)`` (k = ``next_step(blob)``)."""
        import torch
        sch, keep, workspace, aligned, avail = self._prepare(p, workspace)
        st = torch.cuda.current_stream() if stream is None else stream
        _check(lib().pa_checkpoint_load(self._h, ctypes.byref(sch), p.R, p.seed, p.inst, blob,
                                        len(blob), ctypes.c_void_p(aligned), avail,
                                        ctypes.c_void_p(st.cuda_stream)))
        self._started(p, sch, keep, workspace, st)
        return self

    # ---- results (each synchronises the run's stream) ----
    def best_cut(self) -> int:
        cut = ctypes.c_int64()
        e = ctypes.c_int32()
        _check(lib().pa_best_cut(self._h, ctypes.byref(cut), ctypes.byref(e)))
        return int(cut.value)

    def best_info(self):
        out = np.zeros(4, dtype=np.int64)
        _check(lib().pa_best_info(self._h, _p(out)))
        return dict(E=int(out[0]), step=int(out[1]), sweep=int(out[2]), replica=int(out[3]))

    def best_config(self) -> np.ndarray:
        x = np.zeros(self.n, dtype=np.int8)
        _check(lib().pa_best_config(self._h, _p(x)))
        return x

    def best_config_hex(self) -> str:
        buf = ctypes.create_string_buffer((self.n + 3) // 4 + 1)
        _check(lib().pa_best_config_hex(self._h, buf, len(buf)))
        return buf.value.decode()

    def population(self, fields: bool = False):
        """Final population ``(x, E)``, or ``(x, h, E)`` with the local
        fields h_i = sum_j w_ij x_j when ``fields`` is set."""
        x = np.zeros((self._R, self.n), dtype=np.int8)
        E = np.zeros(self._R, dtype=np.int32)
        h = np.zeros((self._R, self.n), dtype=np.int16) if fields else None
        _check(lib().pa_get_population(self._h, _p(x), _p(h), _p(E)))
        return (x, h, E) if fields else (x, E)

    def initial_population(self):
        x = np.zeros((self._R, self.n), dtype=np.int8)
        _check(lib().pa_get_initial_population(self._h, _p(x)))
        return x

    def step_stats(self) -> np.ndarray:
        out = np.zeros((self._K, STAT_FIELDS), dtype=np.int64)
        _check(lib().pa_get_step_stats(self._h, _p(out)))
        return out

    def counts(self) -> np.ndarray:
        out = np.zeros((self._K, self._R), dtype=np.int32)
        _check(lib().pa_get_counts(self._h, _p(out)))
        return out

    def launch_info(self):
        out = np.zeros(8, dtype=np.int64)
        _check(lib().pa_get_launch_info(self._h, _p(out)))
        keys = ("sweep_kernel", "tile_replicas", "threads", "workgroups", "lds_bytes", "levels",
                "rounds", "sweep_launches")
        return dict(zip(keys, (int(v) for v in out)))

    def set_fault_step(self, k: int):
        """Fault injection (pa_set_fault_step): the next run that would
        enqueue step ``k`` stops before it and raises PAError with status
        PA_EABORTED, keeping the run's first ``k`` steps; -1 clears it."""
        _check(lib().pa_set_fault_step(self._h, int(k)))
        return self

    def set_timing(self, every):
        """Time the sweep launches of every ``every``-th step of later runs
        (True = every step, False/0 = off)."""
        _check(lib().pa_set_timing(self._h, int(every)))

    def sweep_time(self):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        _check(lib().pa_get_sweep_time(self._h, ctypes.byref(ms), ctypes.byref(n)))
        return float(ms.value), int(n.value)


def build_tables(p: RunParams, d_max: int, e_span: int):
    """The run's fixed-point tables (pa_build_tables): thresholds
    [K][levels][d_max + 1] and weights [K - 1][e_span + 1] (adaptive steps:
    [min(adapt_jump, K - 1)][e_span + 1], one row per jump), as uint64 arrays."""
    sch, keep = Solver._schedule(p)
    n = ctypes.c_size_t()
    _check(lib().pa_build_tables(ctypes.byref(sch), d_max, e_span, None, ctypes.byref(n)))
    buf = np.zeros(n.value // 8, dtype=np.uint64)
    _check(lib().pa_build_tables(ctypes.byref(sch), d_max, e_span, _p(buf), ctypes.byref(n)))
    K = len(p.betas)
    L = p.as_max_level + 1 if p.as_enable else 1
    nt = K * L * (d_max + 1)
    rows = min(p.adapt_jump, K - 1) if p.beta_adapt else K - 1
    return buf[:nt].reshape(K, L, d_max + 1), buf[nt:].reshape(rows, e_span + 1)


def run_batch(solvers, params, streams):
    """Enqueue independent runs (one per distinct solver) through pa_run_batch,
    run i on ``streams[i % len(streams)]`` (torch.cuda streams)."""
    if len(solvers) != len(params):
        raise ValueError("one RunParams per solver")
    runs = (BatchRun * len(solvers))()
    held = []
    for i, (s, p) in enumerate(zip(solvers, params)):
        sch, keep, workspace, aligned, avail = s._prepare(p)
        held.append((s, p, sch, keep, workspace))
        runs[i] = BatchRun(s._h.value, ctypes.pointer(sch), p.R, p.seed, p.inst, aligned, avail)
    hs = (ctypes.c_void_p * len(streams))(*[st.cuda_stream for st in streams])
    st = lib().pa_run_batch(runs, len(solvers), hs, len(streams))
    # Keep every workspace alive: runs before a failing one stay enqueued.
    for i, (s, p, sch, keep, workspace) in enumerate(held):
        s._started(p, sch, keep, workspace, streams[i % len(streams)])
    _check(st)
    return solvers


class FusedBatch:
    """Runs sharing kernel launches (pa_fused_*): one solver per run; after
    ``run`` each solver answers the result calls as after ``Solver.run``."""

    def __init__(self, solvers, params):
        if len(solvers) != len(params):
            raise ValueError("one RunParams per solver")
        self.solvers = list(solvers)
        self.params = list(params)
        self._keep = [Solver._schedule(p) for p in self.params]
        entries = (FusedEntry * len(self.solvers))()
        for i, (s, p, (sch, _)) in enumerate(zip(self.solvers, self.params, self._keep)):
            entries[i] = FusedEntry(s._h.value, ctypes.pointer(sch), p.R, p.seed, p.inst)
        h = ctypes.c_void_p()
        _check(lib().pa_fused_create(ctypes.byref(h), entries, len(self.solvers)))
        self._h = h
        self._workspace = None
        self._need = {}

    def close(self):
        if getattr(self, "_h", None):
            lib().pa_fused_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_bytes(self) -> int:
        b = ctypes.c_size_t()
        _check(lib().pa_fused_workspace_bytes(self._h, ctypes.byref(b)))
        return int(b.value)

    def _ws(self):
        import torch
        need = self.workspace_bytes()
        if self._workspace is None or self._workspace.numel() < need + 256:
            self._workspace = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
        base = self._workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        return aligned, self._workspace.numel() - (aligned - base)

    def tune(self, probe_steps: int = 3, stream=None):
        import torch
        ws, n = self._ws()
        st = torch.cuda.current_stream() if stream is None else stream
        _check(lib().pa_fused_tune(self._h, ctypes.c_void_p(ws), n, ctypes.c_void_p(st.cuda_stream),
                                   probe_steps))
        self._workspace.record_stream(st)
        return self.info()

    def set_graph(self, on: bool):
        _check(lib().pa_fused_set_graph(self._h, 1 if on else 0))

    def run(self, stream=None):
        import torch
        ws, n = self._ws()
        st = torch.cuda.current_stream() if stream is None else stream
        _check(lib().pa_fused_run(self._h, ctypes.c_void_p(ws), n, ctypes.c_void_p(st.cuda_stream)))
        for s, p, (sch, keep) in zip(self.solvers, self.params, self._keep):
            s._started(p, sch, keep, self._workspace, st)
        return self

    def info(self):
        ng = ctypes.c_int32()
        _check(lib().pa_fused_info(self._h, None, 0, ctypes.byref(ng)))
        out = np.zeros((max(ng.value, 1), 8), dtype=np.int64)
        _check(lib().pa_fused_info(self._h, _p(out), ng.value, ctypes.byref(ng)))
        keys = ("record_mode", "runs", "tile_replicas", "threads", "offset_entries", "workgroups",
                "lds_bytes", "fs_per_attempt")
        return [dict(zip(keys, (int(v) for v in row))) for row in out[:ng.value]]


class Pool:
    """A resident pool of runs advanced together, one step per iteration
    (pa_pool_*), inside a device region of ``budget`` bytes; or, with
    ``workspace=(address, bytes)``, inside caller memory."""

    def __init__(self, budget: int = 0, workspace=None):
        if workspace is None:
            import torch
            self._mem = torch.empty(int(budget) + 256, dtype=torch.uint8, device="cuda")
            base = self._mem.data_ptr()
            addr = (base + 255) // 256 * 256
            size = self._mem.numel() - (addr - base)
        else:
            self._mem = None
            addr, size = workspace
        h = ctypes.c_void_p()
        _check(lib().pa_pool_create(ctypes.byref(h), ctypes.c_void_p(addr), size))
        self._h = h
        self._keep = {}

    def close(self):
        if getattr(self, "_h", None):
            lib().pa_pool_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, solver: "Solver", p: RunParams) -> int:
        sch, keep = Solver._schedule(p)
        e = FusedEntry(solver._h.value, ctypes.pointer(sch), p.R, p.seed, p.inst)
        t = ctypes.c_int64()
        _check(lib().pa_pool_submit(self._h, ctypes.byref(e), ctypes.byref(t)))
        self._keep[t.value] = (solver, p, sch, keep)
        return int(t.value)

    def cancel(self, ticket: int):
        _check(lib().pa_pool_cancel(self._h, ticket))
        self._keep.pop(ticket, None)

    def advance(self, stream=None, iterations: int = 1) -> int:
        """Enqueue up to ``iterations`` iterations; return how many were."""
        import torch
        st = torch.cuda.current_stream() if stream is None else stream
        n = ctypes.c_int32()
        _check(lib().pa_pool_advance(self._h, ctypes.c_void_p(st.cuda_stream), iterations,
                                     ctypes.byref(n)))
        return int(n.value)

    def poll(self, cap: int = 256):
        out = np.zeros(cap, dtype=np.int64)
        n = ctypes.c_int32()
        _check(lib().pa_pool_poll(self._h, _p(out), cap, ctypes.byref(n)))
        done = [int(t) for t in out[:n.value]]
        for t in done:
            solver, p, sch, keep = self._keep[t]
            solver._started(p, sch, keep, self._mem)
        return done

    def release(self, ticket: int):
        _check(lib().pa_pool_release(self._h, ticket))
        self._keep.pop(ticket, None)

    def info(self):
        out = np.zeros(6, dtype=np.int64)
        _check(lib().pa_pool_info(self._h, _p(out)))
        keys = ("waiting", "stepping", "finished", "bytes_in_use", "bytes_for_runs", "iterations")
        return dict(zip(keys, (int(v) for v in out)))


def params_from_workload(wl: dict, **over) -> RunParams:
    d = dict(wl)
    d.update(over)
    return RunParams(betas=d["betas"], sweeps=d["sweeps"], R=d["R"], seed=d["seed"],
                     inst=d.get("inst", 0), order=d.get("order"), as_enable=d["as_enable"],
                     as_stall_steps=d["as_stall_steps"], as_max_level=d["as_max_level"],
                     as_frozen_inv=d["as_frozen_inv"], as_gamma=d["as_gamma"],
                     nl_period=d["nl_period"], sweep_kernel=d.get("sweep_kernel", 0),
                     tile_replicas=d.get("tile_replicas", 0), wg_threads=d.get("wg_threads", 0),
                     record=d.get("record", 0), nl_kind=d.get("nl_kind", 0),
                     beta_adapt=d.get("beta_adapt", 0), adapt_jump=d.get("adapt_jump", 8),
                     adapt_num=d.get("adapt_num", 1), adapt_den=d.get("adapt_den", 2),
                     field_bits=d.get("field_bits", 0))


def next_step(blob: bytes) -> int:
    """The step a checkpoint continues at (its header: magic, key, size, then
    n, R, K, G, words, next step, record, version as int32)."""
    import struct
    if len(blob) < 56 or blob[:8] != b"PACKPT01":
        raise ValueError("not a checkpoint of this library")
    return struct.unpack_from("<8i", blob, 24)[5]
