"""ctypes binding of the CPU oracle (``oracle/pa_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check and the
CPU-baseline leg of the benchmark, never by the product package. The oracle
follows the paper's objective (section 1, eq. (1)), its Ising mapping
(section 2) and the integer-exact readings of population annealing with
adaptive stochasticity and non-local moves documented in ``pa_oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pa_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
STAT_FIELDS = 10
STAT_NAMES = ("E_min", "E_sum", "uphill_attempts", "uphill_accepts", "level",
              "best_E", "parents", "weight_sum", "grid_index", "jump")

_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (portable flags: no -march, no fast-math)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-std=c11", "-Wall", "-fopenmp", "-shared",
                               "-fPIC", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def use_native_build() -> str:
    """Switch this process to a build of the same source for the host it runs
    on (-O3 -march=native; no fast-math, so results are unchanged), compiled
    into a per-host file on first use. Timing only: the tests use the
    portable build."""
    global _lib, LIB
    import platform
    import tempfile
    tag = platform.node().replace("/", "_") or "host"
    path = os.path.join(tempfile.gettempdir(), f"liboracle_native_{tag}_{os.getuid()}.so")
    if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(SRC):
        tmp = path + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O3", "-march=native", "-std=c11", "-Wall", "-fopenmp",
                               "-shared", "-fPIC", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, path)
    if _lib is not None and LIB == path:
        return path
    LIB = path
    _lib = None
    lib()
    return path


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        u32, u64, i32, i64, f64 = (ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32,
                                   ctypes.c_int64, ctypes.c_double)
        L.oracle_philox4x32_10.argtypes = [P, P, P]
        L.oracle_philox4x32_10.restype = None
        L.oracle_draw.argtypes = [u64, u32, u32, u32, u32, u32, u32]
        L.oracle_draw.restype = u32
        L.oracle_resample_uniform.argtypes = [u64, u32, u32]
        L.oracle_resample_uniform.restype = u64
        L.oracle_threshold.argtypes = [f64, i32]
        L.oracle_threshold.restype = u64
        L.oracle_weight.argtypes = [f64, i64]
        L.oracle_weight.restype = u64
        L.oracle_level_beta.argtypes = [f64, f64, i32]
        L.oracle_level_beta.restype = f64
        L.oracle_energy.argtypes = [i32, P, P, P, P]
        L.oracle_energy.restype = i64
        L.oracle_resample_counts.argtypes = [i32, P, u64, P]
        L.oracle_resample_counts.restype = u64
        L.oracle_icm_pair.argtypes = [i32, P, P, P, P, u32, P]
        L.oracle_icm_pair.restype = i32
        L.oracle_adapt_jump.argtypes = [i32, P, i64, P, i32, i32, i32]
        L.oracle_adapt_jump.restype = i32
        L.oracle_bond_threshold.argtypes = [f64]
        L.oracle_bond_threshold.restype = u64
        L.oracle_wolff.argtypes = [i32, P, P, P, P, P, u64, u64, u32, u32, u32, P]
        L.oracle_wolff.restype = i32
        L.oracle_run.argtypes = [i32, P, P, P, i32, P, i32, P, i32, i32, i32, i32, f64, i32, i32,
                                 i32, i32, i32, i32, i32, u64, u32, i32, P, P, P, P, P, P, P]
        L.oracle_run.restype = ctypes.c_int
        L.oracle_num_threads.argtypes = []
        L.oracle_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def draw(seed, inst, tag, sweep, step, node, replica) -> int:
    return int(lib().oracle_draw(seed, inst, tag, sweep, step, node, replica))


def threshold(beta: float, m: int) -> int:
    return int(lib().oracle_threshold(beta, m))


def weight(dbeta: float, n: int) -> int:
    return int(lib().oracle_weight(dbeta, n))


def level_beta(beta: float, gamma: float, level: int) -> float:
    return float(lib().oracle_level_beta(beta, gamma, level))


def energy(g, x) -> int:
    x = np.ascontiguousarray(x, dtype=np.int8)
    return int(lib().oracle_energy(g.n, _p(g.row_ptr), _p(g.col), _p(g.w), _p(x)))


def resample_counts(W, U: int):
    W = np.ascontiguousarray(W, dtype=np.uint64)
    n = np.zeros(W.shape[0], dtype=np.int32)
    S = lib().oracle_resample_counts(W.shape[0], _p(W), U, _p(n))
    return n, int(S)


def icm_pair(g, xa, xb, d: int):
    """Apply the cluster move to copies of xa, xb; return (xa', xb', mask, size)."""
    xa = np.array(xa, dtype=np.int8)
    xb = np.array(xb, dtype=np.int8)
    mask = np.zeros(g.n, dtype=np.uint8)
    size = lib().oracle_icm_pair(g.n, _p(g.row_ptr), _p(g.col), _p(xa), _p(xb), d, _p(mask))
    return xa, xb, mask.astype(bool), int(size)


def bond_threshold(a: float) -> int:
    return int(lib().oracle_bond_threshold(a))


def wolff(g, x, q: int, seed: int, inst: int, step: int, replica: int):
    """One single-replica cluster update of a copy of x with bond threshold q;
    return (x', mask, size)."""
    x = np.array(x, dtype=np.int8)
    mask = np.zeros(g.n, dtype=np.uint8)
    size = lib().oracle_wolff(g.n, _p(g.row_ptr), _p(g.col), _p(g.w), _p(x), None, q, seed, inst,
                              step, replica, _p(mask))
    return x, mask.astype(bool), int(size)


def adapt_jump(E, betas, jmax: int, num: int, den: int) -> int:
    E = np.ascontiguousarray(E, dtype=np.int32)
    b = np.ascontiguousarray(betas, dtype=np.float64)
    return int(lib().oracle_adapt_jump(E.shape[0], _p(E), int(E.min()), _p(b), jmax, num, den))


def num_threads() -> int:
    return int(lib().oracle_num_threads())


@dataclass
class RunResult:
    x_init: np.ndarray
    x: np.ndarray
    E: np.ndarray
    best_E: int
    best_step: int
    best_sweep: int
    best_replica: int
    best_x: np.ndarray
    stats: np.ndarray
    counts: np.ndarray
    w_tot: int

    @property
    def best_cut(self) -> int:
        return (self.w_tot - self.best_E) // 2


def run(g, betas, sweeps, R, seed, inst=0, order=None, as_enable=0, as_stall_steps=20,
        as_max_level=4, as_frozen_inv=256, as_gamma=0.8, nl_period=0, nthreads=0,
        want_population=True, want_counts=True, nl_kind=0, beta_adapt=0, adapt_jump=8,
        adapt_num=1, adapt_den=2) -> RunResult:
    betas = np.ascontiguousarray(betas, dtype=np.float64)
    K = betas.shape[0]
    order_a = None if order is None else np.ascontiguousarray(order, dtype=np.int32)
    x_init = np.zeros((R, g.n), dtype=np.int8) if want_population else None
    x_out = np.zeros((R, g.n), dtype=np.int8) if want_population else None
    E = np.zeros(R, dtype=np.int32)
    best = np.zeros(4, dtype=np.int64)
    best_x = np.zeros(g.n, dtype=np.int8)
    stats = np.zeros((K, STAT_FIELDS), dtype=np.int64)
    counts = np.zeros((K, R), dtype=np.int32) if want_counts else None
    rc = lib().oracle_run(g.n, _p(g.row_ptr), _p(g.col), _p(g.w), K, _p(betas), sweeps,
                          _p(order_a), as_enable, as_stall_steps, as_max_level, as_frozen_inv,
                          as_gamma, nl_period, nl_kind, beta_adapt, adapt_jump, adapt_num, adapt_den,
                          R, seed, inst, nthreads, _p(x_init),
                          _p(x_out),
                          _p(E), _p(best), _p(best_x), _p(stats), _p(counts))
    if rc != 0:
        raise ValueError(f"oracle_run rejected its arguments (rc={rc})")
    w_tot = int(g.w.astype(np.int64).sum()) // 2
    return RunResult(x_init, x_out, E, int(best[0]), int(best[1]), int(best[2]), int(best[3]),
                     best_x, stats, counts, w_tot)


def run_workload(wl: dict, **over) -> RunResult:
    """Run a ``workloads.workload(...)`` dict (keyword overrides allowed)."""
    p = dict(wl)
    p.update(over)
    return run(p["graph"], p["betas"], p["sweeps"], p["R"], p["seed"], p["inst"], p["order"],
               p["as_enable"], p["as_stall_steps"], p["as_max_level"], p["as_frozen_inv"],
               p["as_gamma"], p["nl_period"], p.get("nthreads", 0),
               p.get("want_population", True), p.get("want_counts", True), p.get("nl_kind", 0),
               p.get("beta_adapt", 0), p.get("adapt_jump", 8), p.get("adapt_num", 1),
               p.get("adapt_den", 2))
