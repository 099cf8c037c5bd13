"""Seeded synthetic inputs: graphs, annealing schedules and sweep orders.

This module only *generates inputs*. It holds none of the annealing method's
arithmetic (no Metropolis rule, no fields, no energies, no resampling), so both
the device library and the CPU oracle can be fed from it without sharing any
of the method's code.

The G-set benchmark (random, toroidal and planar graphs, 800 to 20,000 nodes,
binary signed or unsigned weights; paper section 1) is not available offline;
these generators stand in for its random and toroidal families:

* ``random_graph(n, m, seed)``: m distinct node pairs drawn uniformly, weight
  +1 (the G63 shape is n=7,000, m=41,459; paper section 1).
* ``torus(L, seed, signed)``: an L x L periodic grid, node ``r*L + c``, edges to
  the right and downward neighbours, weights +1 or equiprobable +-1.

The random stream is SplitMix64 (Steele, Lea, Flood, OOPSLA 2014), written
out here so the inputs do not depend on a numpy version.
"""
from __future__ import annotations

import numpy as np

_MASK64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def splitmix64(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Return ``count`` SplitMix64 outputs for states seed+(start+1..start+count)*golden."""
    with np.errstate(over="ignore"):
        idx = np.arange(start + 1, start + count + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + idx * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def _uniform_index(words: np.ndarray, n: int) -> np.ndarray:
    """Map 32-bit words to [0, n) by multiply-shift."""
    return ((words.astype(np.uint64) * np.uint64(n)) >> np.uint64(32)).astype(np.int64)


class Graph:
    """Symmetric CSR graph with int8 weights in {-1, +1}.

    ``row_ptr`` (n+1, int32), ``col`` (nnz, int32), ``w`` (nnz, int8). Every
    undirected edge {i, j} appears twice, once in row i and once in row j,
    with equal weight; rows are sorted by column.
    """

    def __init__(self, n: int, row_ptr: np.ndarray, col: np.ndarray, w: np.ndarray, name: str = ""):
        self.n = int(n)
        self.row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
        self.col = np.ascontiguousarray(col, dtype=np.int32)
        self.w = np.ascontiguousarray(w, dtype=np.int8)
        self.name = name

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    @property
    def n_edges(self) -> int:
        return self.nnz // 2

    def edges(self):
        """Return (i, j, w) arrays of the undirected edges with i < j."""
        rows = np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.row_ptr))
        keep = rows < self.col
        return rows[keep], self.col[keep].astype(np.int64), self.w[keep].astype(np.int64)

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr).astype(np.int64)


def from_edges(n: int, i, j, w=None, name: str = "") -> Graph:
    """Build the symmetric CSR of undirected edges (i[k], j[k], w[k])."""
    i = np.asarray(i, dtype=np.int64)
    j = np.asarray(j, dtype=np.int64)
    w = np.ones_like(i) if w is None else np.asarray(w, dtype=np.int64)
    src = np.concatenate([i, j])
    dst = np.concatenate([j, i])
    ww = np.concatenate([w, w])
    order = np.lexsort((dst, src))
    src, dst, ww = src[order], dst[order], ww[order]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, src + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    return Graph(n, row_ptr, dst, ww, name)


def random_graph(n: int, m: int, seed: int, name: str = "") -> Graph:
    """m distinct unordered pairs of [0, n), uniform, weight +1.

    Pairs are drawn as (hi32(z)*n >> 32, lo32(z)*n >> 32) from the SplitMix64
    stream of ``seed``; self pairs are skipped and the first m distinct pairs
    (in stream order) are kept.
    """
    if m > n * (n - 1) // 2:
        raise ValueError("too many edges")
    keys = np.empty(0, dtype=np.int64)
    start = 0
    while keys.shape[0] < m:
        batch = max(1024, 2 * (m - keys.shape[0]))
        z = splitmix64(seed, batch, start)
        start += batch
        a = _uniform_index(z >> np.uint64(32), n)
        b = _uniform_index(z & np.uint64(0xFFFFFFFF), n)
        ok = a != b
        lo = np.minimum(a, b)[ok]
        hi = np.maximum(a, b)[ok]
        cand = np.concatenate([keys, lo * n + hi])
        _, first = np.unique(cand, return_index=True)
        keys = cand[np.sort(first)]
    keys = keys[:m]
    return from_edges(n, keys // n, keys % n, None, name or f"G({n},{m})#{seed}")


def torus(L: int, seed: int, signed: bool = True, name: str = "") -> Graph:
    """L x L periodic grid; node r*L+c joined to (r, c+1) and (r+1, c).

    With ``signed`` each of the 2*L*L edges gets weight +1 or -1 with equal
    probability from bit 0 of the SplitMix64 stream of ``seed`` (edge order:
    all right-edges row-major, then all down-edges row-major).
    """
    if L < 3:
        raise ValueError("torus needs L >= 3")
    r, c = np.divmod(np.arange(L * L, dtype=np.int64), L)
    right = r * L + (c + 1) % L
    down = ((r + 1) % L) * L + c
    i = np.concatenate([r * L + c, r * L + c])
    j = np.concatenate([right, down])
    if signed:
        bits = (splitmix64(seed, 2 * L * L) & np.uint64(1)).astype(np.int64)
        w = 1 - 2 * bits
    else:
        w = np.ones(2 * L * L, dtype=np.int64)
    return from_edges(L * L, i, j, w, name or f"torus{L}{'pm' if signed else ''}#{seed}")


def cycle(n: int) -> Graph:
    i = np.arange(n)
    return from_edges(n, i, (i + 1) % n, None, f"C{n}")


def complete(n: int, weight: int = 1) -> Graph:
    i, j = np.triu_indices(n, 1)
    return from_edges(n, i, j, np.full(i.shape, weight), f"K{n}")


def linear_betas(beta0: float, beta1: float, K: int) -> np.ndarray:
    """beta_k = beta0 + (beta1 - beta0) * k / (K - 1), k = 0..K-1, in FP64."""
    if K == 1:
        return np.array([float(beta0)])
    return np.array([beta0 + (beta1 - beta0) * k / (K - 1) for k in range(K)], dtype=np.float64)


def natural_order(n: int) -> np.ndarray:
    return np.arange(n, dtype=np.int32)


def coloring_order(g: Graph) -> np.ndarray:
    """Sweep order by colour classes of a first-fit greedy colouring in node
    order (node i takes the smallest colour none of its smaller neighbours
    has), nodes ascending within a class. Every class is an independent set,
    so a sweep in this order has as many dependency levels as colours."""
    n = g.n
    color = np.full(n, -1, dtype=np.int64)
    for i in range(n):
        nb = g.col[g.row_ptr[i]:g.row_ptr[i + 1]]
        used = set(int(c) for c in color[nb] if c >= 0)
        c = 0
        while c in used:
            c += 1
        color[i] = c
    return np.lexsort((np.arange(n), color)).astype(np.int32)


def checkerboard_order(L: int) -> np.ndarray:
    """Sites with (r + c) even in row-major order, then the odd sites."""
    r, c = np.divmod(np.arange(L * L), L)
    even = np.nonzero((r + c) % 2 == 0)[0]
    odd = np.nonzero((r + c) % 2 == 1)[0]
    return np.concatenate([even, odd]).astype(np.int32)


# ---------------------------------------------------------------------------
# Named workloads (graph + schedule + population) shaped like the paper's runs.
# ---------------------------------------------------------------------------

def workload(name: str) -> dict:
    """Return a dict with graph, betas, sweeps, order, R, seed, inst, AS/NL params.

    * ``small800``: random G(800, 4000) seed 1, R=128, 50 linear steps
      0.1 -> 3.0, 10 sweeps/step, natural order.
    * ``brute20``: random G(20, 60) seed 2, same schedule, checked against
      exhaustive search.
    * ``g63like``: random G(7000, 41459) seed 3 (the G63 shape), R=4096,
      2000 steps 0.1 -> 5.0, 10 sweeps/step, natural order, adaptive
      stochasticity and non-local moves on.
    * ``g63color``: ``g63like`` swept in greedy-colouring order.
    * ``g63wolff``: ``g63like`` with single-replica cluster updates in place
      of the pair cluster moves.
    * ``torus100``: 100 x 100 torus with +-1 weights, seed 4, R=16384,
      1000 steps 0.1 -> 4.0, 5 sweeps/step, checkerboard order.

    ``desc`` names the workload in one line; ``field_bytes`` (default 2) is
    the width of a local field in the sequential cost model that prices the
    sweep's algorithmic bytes (int16 fields for the random graphs, int8 for
    the degree-4 torus).
    """
    base = dict(seed=42, as_enable=0, as_stall_steps=20, as_max_level=4,
                as_frozen_inv=256, as_gamma=0.8, nl_period=0)
    if name == "small800":
        g = random_graph(800, 4000, 1, "small800")
        return dict(base, graph=g, betas=linear_betas(0.1, 3.0, 50), sweeps=10,
                    order=natural_order(g.n), R=128, inst=0,
                    desc="random G(N=800, M=4000) seed 1, R=128, K=50 linear beta 0.1->3.0, "
                         "S=10, natural order")
    if name == "brute20":
        g = random_graph(20, 60, 2, "brute20")
        return dict(base, graph=g, betas=linear_betas(0.1, 3.0, 50), sweeps=10,
                    order=natural_order(g.n), R=128, inst=0,
                    desc="random G(N=20, M=60) seed 2, R=128, K=50 linear beta 0.1->3.0, "
                         "S=10, natural order")
    if name == "g63like":
        g = random_graph(7000, 41459, 3, "g63like")
        return dict(base, graph=g, betas=linear_betas(0.1, 5.0, 2000), sweeps=10,
                    order=natural_order(g.n), R=4096, inst=1,
                    as_enable=1, nl_period=10,
                    desc="random G(N=7000, M=41459) seed 3 (G63 shape), R=4096, K=2000 linear "
                         "beta 0.1->5.0, S=10, natural order, adaptive stochasticity + "
                         "cluster moves every 10 steps")
    if name == "g63color":
        wl = workload("g63like")
        g = wl["graph"]
        return dict(wl, order=coloring_order(g),
                    desc="random G(N=7000, M=41459) seed 3 (G63 shape), R=4096, K=2000 linear "
                         "beta 0.1->5.0, S=10, greedy-colouring order, adaptive stochasticity + "
                         "cluster moves every 10 steps")
    if name == "g63wolff":
        wl = workload("g63like")
        return dict(wl, nl_kind=1,
                    desc="random G(N=7000, M=41459) seed 3 (G63 shape), R=4096, K=2000 linear "
                         "beta 0.1->5.0, S=10, natural order, adaptive stochasticity + "
                         "single-replica cluster updates every 10 steps")
    if name == "torus100":
        g = torus(100, 4, True, "torus100")
        return dict(base, graph=g, betas=linear_betas(0.1, 4.0, 1000), sweeps=5,
                    order=checkerboard_order(100), R=16384, inst=2, field_bytes=1,
                    desc="100x100 torus, +-1 weights seed 4, R=16384, K=1000 linear beta "
                         "0.1->4.0, S=5, checkerboard order")
    raise KeyError(name)


def batch_workloads(count: int = 64, meta_seed: int = 5, steps: int = 500) -> list:
    """A mix of uneven instances for batched runs, drawn from one SplitMix64
    stream (meta_seed): instance j is a random graph G(N, round(N d / 2)) with
    d ~ U[4, 12] for even j and an L x L torus with +-1 weights, L = round(sqrt N),
    for odd j; N ~ U[800, 7000], R ~ U[256, 4096]; K = ``steps`` linear steps,
    beta 0.1 -> 5.0 and 10 sweeps per step on random graphs (natural order),
    0.1 -> 4.0 and 5 sweeps on tori (checkerboard order). Plain population
    annealing (no noise levels, no cluster moves), run seed 42, instance id j.
    """
    u = splitmix64(meta_seed, 4 * count).astype(np.float64) / 2.0 ** 64
    out = []
    for j in range(count):
        N = 800 + int(u[4 * j] * 6201)
        R = 256 + int(u[4 * j + 1] * 3841)
        gseed = 1000 + j
        if j % 2 == 0:
            d = 4.0 + 8.0 * u[4 * j + 2]
            M = int(round(N * d / 2))
            g = random_graph(N, M, gseed, f"batch{j}-G({N},{M})")
            wl = dict(graph=g, betas=linear_betas(0.1, 5.0, steps), sweeps=10,
                      order=natural_order(g.n))
        else:
            L = int(round(np.sqrt(N)))
            g = torus(L, gseed, True, f"batch{j}-torus{L}")
            wl = dict(graph=g, betas=linear_betas(0.1, 4.0, steps), sweeps=5,
                      order=checkerboard_order(L))
        out.append(dict(wl, R=R, seed=42, inst=j, as_enable=0, as_stall_steps=20, as_max_level=4,
                        as_frozen_inv=256, as_gamma=0.8, nl_period=0,
                        desc=f"{g.name}, R={R}"))
    return out


def serve_requests(count: int = 256, meta_seed: int = 6, steps: int = 500) -> list:
    """A request stream for the serving loop, from one SplitMix64 stream
    (meta_seed): N log-uniform in [800, 20000]; half random graphs
    G(N, round(N d / 2)) with d ~ U[2, 12], half L x L tori with +-1 weights,
    L = round(sqrt N); R log-uniform in [512, 8192]; K = ``steps`` linear steps,
    5 sweeps per step, beta 0.1 -> 5.0 (random) or 0.1 -> 4.0 (torus); plain
    population annealing. Each request carries a unit-rate Poisson arrival
    time (exponential gaps with mean 1 s), to be divided by the offered rate.
    """
    u = splitmix64(meta_seed, 5 * count).astype(np.float64) / 2.0 ** 64
    t = 0.0
    out = []
    for j in range(count):
        N = int(round(np.exp(np.log(800) + u[5 * j] * (np.log(20000) - np.log(800)))))
        R = int(round(np.exp(np.log(512) + u[5 * j + 1] * (np.log(8192) - np.log(512)))))
        t += -np.log1p(-u[5 * j + 4])
        gseed = 5000 + j
        if u[5 * j + 2] < 0.5:
            d = 2.0 + 10.0 * u[5 * j + 3]
            M = int(round(N * d / 2))
            g = random_graph(N, M, gseed, f"req{j}-G({N},{M})")
            wl = dict(graph=g, betas=linear_betas(0.1, 5.0, steps), order=natural_order(g.n))
        else:
            L = int(round(np.sqrt(N)))
            g = torus(L, gseed, True, f"req{j}-torus{L}")
            wl = dict(graph=g, betas=linear_betas(0.1, 4.0, steps), order=checkerboard_order(L))
        out.append(dict(wl, sweeps=5, R=R, seed=42, inst=j, as_enable=0, as_stall_steps=20,
                        as_max_level=4, as_frozen_inv=256, as_gamma=0.8, nl_period=0,
                        arrival=t, desc=f"{g.name}, R={R}"))
    return out
