"""Independent definitions used to pin the oracle (tests only).

Each is written from the mathematics, not from the oracle's code:
eq. (1) of the paper evaluated edge by edge, exhaustive search, exact
Boltzmann enumeration, textbook single-flip local search stated in cut-gain
terms, and connected components from scipy.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.csgraph as csg


def cut_eq1(g, x) -> int:
    """Section 1, eq. (1): 1/2 * sum_{i<j} w_ij (1 - x_i x_j)."""
    i, j, w = g.edges()
    x = np.asarray(x, dtype=np.int64)
    twice = int(np.sum(w * (1 - x[i] * x[j])))
    assert twice % 2 == 0
    return twice // 2


def cut_by_sides(g, side) -> int:
    """Total weight of edges whose endpoints lie on different sides."""
    i, j, w = g.edges()
    side = np.asarray(side, dtype=bool)
    return int(np.sum(w[side[i] != side[j]]))


def brute_force_max_cut(g) -> int:
    """Exhaustive max cut over all 2^(n-1) bipartitions (node 0 fixed)."""
    n = g.n
    assert n <= 22
    i, j, w = g.edges()
    best = None
    codes = np.arange(1 << (n - 1), dtype=np.int64)
    for start in range(0, codes.shape[0], 1 << 16):
        c = codes[start:start + (1 << 16)]
        bits = ((c[:, None] >> np.arange(n - 1)[None, :]) & 1).astype(np.int8)
        side = np.concatenate([np.zeros((c.shape[0], 1), np.int8), bits], axis=1)
        val = ((side[:, i] != side[:, j]) * w[None, :]).sum(axis=1)
        m = int(val.max())
        best = m if best is None else max(best, m)
    return best


def all_energies(g) -> np.ndarray:
    """Ising energy sum_{i<j} w_ij x_i x_j (section 2 mapping) of all 2^n states.

    State index s has x_i = +1 iff bit i of s is set.
    """
    n = g.n
    assert n <= 16
    i, j, w = g.edges()
    s = np.arange(1 << n, dtype=np.int64)
    x = 2 * ((s[:, None] >> np.arange(n)[None, :]) & 1) - 1
    return (x[:, i] * x[:, j] * w[None, :]).sum(axis=1)


def state_index(x) -> np.ndarray:
    """Index of +-1 configurations (rows) in the all_energies enumeration."""
    x = np.asarray(x)
    return (((x > 0).astype(np.int64)) << np.arange(x.shape[-1])[None, :]).sum(axis=1)


def greedy_local_search(g, side, order, sweeps: int) -> np.ndarray:
    """Single-flip local search for max cut, visiting nodes in ``order``.

    A node moves to the other side whenever that does not lower the cut, i.e.
    when the weight of its edges to its own side is at least the weight of its
    edges to the other side.
    """
    side = np.array(side, dtype=bool)
    rp, col, w = g.row_ptr, g.col, g.w.astype(np.int64)
    for _ in range(sweeps):
        for i in order:
            nb = col[rp[i]:rp[i + 1]]
            ww = w[rp[i]:rp[i + 1]]
            same = side[nb] == side[i]
            gain = int(ww[same].sum() - ww[~same].sum())
            if gain >= 0:
                side[i] = not side[i]
    return side


def component_of(g, mask, node) -> np.ndarray:
    """Connected component of ``node`` in the subgraph induced by ``mask``."""
    i, j, _ = g.edges()
    keep = mask[i] & mask[j]
    a = sp.coo_matrix((np.ones(int(keep.sum())), (i[keep], j[keep])), shape=(g.n, g.n))
    _, lab = csg.connected_components(a, directed=False)
    return (lab == lab[node]) & mask


def component_over_edges(n, i, j, active, node) -> np.ndarray:
    """Connected component of ``node`` in the graph on n nodes whose edges are
    (i[k], j[k]) for the k with active[k] (scipy's connected components)."""
    a = sp.coo_matrix((np.ones(int(active.sum())), (i[active], j[active])), shape=(n, n))
    _, lab = csg.connected_components(a, directed=False)
    return lab == lab[node]
