"""G-set graph files and the cut of a configuration (paper section 1).

The G-set benchmark graphs come as plain text: a first line "N M", then M
lines "i j w" giving an undirected edge between variables i and j
(1-based, 1 <= i, j <= N) with integer weight w. The paper's objective,
eq. (1), is the cut weight sum over i < j of w_ij (1 - x_i x_j) / 2 for spins
x in {-1, +1}^N. Variable v is node v - 1 of the solver.

Host-side input/output only: the annealing itself runs in the library.
"""
from __future__ import annotations

import io
import os

import numpy as np

from .workloads import Graph, from_edges


def parse(text: str, name: str = "") -> Graph:
    """Graph of a G-set text. The benchmark's weights are binary, +1 or -1
    (paper section 1), which is also all the solver accepts: other weights
    are rejected, as are self loops, repeated edges and a count of edge lines
    other than M."""
    lines = [ln.split() for ln in text.splitlines()]
    lines = [ln for ln in lines if ln and not ln[0].startswith(("#", "%"))]
    if not lines or len(lines[0]) < 2:
        raise ValueError("G-set text must start with 'N M'")
    n, m = int(lines[0][0]), int(lines[0][1])
    if n < 1 or m < 0:
        raise ValueError(f"bad header: N={n} M={m}")
    body = lines[1:]
    if len(body) != m:
        raise ValueError(f"header announces {m} edges, file has {len(body)}")
    if m == 0:
        return from_edges(n, [], [], [], name)
    if any(len(ln) < 2 for ln in body):
        raise ValueError("edge line with fewer than two fields")
    e = np.array([[int(ln[0]), int(ln[1]), int(ln[2]) if len(ln) > 2 else 1] for ln in body],
                 dtype=np.int64)
    i, j, w = e[:, 0] - 1, e[:, 1] - 1, e[:, 2]
    if np.any((i < 0) | (i >= n) | (j < 0) | (j >= n)):
        raise ValueError("variable index outside 1..N")
    if np.any(i == j):
        raise ValueError("self loop")
    if np.any(np.abs(w) != 1):
        raise ValueError("weights must be +1 or -1 (binary G-set weights)")
    lo, hi = np.minimum(i, j), np.maximum(i, j)
    key = lo * n + hi
    if np.unique(key).shape[0] != m:
        raise ValueError("repeated edge")
    return from_edges(n, lo, hi, w, name)


def load(path: str) -> Graph:
    """Read a G-set file."""
    with open(path) as f:
        return parse(f.read(), os.path.basename(path))


def dumps(g: Graph) -> str:
    """G-set text of a graph (edges with i < j, 1-based, in row order)."""
    i, j, w = g.edges()
    out = io.StringIO()
    out.write(f"{g.n} {i.shape[0]}\n")
    for a, b, c in zip(i.tolist(), j.tolist(), w.tolist()):
        out.write(f"{a + 1} {b + 1} {c}\n")
    return out.getvalue()


def save(g: Graph, path: str) -> None:
    with open(path, "w") as f:
        f.write(dumps(g))


def cut_value(g: Graph, x) -> int:
    """Eq. (1) for spins x (length N, entries -1/+1): total weight of the
    edges whose ends take different spins."""
    x = np.asarray(x).astype(np.int64)
    if x.shape != (g.n,) or np.any((x != 1) & (x != -1)):
        raise ValueError("configuration must hold N entries of -1 or +1")
    i, j, w = g.edges()
    return int(w[x[i] != x[j]].sum())
