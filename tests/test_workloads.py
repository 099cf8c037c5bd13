"""Host checks of the seeded synthetic inputs (no method arithmetic)."""
import numpy as np

from paper_2510_21105_amd import workloads as W


def _levels(g, order):
    pos = np.empty(g.n, dtype=np.int64)
    pos[order] = np.arange(g.n)
    lev = np.zeros(g.n, dtype=np.int64)
    for t in range(g.n):
        i = order[t]
        nb = g.col[g.row_ptr[i]:g.row_ptr[i + 1]]
        earlier = nb[pos[nb] < t]
        lev[i] = 1 + lev[earlier].max() if earlier.size else 0
    return lev


def test_coloring_order_classes_are_independent_sets():
    for g in (W.random_graph(800, 4000, 1), W.random_graph(300, 2000, 9), W.torus(9, 2, True)):
        order = W.coloring_order(g)
        assert np.array_equal(np.sort(order), np.arange(g.n))
        lev = _levels(g, order)
        i, j, _ = g.edges()
        assert np.all(lev[i] != lev[j])                     # no edge inside a level
        # first-fit colours: levels count the colours, far fewer than natural order
        assert lev.max() + 1 <= g.degrees().max() + 1
        assert lev.max() < _levels(g, W.natural_order(g.n)).max()


def test_coloring_order_of_g63_shape_has_few_levels():
    g = W.workload("g63color")["graph"]
    lev = _levels(g, W.workload("g63color")["order"])
    assert lev.max() + 1 <= 10
