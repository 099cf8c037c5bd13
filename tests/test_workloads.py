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


def test_batch_and_request_streams_are_reproducible():
    a, b = W.serve_requests(12), W.serve_requests(12)
    assert [x["R"] for x in a] == [x["R"] for x in b]
    assert all(np.array_equal(x["graph"].col, y["graph"].col) for x, y in zip(a, b))
    arr = [x["arrival"] for x in a]
    assert all(t2 > t1 for t1, t2 in zip(arr, arr[1:]))
    for x in a:
        assert 800 * 0.9 <= x["graph"].n <= 20000 * 1.1 and 512 <= x["R"] <= 8192


def test_percentile():
    from paper_2510_21105_amd.serve import percentile
    assert percentile([3, 1, 2], 50) == 2
    assert percentile(list(range(101)), 99) == 99
