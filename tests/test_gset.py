"""G-set file parsing, writing and the eq. (1) cut of a configuration (host)."""
import itertools
import json
import os

import numpy as np
import pytest

from paper_2510_21105_amd import gset, hexcfg, solve
from paper_2510_21105_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

# Triangle 1-2-3 plus the negative edge 3-4, written as a G-set file.
SMALL = "4 4\n1 2 1\n2 3 1\n1 3 1\n3 4 -1\n"
SMALL_EDGES = [(1, 2, 1), (2, 3, 1), (1, 3, 1), (3, 4, -1)]


def _cut_by_hand(edges, x):
    """Eq. (1) written out: sum over edges of w (1 - x_i x_j) / 2."""
    return sum(w * (1 - x[i - 1] * x[j - 1]) // 2 for i, j, w in edges)


def test_parse_small_file():
    g = gset.parse(SMALL)
    assert g.n == 4 and g.n_edges == 4
    assert g.degrees().tolist() == [2, 2, 3, 1]
    i, j, w = g.edges()
    assert sorted(zip((i + 1).tolist(), (j + 1).tolist(), w.tolist())) == sorted(
        (min(a, b), max(a, b), c) for a, b, c in SMALL_EDGES)


def test_cut_value_matches_eq1_on_every_configuration():
    g = gset.parse(SMALL)
    best = -10
    for bits in itertools.product((-1, 1), repeat=4):
        x = np.array(bits)
        c = gset.cut_value(g, x)
        assert c == _cut_by_hand(SMALL_EDGES, x)
        best = max(best, c)
    # the triangle cuts at most 2 edges; 3-4 (weight -1) is best left uncut
    assert best == 2
    assert gset.cut_value(g, np.array([1, -1, 1, -1])) == 1


def test_cut_value_of_random_graph_against_edge_loop():
    g = W.torus(7, 3, True)
    i, j, w = g.edges()
    rng = np.random.default_rng(0)
    for _ in range(5):
        x = rng.choice([-1, 1], size=g.n)
        direct = sum(int(ww) for a, b, ww in zip(i, j, w) if x[a] != x[b])
        assert gset.cut_value(g, x) == direct


@pytest.mark.parametrize("make", [lambda: W.random_graph(300, 1200, 4),
                                  lambda: W.torus(9, 5, True),
                                  lambda: W.cycle(17)])
def test_write_read_round_trip(tmp_path, make):
    g = make()
    p = tmp_path / "g.txt"
    gset.save(g, str(p))
    h = gset.load(str(p))
    assert h.n == g.n
    assert np.array_equal(h.row_ptr, g.row_ptr)
    assert np.array_equal(h.col, g.col)
    assert np.array_equal(h.w, g.w)
    assert gset.dumps(h) == p.read_text()


def test_edge_order_and_direction_do_not_matter():
    a = gset.parse(SMALL)
    b = gset.parse("4 4\n4 3 -1\n3 1 1\n2 1 1\n3 2 1\n")
    assert np.array_equal(a.col, b.col) and np.array_equal(a.w, b.w)


def test_weights_default_to_one_and_comments_are_skipped():
    g = gset.parse("# comment\n3 2\n1 2\n2 3\n")
    assert g.w.tolist() == [1, 1, 1, 1]


@pytest.mark.parametrize("text, msg", [
    ("3 2\n1 2 1\n", "announces"),
    ("3 1\n1 1 1\n", "self loop"),
    ("3 2\n1 2 1\n2 1 1\n", "repeated"),
    ("3 1\n1 4 1\n", "outside"),
    ("3 1\n0 2 1\n", "outside"),
    ("3 1\n1 2 0\n", "binary"),
    ("3 1\n1 2 200\n", "binary"),
    ("3 1\n1 2 2\n", "binary"),
    ("3 1\n1 2 -3\n", "binary"),
    ("", "start"),
])
def test_bad_files_are_rejected(text, msg):
    with pytest.raises(ValueError, match=msg):
        gset.parse(text)


def test_cut_value_rejects_bad_configurations():
    g = gset.parse(SMALL)
    with pytest.raises(ValueError):
        gset.cut_value(g, np.array([1, -1, 1]))
    with pytest.raises(ValueError):
        gset.cut_value(g, np.array([1, 0, 1, -1]))


def test_check_hex_command(tmp_path, capsys):
    g = W.random_graph(50, 200, 8)
    gp = tmp_path / "g.txt"
    gset.save(g, str(gp))
    x = np.where(np.arange(50) % 3 == 0, 1, -1)
    hp = tmp_path / "c.hex"
    hp.write_text(hexcfg.config_to_hex(x) + "\n")
    out = solve.main(["--gset", str(gp), "--check-hex", str(hp)])
    assert out["cut"] == gset.cut_value(g, x)
    assert out["ones"] == int((x > 0).sum())
    assert json.loads(capsys.readouterr().out.strip().splitlines()[-1])["cut"] == out["cut"]


def test_check_hex_reads_the_papers_configuration_format(tmp_path):
    """The G63 configuration printed in section 3 decodes to 7,000 spins with
    3,425 ones; its cut is evaluated on a G63-shaped stand-in graph (the G63
    file itself is not available)."""
    lines = [l.strip() for l in open(os.path.join(GOLDEN, "g63_config_section3.txt"))
             if l.strip() and not l.startswith("#")]
    hp = tmp_path / "g63.hex"
    hp.write_text("\n".join(lines) + "\n")
    g = W.workload("g63like")["graph"]
    gp = tmp_path / "g63like.txt"
    gset.save(g, str(gp))
    out = solve.main(["--gset", str(gp), "--check-hex", str(hp)])
    assert out["n"] == 7000 and out["ones"] == 3425
    x = hexcfg.hex_to_config("".join(lines), 7000)
    assert out["cut"] == gset.cut_value(g, x)
