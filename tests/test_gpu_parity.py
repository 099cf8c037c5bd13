"""Device (HIP, gfx950) vs CPU oracle: bit-exact parity through the C ABI.

Every comparison is element by element on integers: spins, energies, best
cut / configuration / location, per-step statistics and resampling counts.
"""
import os
import sys
import time

import numpy as np
import pytest

from oracle import oracle as O
from paper_2510_21105_amd import workloads as W
from tests import refs

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-parity] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pa():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_21105_amd import pa as _pa
    _pa.lib()
    return _pa


def _device_run(pa, g, params):
    s = pa.Solver(g)
    s.run(params)
    return s


def _compare(pa, g, wl, over=None, record=3, check_pop=True):
    over = dict(over or {})
    p = pa.params_from_workload(wl, record=record, **over)
    _say(f"{g.name} n={g.n} R={p.R} K={len(p.betas)} S={p.sweeps} tile={p.tile_replicas} "
         f"as={p.as_enable} nl={p.nl_period}")
    t0 = time.time()
    s = _device_run(pa, g, p)
    stats = s.step_stats()
    t1 = time.time()
    ref = O.run_workload(wl, **{k: v for k, v in over.items()
                                if k not in ("tile_replicas", "sweep_kernel")},
                         want_population=check_pop, want_counts=bool(record & 1))
    _say(f"  device {t1 - t0:.2f}s oracle {time.time() - t1:.2f}s launch={s.launch_info()}")
    assert np.array_equal(stats, ref.stats), _first_diff(stats, ref.stats)
    info = s.best_info()
    assert (info["E"], info["step"], info["sweep"], info["replica"]) == \
        (ref.best_E, ref.best_step, ref.best_sweep, ref.best_replica)
    assert np.array_equal(s.best_config(), ref.best_x)
    assert s.best_cut() == ref.best_cut
    if check_pop:
        x, E = s.population()
        assert np.array_equal(E, ref.E)
        assert np.array_equal(x, ref.x)
        if record & 2:
            assert np.array_equal(s.initial_population(), ref.x_init)
    if record & 1:
        assert np.array_equal(s.counts()[:-1], ref.counts[:-1])
    return s, ref


def _first_diff(a, b):
    idx = np.argwhere(a != b)
    if idx.size == 0:
        return "equal"
    k, f = idx[0]
    return f"first stats difference at step {k} field {f}: device {a[k]} oracle {b[k]}"


def test_small800_full_run(pa):
    """800 nodes, 4,000 edges, R=128, 50 steps 0.1->3.0, 10 sweeps/step."""
    wl = W.workload("small800")
    _compare(pa, wl["graph"], wl)


def test_brute20_matches_oracle_and_exhaustive_search(pa):
    wl = W.workload("brute20")
    s, ref = _compare(pa, wl["graph"], wl)
    assert s.best_cut() == refs.brute_force_max_cut(wl["graph"])


SHAPES = [(1, 4), (1, 8), (1, 16), (2, 16), (2, 32), (2, 64)]


@pytest.mark.parametrize("kernel,tile", SHAPES)
def test_launch_shapes_give_identical_results(pa, kernel, tile):
    """Results do not depend on the sweep kernel or replicas per workgroup (ragged R = 150)."""
    wl = dict(W.workload("small800"), R=150, betas=W.linear_betas(0.1, 3.0, 12), sweeps=4)
    _compare(pa, wl["graph"], wl, dict(sweep_kernel=kernel, tile_replicas=tile, as_enable=1,
                                       as_stall_steps=1, as_frozen_inv=4, nl_period=3))


@pytest.mark.parametrize("kernel,tile", [(1, 4), (1, 8), (2, 32)])
def test_signed_torus_launch_shapes(pa, kernel, tile):
    wl = W.workload("torus100")
    wl = dict(wl, R=100, betas=wl["betas"][:4], sweeps=3)
    _compare(pa, wl["graph"], wl, dict(sweep_kernel=kernel, tile_replicas=tile))


def test_g63_shape_truncated_with_as_and_nl(pa):
    """7,000-node G63-shaped graph, ragged R, adaptive levels and cluster moves."""
    wl = W.workload("g63like")
    wl = dict(wl, R=300, betas=wl["betas"][:8], sweeps=3, as_stall_steps=1, as_frozen_inv=8,
              nl_period=2)
    _compare(pa, wl["graph"], wl)


def test_torus_truncated_checkerboard(pa):
    wl = W.workload("torus100")
    wl = dict(wl, R=200, betas=wl["betas"][:6], sweeps=5)
    _compare(pa, wl["graph"], wl)


def test_signed_random_graph_natural_and_random_order(pa):
    base = W.random_graph(1500, 6000, 21)
    i, j, _ = base.edges()
    sgn = np.where(W.splitmix64(77, i.shape[0]) & np.uint64(1), -1, 1)
    g = W.from_edges(base.n, i, j, sgn, "signed1500")
    wl = dict(W.workload("small800"), graph=g, R=96, betas=W.linear_betas(0.2, 2.5, 10),
              sweeps=3, order=W.natural_order(g.n))
    _compare(pa, g, wl)
    order = np.random.default_rng(3).permutation(g.n).astype(np.int32)
    _compare(pa, g, dict(wl, order=order, nl_period=4))


def test_g63_shape_full_population_first_steps(pa):
    """Full R=4,096 population on the 7,000-node graph: first steps exactly."""
    wl = W.workload("g63like")
    wl = dict(wl, betas=wl["betas"][:3], nl_period=2)
    _compare(pa, wl["graph"], wl, record=1)


def test_g63_shape_benchmark_configuration_first_twenty_steps(pa):
    """The benchmark's own workload and launch shape (R = 4,096, 10 sweeps,
    noise levels, cluster moves every 10 steps) for its first 20 steps, two
    of them with cluster moves: population, energies, statistics, copy counts
    and best record equal the oracle's."""
    wl = W.workload("g63like")
    wl = dict(wl, betas=wl["betas"][:20])
    s, ref = _compare(pa, wl["graph"], wl, record=1)
    assert s.launch_info()["threads"] == 448


def test_g63_shape_benchmark_configuration_late_schedule(pa):
    """The benchmark's workload and launch shape (R = 4,096, 448 threads, 10
    sweeps, cluster moves every 10 steps) over a 20-step window from the end
    of its schedule (every 10th inverse temperature from 4.51 to 4.98): a
    quench in which the noise level rises (one stall step) and falls back,
    with two cluster moves. Everything equals the oracle."""
    wl = W.workload("g63like")
    wl = dict(wl, betas=wl["betas"][-200::10], as_stall_steps=1)
    s, ref = _compare(pa, wl["graph"], wl, record=1)
    assert s.launch_info()["threads"] == 448 and s.launch_info()["tile_replicas"] == 8
    lv = ref.stats[:, 4]
    assert lv.max() >= 1 and np.any(np.diff(lv) < 0)


def test_step_stats_fill_exactly_k_rows(pa):
    """pa_get_step_stats writes K * PA_STAT_FIELDS int64 and nothing past them."""
    import ctypes
    wl = dict(W.workload("small800"), betas=W.workload("small800")["betas"][:7])
    s = _device_run(pa, wl["graph"], pa.params_from_workload(wl))
    K, F = 7, pa.STAT_FIELDS
    guard = np.int64(0x5A5A5A5A5A5A5A5A)
    buf = np.full(K * F + 16, guard, dtype=np.int64)
    assert pa.lib().pa_get_step_stats(s._h, ctypes.c_void_p(buf.ctypes.data)) == pa.PA_OK
    assert np.all(buf[K * F:] == guard)
    assert np.array_equal(buf[:K * F].reshape(K, F), s.step_stats())
    assert not np.any(buf[:K * F] == guard)


def test_torus_full_population_first_step(pa):
    wl = W.workload("torus100")
    wl = dict(wl, betas=wl["betas"][:2])
    _compare(pa, wl["graph"], wl, record=0)


# ------------------------------------------------- device statistics ----

def test_device_samples_boltzmann_and_estimates_free_energy(pa):
    """The device's own statistics, independent of the oracle (another seed
    than the oracle's pins): at fixed beta the population of an 8-node signed
    graph follows exp(-beta E) / Z (chi-square over all 256 states, the wrong
    exponent rejected), and the PA free-energy estimator from the device's
    per-step weight sums reproduces ln Z of a 12-node graph by enumeration."""
    import math
    g = W.from_edges(8, [0, 0, 1, 2, 3, 4, 5, 6, 1, 2, 0, 3],
                     [1, 2, 3, 4, 5, 6, 7, 7, 5, 6, 7, 6],
                     [1, -1, 1, 1, -1, 1, 1, -1, 1, 1, -1, 1])
    beta, R = 0.6, 32768
    wl = dict(W.workload("small800"), graph=g, R=R, betas=[beta], sweeps=64, seed=17, inst=0,
              order=None, nl_period=0, as_enable=0)
    s = pa.Solver(g).run(pa.params_from_workload(wl))
    x, _ = s.population()
    E = refs.all_energies(g)
    prob = np.exp(-beta * (E - E.min()))
    prob /= prob.sum()
    obs = np.bincount(refs.state_index(x), minlength=prob.shape[0])
    chi2 = float(((obs - R * prob) ** 2 / (R * prob)).sum())
    assert chi2 < 400.0                    # 255 degrees of freedom: about 6 sd
    bad = np.exp(-0.5 * beta * (E - E.min()))
    bad /= bad.sum()
    assert float(((obs - R * bad) ** 2 / (R * bad)).sum()) > 2000.0
    g = W.random_graph(12, 30, 9)
    betas = W.linear_betas(0.0, 1.5, 31)
    R = 20000
    wl = dict(W.workload("small800"), graph=g, R=R, betas=betas, sweeps=5, seed=23, inst=0,
              order=None, nl_period=0, as_enable=0)
    st = pa.Solver(g).run(pa.params_from_workload(wl)).step_stats()
    est = g.n * math.log(2.0)
    for k in range(len(betas) - 1):
        est += math.log(float(st[k, 7]) / (R * 2.0 ** 32)) - (betas[k + 1] - betas[k]) * float(st[k, 0])
    E = refs.all_energies(g)
    b = betas[-1]
    exact = float(np.log(np.exp(-b * (E - E.min())).sum()) - b * E.min())
    assert abs(est - exact) < 0.03


# ---------------------------------------------------------------- edges ----

def test_single_replica_and_single_step(pa):
    g = W.random_graph(200, 600, 5)
    wl = dict(W.workload("small800"), graph=g, R=1, betas=[1.0], sweeps=3,
              order=W.natural_order(g.n))
    _compare(pa, g, wl)


def test_two_nodes_and_isolated_nodes(pa):
    g = W.from_edges(2, [0], [1], None, "K2")
    wl = dict(W.workload("small800"), graph=g, R=4, betas=W.linear_betas(0.1, 2.0, 5),
              sweeps=2, order=None, nl_period=1)
    _compare(pa, g, wl)
    g2 = W.from_edges(50, [0, 1, 2], [1, 2, 3], None, "sparse50")   # 46 isolated nodes
    wl2 = dict(wl, graph=g2, R=70, nl_period=2)
    _compare(pa, g2, wl2)


def test_beta_zero_negates(pa):
    g = W.random_graph(300, 900, 6)
    wl = dict(W.workload("small800"), graph=g, R=65, betas=[0.0], sweeps=1,
              order=W.natural_order(g.n))
    s, ref = _compare(pa, g, wl)
    x, _ = s.population()
    assert np.array_equal(x, -s.initial_population())


def test_workspace_too_small_is_rejected(pa):
    import torch
    wl = W.workload("small800")
    s = pa.Solver(wl["graph"])
    p = pa.params_from_workload(wl)
    ws = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(pa.PAError) as e:
        s.run(p, workspace=ws)
    assert e.value.status == pa.PA_EWORKSPACE


def test_results_before_run_are_rejected(pa):
    s = pa.Solver(W.cycle(10))
    with pytest.raises(pa.PAError) as e:
        s.best_cut()
    assert e.value.status == pa.PA_ESTATE


def test_hex_export_matches_config(pa):
    from paper_2510_21105_amd.hexcfg import hex_to_config
    wl = W.workload("brute20")
    s = _device_run(pa, wl["graph"], pa.params_from_workload(wl))
    assert np.array_equal(hex_to_config(s.best_config_hex(), wl["graph"].n), s.best_config())


# ----------------------------------------------------------- full size ----

def test_g63_shape_full_run_properties(pa):
    """The whole 2,000-step G63-shaped run in the benchmark's launch shape.

    The oracle cannot replay 5.7e11 attempts here; the checks are properties
    that hold at any size: every tracked energy equals the energy recomputed
    from the spins, the best cut equals eq. (1) of the best configuration,
    the population stays at R and the best never worsens.
    """
    wl = W.workload("g63like")
    g = wl["graph"]
    p = pa.params_from_workload(wl)
    t0 = time.time()
    s = _device_run(pa, g, p)
    cut = s.best_cut()
    _say(f"g63like full run {time.time() - t0:.1f}s best cut {cut} launch={s.launch_info()}")
    x, E = s.population()
    i, j, w = g.edges()
    for a in range(0, p.R, 512):
        xb = x[a:a + 512].astype(np.int64)
        assert np.array_equal((xb[:, i] * xb[:, j] * w[None, :]).sum(axis=1), E[a:a + 512])
    bx = s.best_config()
    assert refs.cut_eq1(g, bx) == cut
    st = s.step_stats()
    assert np.all(np.diff(st[:, 5]) <= 0) and st[-1, 5] == s.best_info()["E"]
    assert np.all(st[:-1, 6] >= 1) and np.all(st[:-1, 6] <= p.R)
    assert np.all((st[:, 4] >= 0) & (st[:, 4] <= p.as_max_level))
    assert int(E.min()) >= s.best_info()["E"]
    assert cut > 26000   # G63-shaped graphs reach ~27,000 (paper: 27,047 on G63)


def _hub_graph():
    """Random graph plus one hub of degree > 30 (neighbours beyond the
    register-held block columns are read from global memory)."""
    base = W.random_graph(300, 900, 6)
    i, j, w = base.edges()
    hub = np.arange(1, 300, 7)                    # 43 neighbours of node 0
    keep = (i != 0) & (j != 0)
    ii = np.concatenate([i[keep], np.zeros(hub.size, np.int64)])
    jj = np.concatenate([j[keep], hub])
    sgn = np.where(W.splitmix64(11, ii.size) & np.uint64(1), -1, 1)
    return W.from_edges(300, ii, jj, sgn, "hub300")


BLOCK_CLASSES = {
    "deg4": lambda: W.torus(10, 7, True, "torus10"),
    "deg8": lambda: W.random_graph(400, 600, 2),
    "deg13": lambda: W.random_graph(300, 900, 6),
    "deg19": lambda: W.random_graph(1500, 6000, 21),
    "deg27": lambda: W.random_graph(600, 4000, 5),
    "hub": _hub_graph,
}


@pytest.mark.parametrize("cls", sorted(BLOCK_CLASSES))
def test_every_adjacency_block_size(pa, cls):
    """Maximum degrees in each adjacency-block size class (<= 4, <= 8, <= 16,
    <= 24, <= 30, > 30) through the node-per-lane kernel."""
    g = BLOCK_CLASSES[cls]()
    _say(f"{cls}: n={g.n} dmax={g.degrees().max()}")
    wl = dict(W.workload("small800"), graph=g, R=72, betas=W.linear_betas(0.2, 2.5, 5),
              sweeps=2, order=W.natural_order(g.n), nl_period=2)
    for tile in (4, 8):
        _compare(pa, g, wl, dict(sweep_kernel=1, tile_replicas=tile))


def _cycle_with_hub(n: int, deg: int):
    """Signed cycle on n nodes plus chords from node 0 to deg - 2 others, so
    node 0 has degree deg and every other node degree 2 or 3."""
    i = list(range(n))
    j = [(k + 1) % n for k in range(n)]
    targets = np.linspace(2, n - 2, deg - 2).round().astype(int)
    assert len(set(targets.tolist())) == deg - 2
    i += [0] * (deg - 2)
    j += targets.tolist()
    sgn = np.where(W.splitmix64(17 + deg, len(i)) & np.uint64(1), -1, 1)
    return W.from_edges(n, np.array(i), np.array(j), sgn, f"cyclehub{deg}")


@pytest.mark.parametrize("deg", [5, 8, 9, 12, 13, 16, 17, 20, 21, 24, 25, 28, 29, 30, 31, 33])
def test_hub_degree_at_every_read_boundary(pa, deg):
    """The node-per-lane kernel reads adjacency entries in groups sized by the
    largest degree in a wave; every lane of the hub's wave reads that many
    entries of its own block. One hub degree on each side of every group
    boundary, both tile widths, against the oracle."""
    g = _cycle_with_hub(160, deg)
    assert int(g.degrees().max()) == deg
    wl = dict(W.workload("small800"), graph=g, R=72, betas=W.linear_betas(0.2, 2.5, 4),
              sweeps=2, order=W.natural_order(g.n), nl_period=0)
    for tile in (4, 8):
        _compare(pa, g, wl, dict(sweep_kernel=1, tile_replicas=tile))


def test_tiny_inverse_temperatures(pa):
    """beta = 0 and 1e-20 (every uphill move accepted), 1e-17 (exp rounds to 1
    for the smallest moves only: served by the word kernel), then normal."""
    g = W.random_graph(800, 4000, 1, "small800")
    wl = dict(W.workload("small800"), R=70, betas=[0.0, 1e-20, 0.3], sweeps=2)
    s, _ = _compare(pa, g, wl, dict(sweep_kernel=1))
    assert s.launch_info()["sweep_kernel"] == 1
    s, _ = _compare(pa, g, dict(wl, betas=[1e-20, 1e-17, 0.3]))
    assert s.launch_info()["sweep_kernel"] == 2


def test_batched_runs_equal_solo_runs(pa):
    """Runs enqueued together on two streams give exactly the results of
    the same runs alone (uneven random graphs and tori, K = 12)."""
    import torch
    wls = W.batch_workloads(6, steps=12)
    params = [pa.params_from_workload(w, R=min(w["R"], 700)) for w in wls]
    solvers = [pa.Solver(w["graph"]) for w in wls]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    pa.run_batch(solvers, params, streams)
    for w, p, s in zip(wls, params, solvers):
        solo = pa.Solver(w["graph"]).run(p)
        _say(f"batch vs solo {w['desc']} cut {s.best_cut()}")
        assert s.best_cut() == solo.best_cut()
        assert s.best_info() == solo.best_info()
        assert np.array_equal(s.best_config(), solo.best_config())
        assert np.array_equal(s.step_stats(), solo.step_stats())
        x1, E1 = s.population()
        x2, E2 = solo.population()
        assert np.array_equal(E1, E2) and np.array_equal(x1, x2)
    # every instance also matches the oracle: statistics, population, best
    for w, p, s in zip(wls, params, solvers):
        ref = O.run_workload(dict(w, R=p.R), want_counts=False)
        assert np.array_equal(s.step_stats(), ref.stats), w["desc"]
        x, E = s.population()
        assert np.array_equal(E, ref.E) and np.array_equal(x, ref.x), w["desc"]
        info = s.best_info()
        assert (info["E"], info["step"], info["sweep"], info["replica"]) == \
            (ref.best_E, ref.best_step, ref.best_sweep, ref.best_replica), w["desc"]
        assert np.array_equal(s.best_config(), ref.best_x), w["desc"]


def test_batch_with_adaptive_runs_interleaves_and_equals_oracle(pa):
    """A batch holding adaptive-step runs is enqueued in 64-step chunks, one
    chunk of each run in turn: every run, adaptive (ending at different steps)
    or plain (K = 150, three chunks), equals the same run alone and the
    oracle."""
    import torch
    mk = []
    for j, (n, m, jump, num, den) in enumerate([(500, 2500, 16, 1, 4), (700, 2100, 8, 1, 2),
                                                (400, 2000, 64, 0, 1)]):
        g = W.random_graph(n, m, 40 + j)
        mk.append(dict(W.workload("small800"), graph=g, R=96 + 32 * j, betas=W.linear_betas(0.1, 3.0, 200),
                       sweeps=2, order=W.natural_order(g.n), beta_adapt=1, adapt_jump=jump,
                       adapt_num=num, adapt_den=den, inst=j, desc=f"adaptive {j}"))
    g = W.random_graph(600, 2400, 44)
    mk.append(dict(W.workload("small800"), graph=g, R=80, betas=W.linear_betas(0.1, 3.0, 150), sweeps=2,
                   order=W.natural_order(g.n), inst=3, desc="plain K=150"))
    params = [pa.params_from_workload(w) for w in mk]
    solvers = [pa.Solver(w["graph"]) for w in mk]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    _say("batch with adaptive runs")
    pa.run_batch(solvers, params, streams)
    for w, p, s in zip(mk, params, solvers):
        solo = pa.Solver(w["graph"]).run(p)
        assert np.array_equal(s.step_stats(), solo.step_stats()), w["desc"]
        assert s.best_info() == solo.best_info(), w["desc"]
        ref = O.run_workload(dict(w, R=p.R), want_counts=False)
        assert np.array_equal(s.step_stats(), ref.stats), w["desc"]
        x, E = s.population()
        assert np.array_equal(E, ref.E) and np.array_equal(x, ref.x), w["desc"]
        info = s.best_info()
        assert (info["E"], info["step"], info["sweep"], info["replica"]) == \
            (ref.best_E, ref.best_step, ref.best_sweep, ref.best_replica), w["desc"]


def _fused_mix():
    wls = W.batch_workloads(6, steps=12)
    wls[2] = dict(wls[2], as_enable=1, as_stall_steps=1, as_frozen_inv=8)   # noise levels too
    return wls, [pa_params(w) for w in wls]


def pa_params(w):
    from paper_2510_21105_amd import pa as _pa
    return _pa.params_from_workload(w, R=min(w["R"], 700), record=3)


def _check_against_oracle(s, w, p):
    ref = O.run_workload(dict(w, R=p.R), want_counts=True)
    assert np.array_equal(s.step_stats(), ref.stats), w["desc"]
    x, E = s.population()
    assert np.array_equal(E, ref.E) and np.array_equal(x, ref.x), w["desc"]
    info = s.best_info()
    assert (info["E"], info["step"], info["sweep"], info["replica"]) == \
        (ref.best_E, ref.best_step, ref.best_sweep, ref.best_replica), w["desc"]
    assert np.array_equal(s.best_config(), ref.best_x), w["desc"]
    assert np.array_equal(s.counts()[:-1], ref.counts[:-1]), w["desc"]
    assert np.array_equal(s.initial_population(), ref.x_init), w["desc"]


def test_fused_batch_equals_oracle(pa):
    """Uneven random graphs and signed tori sharing launches (one sweep launch
    and one epilogue launch per step for each record mode): every run equals
    the oracle in statistics, population, best record, configuration, copy
    counts and initial population."""
    wls, params = _fused_mix()
    solvers = [pa.Solver(w["graph"]) for w in wls]
    fb = pa.FusedBatch(solvers, params)
    info = fb.info()
    _say(f"fused groups {info}")
    assert {g["record_mode"] for g in info} == {0, 2}
    assert sum(g["runs"] for g in info) == len(wls)
    fb.run()
    for w, p, s in zip(wls, params, solvers):
        _check_against_oracle(s, w, p)


def test_fused_batch_tuned_graph_replays_equal_eager(pa):
    """After the autotuner picks each group's shape, the HIP-graph step loop
    replayed three times (with eager runs and synchronisations between) and
    the same launches enqueued directly all give identical results, equal to
    each run alone."""
    import torch
    wls, params = _fused_mix()
    solvers = [pa.Solver(w["graph"]) for w in wls]
    fb = pa.FusedBatch(solvers, params)
    info = fb.tune(probe_steps=2)
    _say(f"tuned groups {info}")
    assert all(g["fs_per_attempt"] > 0 for g in info)
    solo = [pa.Solver(w["graph"]).run(p) for w, p in zip(wls, params)]
    want = [(s.step_stats(), s.population(), s.best_info()) for s in solo]

    def same():
        for s, (st, (x, E), bi) in zip(solvers, want):
            assert np.array_equal(s.step_stats(), st)
            x2, E2 = s.population()
            assert np.array_equal(E2, E) and np.array_equal(x2, x)
            assert s.best_info() == bi

    for rep in range(3):
        fb.run()
        torch.cuda.synchronize()
        same()
        pa.Solver(wls[0]["graph"]).run(params[0])      # unrelated eager work in between
        torch.cuda.synchronize()
    fb.set_graph(False)
    fb.run()
    same()


def test_fused_batch_rejects_runs_it_cannot_share(pa):
    wl = dict(W.workload("small800"), nl_period=3)
    s = pa.Solver(wl["graph"])
    with pytest.raises(pa.PAError) as e:
        pa.FusedBatch([s], [pa.params_from_workload(wl)])
    assert e.value.status == pa.PA_EINVAL and "non-local" in str(e.value)


def test_greedy_coloring_order(pa):
    """Colour-class order (few dependency levels) on a signed and an unsigned graph."""
    g = W.random_graph(800, 4000, 1, "small800")
    wl = dict(W.workload("small800"), R=96, betas=W.linear_betas(0.1, 3.0, 10), sweeps=4,
              order=W.coloring_order(g), as_enable=1, as_stall_steps=1, as_frozen_inv=4, nl_period=3)
    s, _ = _compare(pa, g, wl)
    assert s.launch_info()["levels"] <= 12
    t = W.torus(20, 5, True, "torus20")
    _compare(pa, t, dict(wl, graph=t, order=W.coloring_order(t)))


def test_served_requests_equal_solo_runs(pa):
    """Requests served concurrently under a workspace budget that forces
    queueing give the results of the same runs alone."""
    from paper_2510_21105_amd import serve as S
    reqs = W.serve_requests(6, steps=6)
    items = []
    for j, r in enumerate(reqs):
        g = W.random_graph(min(r["graph"].n, 1500), min(r["graph"].n_edges, 4000), 300 + j)
        items.append((g, pa.params_from_workload(dict(r, graph=g, order=None), R=min(r["R"], 600))))
    needs = [pa.Solver(g).workspace_bytes(p) + 256 for g, p in items]
    srv = S.Server(hbm_budget=int(2.5 * max(needs)), n_streams=3)
    res = srv.serve([S.Request(j, g, p, 0.0) for j, (g, p) in enumerate(items)], realtime=False)
    assert sorted(r.rid for r in res) == list(range(len(items)))
    for r in res:
        g, p = items[r.rid]
        solo = pa.Solver(g).run(p)
        assert r.best_cut == solo.best_cut() and r.best_E == solo.best_info()["E"]
        # and the oracle's run of the same request: statistics, best record, configuration
        ref = O.run(g, p.betas, p.sweeps, p.R, p.seed, p.inst, p.order, want_population=False,
                    want_counts=False)
        assert np.array_equal(r.stats, ref.stats), r.rid
        assert r.best_info == dict(E=ref.best_E, step=ref.best_step, sweep=ref.best_sweep,
                                   replica=ref.best_replica), r.rid
        assert np.array_equal(r.best_x, ref.best_x) and r.best_cut == ref.best_cut, r.rid
    # the last request is still waiting when cancelled; the others are unchanged
    res2 = srv.serve([S.Request(j, g, p, 0.0) for j, (g, p) in enumerate(items)], realtime=False,
                     cancel=[(0.0, len(items) - 1)])
    got = {r.rid: r for r in res2}
    assert got[len(items) - 1].cancelled and sorted(got) == list(range(len(items)))
    for r in res:
        if r.rid != len(items) - 1:
            assert not got[r.rid].cancelled and got[r.rid].best_cut == r.best_cut


def test_pool_server_continuous_batching_equals_oracle(pa):
    """Requests served by the resident pool (each iteration one step of every
    admitted request in shared launches; a budget that holds about two of
    them, so requests wait, join as others leave, and run at different steps
    side by side): every result equals the oracle's run of the request, with
    a cancellation of a request that is still waiting."""
    from paper_2510_21105_amd import serve as S
    reqs = W.serve_requests(7, steps=9)
    items = []
    for j, r in enumerate(reqs):
        if j % 2:
            L = 10 + 3 * j
            g = W.torus(L, 40 + j, True, f"torus{L}")
            order = W.checkerboard_order(L)
        else:
            g = W.random_graph(min(r["graph"].n, 1500), min(r["graph"].n_edges, 4000), 300 + j)
            order = None
        items.append((g, pa.params_from_workload(dict(r, graph=g, order=order), R=min(r["R"], 600))))
    needs = [pa.Solver(g).workspace_bytes(p) for g, p in items]
    budget = int(2.3 * max(needs)) + (11 << 20)      # runs + the lanes' argument tables
    srv = S.PoolServer(hbm_budget=budget)
    res = srv.serve([S.Request(j, g, p, 0.0) for j, (g, p) in enumerate(items)], realtime=False,
                    cancel=[(0.0, len(items) - 1)])
    got = {r.rid: r for r in res}
    assert sorted(got) == list(range(len(items)))
    assert got[len(items) - 1].cancelled
    for rid, r in got.items():
        if r.cancelled:
            continue
        g, p = items[rid]
        ref = O.run(g, p.betas, p.sweeps, p.R, p.seed, p.inst, p.order, want_population=False,
                    want_counts=False)
        assert np.array_equal(r.stats, ref.stats), rid
        assert r.best_info == dict(E=ref.best_E, step=ref.best_step, sweep=ref.best_sweep,
                                   replica=ref.best_replica), rid
        assert np.array_equal(r.best_x, ref.best_x) and r.best_cut == ref.best_cut, rid


def _edge_runs():
    """Degenerate runs: one replica and one step, a 2-node graph, isolated
    nodes, inverse temperature 0, a ragged population of 65 and a signed
    torus of 3 x 3."""
    base = dict(W.workload("small800"), nl_period=0, as_enable=0)
    out = []
    g = W.random_graph(200, 600, 5)
    out.append(dict(base, graph=g, R=1, betas=[1.0], sweeps=3, order=W.natural_order(g.n), inst=0))
    g = W.from_edges(2, [0], [1], None, "K2")
    out.append(dict(base, graph=g, R=4, betas=W.linear_betas(0.1, 2.0, 5), sweeps=2, order=None, inst=1))
    g = W.from_edges(50, [0, 1, 2], [1, 2, 3], None, "sparse50")
    out.append(dict(base, graph=g, R=70, betas=W.linear_betas(0.1, 2.0, 5), sweeps=2, order=None, inst=2))
    g = W.random_graph(300, 900, 6)
    out.append(dict(base, graph=g, R=65, betas=[0.0, 0.0], sweeps=1, order=W.natural_order(g.n), inst=3))
    g = W.torus(3, 7, True, "torus3")
    out.append(dict(base, graph=g, R=33, betas=W.linear_betas(0.1, 3.0, 4), sweeps=2,
                    order=W.checkerboard_order(3), inst=4))
    return out


def _check_stats_best(s, w, p):
    ref = O.run_workload(dict(w, R=p.R), want_counts=False)
    assert np.array_equal(s.step_stats(), ref.stats), w["graph"].name
    x, E = s.population()
    assert np.array_equal(E, ref.E) and np.array_equal(x, ref.x), w["graph"].name
    info = s.best_info()
    assert (info["E"], info["step"], info["sweep"], info["replica"]) == \
        (ref.best_E, ref.best_step, ref.best_sweep, ref.best_replica), w["graph"].name
    assert np.array_equal(s.best_config(), ref.best_x), w["graph"].name


def test_fused_batch_degenerate_runs_equal_oracle(pa):
    """A fused batch of degenerate runs (R = 1 with K = 1, a 2-node graph,
    isolated nodes, beta = 0, a ragged R, a 3 x 3 signed torus) equals the
    oracle run by run, untuned and tuned."""
    wls = _edge_runs()
    params = [pa.params_from_workload(w) for w in wls]
    solvers = [pa.Solver(w["graph"]) for w in wls]
    fb = pa.FusedBatch(solvers, params)
    _say(f"fused degenerate {fb.info()}")
    fb.run()
    for w, p, s in zip(wls, params, solvers):
        _check_stats_best(s, w, p)
    fb.tune(probe_steps=1)
    fb.run()
    for w, p, s in zip(wls, params, solvers):
        _check_stats_best(s, w, p)


def test_pool_degenerate_runs_equal_oracle(pa):
    """The same degenerate runs served by the resident pool equal the oracle."""
    from paper_2510_21105_amd import serve as S
    wls = _edge_runs()
    items = [(w["graph"], pa.params_from_workload(w)) for w in wls]
    srv = S.PoolServer(hbm_budget=64 << 20)
    res = srv.serve([S.Request(j, g, p, 0.0) for j, (g, p) in enumerate(items)], realtime=False)
    got = {r.rid: r for r in res}
    assert sorted(got) == list(range(len(items)))
    for rid, r in got.items():
        g, p = items[rid]
        ref = O.run(g, p.betas, p.sweeps, p.R, p.seed, p.inst, p.order, want_population=False,
                    want_counts=False)
        assert np.array_equal(r.stats, ref.stats), g.name
        assert r.best_info == dict(E=ref.best_E, step=ref.best_step, sweep=ref.best_sweep,
                                   replica=ref.best_replica), g.name
        assert np.array_equal(r.best_x, ref.best_x) and r.best_cut == ref.best_cut, g.name


def test_pool_runs_at_different_steps_share_launches(pa):
    """Two runs of one launch shape (one lane) admitted three iterations apart
    advance in the same launches at different steps, beside a signed torus in
    a lane of its own; each equals the oracle, population included."""
    import torch
    wl = W.workload("small800")
    a = dict(wl, R=96, betas=wl["betas"][:8])
    b = dict(wl, R=70, betas=W.linear_betas(0.2, 2.0, 6), sweeps=3, inst=5, seed=7)
    c = dict(wl, graph=W.torus(12, 3, True, "torus12"), order=W.checkerboard_order(12), R=70,
             betas=W.linear_betas(0.2, 2.0, 5), sweeps=3, inst=6)
    pool = pa.Pool(64 << 20)
    st = torch.cuda.Stream()
    sa, sb, sc = pa.Solver(a["graph"]), pa.Solver(b["graph"]), pa.Solver(c["graph"])
    ta = pool.submit(sa, pa.params_from_workload(a))
    assert pool.advance(st, 3) == 3
    torch.cuda.synchronize()
    tb = pool.submit(sb, pa.params_from_workload(b))
    tc = pool.submit(sc, pa.params_from_workload(c))
    steps = 3
    while pool.info()["stepping"] or pool.info()["waiting"]:
        n = pool.advance(st, 2)
        steps += n
        if n == 0:
            time.sleep(0.001)
    torch.cuda.synchronize()
    done = set(pool.poll())
    # lane of a and b: a's 8 steps from lane iteration 0, b's 6 from 3 -> 9
    # iterations; the torus lane: 5
    assert done == {ta, tb, tc} and steps == 9 + 5
    for s, w in ((sa, a), (sb, b), (sc, c)):
        ref = O.run_workload(w)
        assert np.array_equal(s.step_stats(), ref.stats)
        x, E = s.population()
        assert np.array_equal(E, ref.E) and np.array_equal(x, ref.x)
        assert np.array_equal(s.best_config(), ref.best_x)
    for t in (ta, tb, tc):
        pool.release(t)
    assert pool.info()["bytes_in_use"] == 0
    pool.close()


def test_cluster_moves_on_a_collapsing_population(pa):
    """Cold schedule with strong resampling: replica pairs soon differ in few
    spins, so the cluster move runs on small disagreement sets (adjacency-row
    path) as well as large ones (edge-list path)."""
    wl = dict(W.workload("small800"), R=64, betas=W.linear_betas(1.5, 6.0, 24), sweeps=2,
              nl_period=1)
    _compare(pa, wl["graph"], wl)
    wl2 = dict(W.workload("g63like"), R=48, betas=W.linear_betas(2.0, 6.0, 16), sweeps=1,
               nl_period=1, as_enable=0)
    _compare(pa, wl2["graph"], wl2)


def test_torus_full_run_properties(pa):
    """The whole 1,000-step signed-torus run (R = 16,384, checkerboard order) in
    the benchmark's launch shape, checked by size-independent properties."""
    wl = W.workload("torus100")
    g = wl["graph"]
    p = pa.params_from_workload(wl)
    s = _device_run(pa, g, p)
    cut = s.best_cut()
    _say(f"torus100 full run best cut {cut} launch={s.launch_info()}")
    x, E = s.population()
    i, j, w = g.edges()
    for a in range(0, p.R, 2048):
        xb = x[a:a + 2048].astype(np.int64)
        assert np.array_equal((xb[:, i] * xb[:, j] * w[None, :]).sum(axis=1), E[a:a + 2048])
    assert refs.cut_eq1(g, s.best_config()) == cut
    st = s.step_stats()
    assert np.all(np.diff(st[:, 5]) <= 0) and st[-1, 5] == s.best_info()["E"]
    assert np.all(st[:-1, 6] >= 1) and np.all(st[:-1, 6] <= p.R)
    assert int(E.min()) >= s.best_info()["E"]
    # The +-1 square-lattice spin glass has a ground-state energy of about
    # -1.40 per spin; a 1,000-step anneal gets within about 1.5 % of it.
    e_best = s.best_info()["E"] / g.n
    _say(f"torus100 best energy per spin {e_best:.4f}")
    assert -1.45 < e_best < -1.38


def test_repeated_runs_are_identical(pa):
    """Two runs of one solver with the same inputs agree exactly; another seed differs."""
    wl = dict(W.workload("g63like"), R=256, betas=W.workload("g63like")["betas"][:20], nl_period=5)
    g = wl["graph"]
    s = pa.Solver(g)
    p = pa.params_from_workload(wl)
    s.run(p)
    a_stats, (a_x, a_E) = s.step_stats(), s.population()
    s.run(p)
    assert np.array_equal(s.step_stats(), a_stats)
    b_x, b_E = s.population()
    assert np.array_equal(a_x, b_x) and np.array_equal(a_E, b_E)
    s.run(pa.params_from_workload(wl, seed=43))
    assert not np.array_equal(s.population()[1], a_E)


@pytest.mark.parametrize("graph", ["small800", "torus20"])
def test_population_fields_are_the_local_fields_of_the_spins(pa, graph):
    """pa_get_population's h: h_i = sum_j w_ij x_j of the returned spins and
    E = (1/2) sum_i x_i h_i for every replica (eq. (1) up to W_tot), also
    for a range of steps that stops while the next population is still read
    through the resampling parents; x and E equal the two-output call. The
    torus has weights of both signs."""
    from scipy import sparse
    wl = dict(W.workload("small800"), R=192, betas=W.workload("small800")["betas"][:6])
    if graph == "torus20":
        wl = dict(wl, graph=W.torus(20, 9, True, "torus20"), order=W.checkerboard_order(20))
    g = wl["graph"]
    assert graph != "torus20" or (np.asarray(g.w) < 0).any()
    A = sparse.csr_matrix((np.asarray(g.w, dtype=np.int32), np.asarray(g.col), np.asarray(g.row_ptr)),
                          shape=(g.n, g.n))
    s = pa.Solver(g)
    p = pa.params_from_workload(wl)
    for k_end in (3, 6):
        s.run_steps(p, 0, k_end)
        x, h, E = s.population(fields=True)
        x2, E2 = s.population()
        assert np.array_equal(x, x2) and np.array_equal(E, E2)
        want = (A @ x.T.astype(np.int32)).T
        assert np.array_equal(h.astype(np.int32), want), f"fields differ after {k_end} steps"
        assert np.array_equal((x.astype(np.int64) * h).sum(axis=1), 2 * E.astype(np.int64))


def test_gset_file_command_line_solve(pa, tmp_path):
    """A G-set file through the command-line solve: its best cut and hex
    configuration equal the oracle's run of the same schedule, and the hex
    decodes to a configuration with that eq. (1) cut."""
    from paper_2510_21105_amd import gset, hexcfg, solve
    g = W.random_graph(300, 1200, 12)
    gp, hp = tmp_path / "g.txt", tmp_path / "best.hex"
    gset.save(g, str(gp))
    _say(f"solve command on {gp.name}: n={g.n} m={g.n_edges}")
    out = solve.main(["--gset", str(gp), "--replicas", "192", "--steps", "30", "--sweeps", "4",
                      "--nl-period", "5", "--instance", "3", "--hex-out", str(hp)])
    h = gset.load(str(gp))
    wl = dict(graph=h, betas=W.linear_betas(0.1, 5.0, 30), sweeps=4, order=W.natural_order(h.n),
              R=192, seed=42, inst=3, as_enable=1, as_stall_steps=20, as_max_level=4,
              as_frozen_inv=256, as_gamma=0.8, nl_period=5)
    ref = O.run_workload(wl, want_population=False, want_counts=False)
    assert out["best_cut"] == ref.best_cut
    x = hexcfg.hex_to_config(hp.read_text(), g.n)
    assert np.array_equal(x, ref.best_x)
    assert gset.cut_value(g, x) == out["best_cut"]


# ------------------------------------------- single-replica cluster move ----

def _signed(base, seed, name):
    i, j, _ = base.edges()
    sgn = np.where(W.splitmix64(seed, i.shape[0]) & np.uint64(1), -1, 1)
    return W.from_edges(base.n, i, j, sgn, name)


@pytest.mark.parametrize("kernel,tile", [(1, 4), (1, 8), (2, 16)])
def test_single_replica_cluster_moves_signed_graph(pa, kernel, tile):
    """Wolff updates after every second step on a signed random graph with an
    odd population (no pairing needed), each sweep kernel."""
    g = _signed(W.random_graph(600, 2400, 31), 78, "signed600")
    wl = dict(W.workload("small800"), graph=g, R=99, betas=W.linear_betas(0.1, 3.0, 12),
              sweeps=3, order=W.natural_order(g.n), nl_period=2, nl_kind=1)
    _compare(pa, g, wl, dict(sweep_kernel=kernel, tile_replicas=tile))


def test_single_replica_cluster_moves_torus_every_step(pa):
    wl = W.workload("torus100")
    wl = dict(wl, R=160, betas=wl["betas"][:6], sweeps=2, nl_period=1, nl_kind=1)
    _compare(pa, wl["graph"], wl)


def test_single_replica_cluster_moves_g63_shape_with_noise_levels(pa):
    """7,000-node G63-shaped graph, ragged R, adaptive levels changing the
    bond temperature between steps."""
    wl = W.workload("g63like")
    wl = dict(wl, R=300, betas=W.linear_betas(4.0, 5.0, 16), sweeps=2, as_stall_steps=1,
              as_frozen_inv=8, nl_period=2, nl_kind=1)
    s, ref = _compare(pa, wl["graph"], wl)
    lv = ref.stats[:, 4]
    assert np.any(lv[1::2] > 0)      # a cluster-move step ran at a raised level


def test_single_replica_cluster_moves_at_high_and_zero_beta(pa):
    """beta = 0 (no active bond: one spin flips per replica) and a large beta
    (nearly every satisfied bond active: large clusters)."""
    g = W.random_graph(500, 3000, 41)
    for betas in (np.zeros(4), np.full(4, 6.0)):
        wl = dict(W.workload("small800"), graph=g, R=70, betas=betas, sweeps=1,
                  order=W.natural_order(g.n), nl_period=1, nl_kind=1)
        _compare(pa, g, wl)


# ------------------------------------------------- resumable runs, checkpoints ----

def _results(s):
    x, E = s.population()
    info = s.best_info()
    return dict(stats=s.step_stats(), x=x, E=E, best=(info["E"], info["step"], info["sweep"],
                info["replica"]), bx=s.best_config())


def _assert_same(a, b):
    assert np.array_equal(a["stats"], b["stats"]), _first_diff(a["stats"], b["stats"])
    assert np.array_equal(a["x"], b["x"]) and np.array_equal(a["E"], b["E"])
    assert a["best"] == b["best"] and np.array_equal(a["bx"], b["bx"])


@pytest.mark.parametrize("over", [dict(), dict(sweep_kernel=2, tile_replicas=32),
                                  dict(nl_kind=1, nl_period=3)])
def test_split_run_equals_one_run(pa, over):
    """Steps in three ranges give exactly the one-call run (both sweep kernels,
    both kinds of non-local move), and equal the oracle."""
    wl = W.workload("g63like")
    wl = dict(wl, R=200, betas=wl["betas"][:9], sweeps=2, as_stall_steps=1, as_frozen_inv=8,
              nl_period=over.get("nl_period", 2), nl_kind=over.get("nl_kind", 0))
    kw = {k: v for k, v in over.items() if k in ("sweep_kernel", "tile_replicas")}
    p = pa.params_from_workload(wl, record=3, **kw)
    _say(f"split run {over}")
    one = pa.Solver(wl["graph"]).run(p)
    ref_one = _results(one)
    s = pa.Solver(wl["graph"])
    s.run_steps(p, 0, 4)
    mid = _results(s)                       # population the fifth step starts from
    s.run_steps(p, 4, 7).run_steps(p, 7, 9)
    _assert_same(_results(s), ref_one)
    assert np.array_equal(s.counts()[:-1], one.counts()[:-1])
    assert np.array_equal(s.initial_population(), one.initial_population())
    ref = O.run_workload(wl, want_counts=False)
    assert np.array_equal(ref_one["stats"], ref.stats) and np.array_equal(ref_one["x"], ref.x)
    # the mid-run population is a valid resampled population of the run
    i, j, w = wl["graph"].edges()
    for q in range(0, p.R, 37):
        xq = mid["x"][q].astype(np.int64)
        assert int(mid["E"][q]) == int(np.sum(w * xq[i] * xq[j]))


@pytest.mark.parametrize("kind", [0, 1])
def test_checkpoint_resume_in_new_solver_and_other_launch_shape(pa, kind):
    """Checkpoint after step 5, restore into a new solver with another launch
    shape, finish: identical to the uninterrupted run and to the oracle."""
    wl = W.workload("g63like")
    wl = dict(wl, R=160, betas=W.linear_betas(0.5, 5.0, 12), sweeps=2, as_stall_steps=1,
              as_frozen_inv=8, nl_period=3, nl_kind=kind)
    p = pa.params_from_workload(wl, record=3)
    _say(f"checkpoint kind={kind}")
    full = _results(pa.Solver(wl["graph"]).run(p))
    a = pa.Solver(wl["graph"]).run_steps(p, 0, 5)
    blob = a.checkpoint()
    assert pa.next_step(blob) == 5
    mid = _results(a)
    assert a.checkpoint() == blob                       # saving twice gives the same bytes
    a.run_steps(p, 5, 12)                               # the saved run still continues
    _assert_same(_results(a), full)
    q = pa.params_from_workload(wl, record=3, sweep_kernel=2, tile_replicas=16)
    b = pa.Solver(wl["graph"]).restore(q, blob)
    m2 = _results(b)
    assert np.array_equal(m2["x"], mid["x"]) and np.array_equal(m2["E"], mid["E"])
    b.run_steps(q, 5, 12)
    _assert_same(_results(b), full)
    ref = O.run_workload(wl, want_counts=False)
    assert np.array_equal(full["stats"], ref.stats) and np.array_equal(full["x"], ref.x)
    assert full["best"] == (ref.best_E, ref.best_step, ref.best_sweep, ref.best_replica)
    # a checkpoint of another seed or schedule is refused
    with pytest.raises(pa.PAError):
        pa.Solver(wl["graph"]).restore(pa.params_from_workload(wl, record=3, seed=43), blob)
    with pytest.raises(pa.PAError):
        pa.Solver(wl["graph"]).restore(pa.params_from_workload(dict(wl, sweeps=3), record=3), blob)


def test_injected_fault_stops_the_run_and_it_resumes(pa):
    """A fault injected at step 6 stops pa_run there with PA_EABORTED; the
    solver holds the first 6 steps, which continue in place, or through a
    checkpoint in a new solver, to the uninterrupted run's results and the
    oracle's. The hook fires once."""
    wl = W.workload("g63like")
    wl = dict(wl, R=160, betas=W.linear_betas(0.5, 5.0, 12), sweeps=2, as_stall_steps=1,
              as_frozen_inv=8, nl_period=3)
    p = pa.params_from_workload(wl, record=3)
    _say("fault injection at step 6")
    full = _results(pa.Solver(wl["graph"]).run(p))
    a = pa.Solver(wl["graph"]).set_fault_step(6)
    with pytest.raises(pa.PAError) as e:
        a.run(p)
    assert e.value.status == pa.PA_EABORTED
    blob = a.checkpoint()
    assert pa.next_step(blob) == 6
    ref6 = _results(pa.Solver(wl["graph"]).run_steps(p, 0, 6))
    got6 = _results(a)
    assert np.array_equal(got6["x"], ref6["x"]) and np.array_equal(got6["E"], ref6["E"])
    a.run_steps(p, 6, 12)
    _assert_same(_results(a), full)
    b = pa.Solver(wl["graph"]).restore(p, blob).run_steps(p, 6, 12)
    _assert_same(_results(b), full)
    a.run(p)                                             # the hook has cleared itself
    _assert_same(_results(a), full)
    ref = O.run_workload(wl, want_counts=False)
    assert np.array_equal(full["stats"], ref.stats) and np.array_equal(full["x"], ref.x)
    assert full["best"] == (ref.best_E, ref.best_step, ref.best_sweep, ref.best_replica)


def test_command_line_checkpoint_and_resume(pa, tmp_path):
    """The solve command with checkpoints every 7 steps, and resumed from a
    checkpoint taken after step 9, both give the uninterrupted run's result."""
    from paper_2510_21105_amd import gset, solve
    g = W.random_graph(400, 1600, 13)
    gp = tmp_path / "g.txt"
    gset.save(g, str(gp))
    args = ["--gset", str(gp), "--replicas", "128", "--steps", "20", "--sweeps", "3",
            "--nl-period", "4", "--instance", "5"]
    _say("solve command: plain, checkpointed, resumed")
    plain = solve.main(args)
    ck = tmp_path / "run.ckpt"
    chk = solve.main(args + ["--checkpoint", str(ck), "--checkpoint-every", "7"])
    assert (chk["best_cut"], chk["hex"]) == (plain["best_cut"], plain["hex"])
    assert pa.next_step(ck.read_bytes()) == 20
    # a checkpoint after step 9, written through the library, resumed by the command
    h = gset.load(str(gp))
    wl = dict(graph=h, betas=W.linear_betas(0.1, 5.0, 20), sweeps=3, order=W.natural_order(h.n),
              R=128, seed=42, inst=5, as_enable=1, as_stall_steps=20, as_max_level=4,
              as_frozen_inv=256, as_gamma=0.8, nl_period=4)
    s = pa.Solver(h).run_steps(pa.params_from_workload(wl), 0, 9)
    mid = tmp_path / "mid.ckpt"
    mid.write_bytes(s.checkpoint())
    res = solve.main(args + ["--resume", str(mid)])
    assert (res["best_cut"], res["hex"]) == (plain["best_cut"], plain["hex"])


# ------------------------------------------------------- adaptive steps ----

@pytest.mark.parametrize("over", [dict(), dict(sweep_kernel=2, tile_replicas=32),
                                  dict(nl_kind=1), dict(tile_replicas=4)])
def test_adaptive_steps_match_oracle(pa, over):
    """Adaptive temperature steps on the G63-shaped graph (ragged R, noise
    levels, cluster moves): grid points, jumps, every statistic, population
    and best equal the oracle's."""
    wl = W.workload("g63like")
    wl = dict(wl, R=200, betas=W.linear_betas(0.1, 5.0, 400), sweeps=2, as_stall_steps=2,
              as_frozen_inv=8, nl_period=3, nl_kind=over.get("nl_kind", 0), beta_adapt=1,
              adapt_jump=16, adapt_num=1, adapt_den=4)
    kw = {k: v for k, v in over.items() if k in ("sweep_kernel", "tile_replicas")}
    s, ref = _compare(pa, wl["graph"], wl, kw)
    steps = int(np.count_nonzero(ref.stats[:, 9])) + 1
    assert steps < len(wl["betas"]) and len(set(ref.stats[:steps - 1, 9].tolist())) > 1
    assert ref.stats[steps - 1, 8] == len(wl["betas"]) - 1


def test_adaptive_steps_end_early_and_stop_enqueueing(pa):
    """Target 0 takes the largest jumps: the run ends after a few of its 300
    possible steps; the rest are empty, as in the oracle (the host stops
    enqueueing after its first look)."""
    g = W.random_graph(500, 2500, 17)
    wl = dict(W.workload("small800"), graph=g, R=96, betas=W.linear_betas(0.1, 3.0, 300),
              sweeps=2, order=W.natural_order(g.n), beta_adapt=1, adapt_jump=64, adapt_num=0,
              adapt_den=1)
    s, ref = _compare(pa, g, wl)
    assert ref.stats[:6, 8].tolist() == [0, 64, 128, 192, 256, 299]
    assert not ref.stats[6:].any()


def test_adaptive_steps_large_ragged_population(pa):
    """R = 10,000: the resampling reads each thread's ten weights as a chunk of
    8 plus a ragged 2, and every jump test reads the table in chunks of 512
    replicas with a ragged tail."""
    g = W.random_graph(300, 1200, 19)
    wl = dict(W.workload("small800"), graph=g, R=10000, betas=W.linear_betas(0.1, 3.0, 40),
              sweeps=2, order=W.natural_order(g.n), nl_period=0, beta_adapt=1, adapt_jump=8,
              adapt_num=1, adapt_den=2)
    s, ref = _compare(pa, g, wl, record=1)
    assert len(set(ref.stats[:, 9].tolist())) > 2


def test_adaptive_steps_checkpoint_and_resume(pa):
    wl = W.workload("g63like")
    wl = dict(wl, R=128, betas=W.linear_betas(0.1, 5.0, 300), sweeps=2, nl_period=4, beta_adapt=1,
              adapt_jump=24, adapt_num=1, adapt_den=3)
    p = pa.params_from_workload(wl, record=1)
    full = _results(pa.Solver(wl["graph"]).run(p))
    a = pa.Solver(wl["graph"]).run_steps(p, 0, 30)
    blob = a.checkpoint()
    q = pa.params_from_workload(wl, record=1, sweep_kernel=2, tile_replicas=16)
    b = pa.Solver(wl["graph"]).restore(q, blob)
    b.run_steps(q, 30, len(wl["betas"]))
    _assert_same(_results(b), full)
    ref = O.run_workload(wl, want_counts=False)
    assert np.array_equal(full["stats"], ref.stats) and np.array_equal(full["x"], ref.x)


@pytest.mark.parametrize("L,R,tile", [(80, 4096, 8), (100, 16384, 4)])
def test_sign_bit_records_on_large_populations(pa, L, R, tile):
    """Signed tori with enough workgroups that kernel 1 marks negative edges by
    sign bits in the block entries (byte-offset entries in both cases) instead
    of complemented records: the whole population equals the oracle's."""
    base = W.workload("torus100")
    g = W.torus(L, 4, True, f"torus{L}")
    wl = dict(base, graph=g, order=W.checkerboard_order(L), R=R, betas=base["betas"][:2], sweeps=3)
    s, _ = _compare(pa, g, wl, dict(tile_replicas=tile), record=0)
    info = s.launch_info()
    # one record per node and replica (no complemented copies)
    assert info["lds_bytes"] < 2 * g.n * tile, info


# ------------------------------------------------------- maximum sizes ----

def _signed_ring(n: int, seed: int):
    """Ring lattice on n nodes with neighbours at distance 1 and 2 (degree 4),
    +-1 weights from the SplitMix64 stream of ``seed``."""
    i = np.concatenate([np.arange(n), np.arange(n)])
    j = np.concatenate([(np.arange(n) + 1) % n, (np.arange(n) + 2) % n])
    sgn = np.where(W.splitmix64(seed, i.shape[0]) & np.uint64(1), -1, 1)
    return W.from_edges(n, i, j, sgn, f"ring{n}")


def _max_case(name):
    if name == "R32768":
        return W.random_graph(120, 400, 31, "r120"), 32768
    if name == "n32767":
        return W.random_graph(32767, 98301, 32, "n32767"), 40
    if name == "signed32511":
        return _signed_ring(32511, 33), 40
    if name == "deg4096":
        return _cycle_with_hub(5000, 4096), 24
    raise KeyError(name)


@pytest.mark.parametrize("name", ["R32768", "n32767", "signed32511", "deg4096"])
def test_maximum_sizes(pa, name):
    """The documented limits: the largest population (R = 32,768, so 16,384
    pair moves per call), the most nodes (32,767, cluster moves with their LDS
    near full), the largest signed graph that kernel 1 holds (32,511 nodes,
    sign-bit records with bit-15 index entries) and the largest degree (4,096,
    served by the word kernel). Whole population, statistics and best record
    against the oracle, with noise levels and a cluster move every step."""
    g, R = _max_case(name)
    wl = dict(W.workload("small800"), graph=g, R=R, betas=W.linear_betas(0.3, 1.5, 3), sweeps=2,
              order=W.natural_order(g.n), nl_period=1, as_stall_steps=1, as_frozen_inv=8)
    s, _ = _compare(pa, g, wl, record=1)
    info = s.launch_info()
    if name == "signed32511":
        assert info["sweep_kernel"] == 1 and info["lds_bytes"] < 2 * g.n * info["tile_replicas"], info
    if name == "deg4096":
        assert info["sweep_kernel"] == 2, info


def test_large_torus_one_workgroup_per_cu(pa):
    """A 140 x 140 signed torus (19,600 nodes, the size of the largest G-set
    tori) with a population large enough for sign-bit records: 8-replica
    tiles of 157 KB, one per CU, run with 1,024 threads. Whole population
    against the oracle."""
    base = W.workload("torus100")
    g = W.torus(140, 81, True, "torus140")
    wl = dict(base, graph=g, order=W.checkerboard_order(140), R=4096, betas=base["betas"][:2], sweeps=2)
    s, _ = _compare(pa, g, wl, record=0)
    info = s.launch_info()
    assert info["tile_replicas"] == 8 and info["threads"] == 1024, info


def test_sweep_timing_samples_every_nth_step(pa):
    """Timing mode with stride 3 times the sweep launches of steps 0, 3, 6,
    ... only, and does not change the results."""
    wl = dict(W.workload("small800"), betas=W.workload("small800")["betas"][:10])
    p = pa.params_from_workload(wl, record=0)
    s = pa.Solver(wl["graph"])
    s.set_timing(3)
    s.run(p)
    ms, n = s.sweep_time()
    assert n == 4 and ms > 0.0
    x1, E1 = s.population()
    s.set_timing(0)
    s.run(p)
    x0, E0 = s.population()
    assert np.array_equal(x0, x1) and np.array_equal(E0, E1)
    with pytest.raises(pa.PAError) as e:
        s.sweep_time()
    assert e.value.status == pa.PA_ESTATE
