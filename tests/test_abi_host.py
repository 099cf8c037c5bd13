"""Host-side checks of the C ABI (no GPU needed, no device compute).

The library must load, export every function ``include/pa.h`` declares,
lay out ``pa_schedule`` exactly as the Python binding does, and reject
malformed graphs and schedules with the documented status codes before any
device call.
"""
import ctypes
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

from paper_2510_21105_amd import pa, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pa.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pa_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    L = pa.lib()
    names = declared_functions()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert set(names) == set(pa.EXPORTS)


def test_schedule_layout_matches_header():
    fields = [f[0] for f in pa.Schedule._fields_]
    prog = "#include <stdio.h>\n#include <stddef.h>\n#include \"pa.h\"\nint main(void){\n"
    prog += 'printf("%zu\\n", sizeof(pa_schedule));\n'
    for f in fields:
        prog += f'printf("%zu\\n", offsetof(pa_schedule, {f}));\n'
    prog += "return 0;}\n"
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "layout.c")
        exe = os.path.join(d, "layout")
        open(src, "w").write(prog)
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), src, "-o", exe])
        vals = [int(v) for v in subprocess.check_output([exe]).split()]
    assert vals[0] == ctypes.sizeof(pa.Schedule)
    for f, off in zip(fields, vals[1:]):
        assert getattr(pa.Schedule, f).offset == off, f


def test_stat_field_count_matches_header():
    """pa_get_step_stats writes K * PA_STAT_FIELDS int64: the binding and the
    oracle read rows of the same width, and the header documents every field."""
    from oracle import oracle as O
    prog = '#include <stdio.h>\n#include "pa.h"\nint main(void){printf("%d\\n", PA_STAT_FIELDS);return 0;}\n'
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "f.c")
        exe = os.path.join(d, "f")
        open(src, "w").write(prog)
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), src, "-o", exe])
        nf = int(subprocess.check_output([exe]).strip())
    assert nf == pa.STAT_FIELDS == O.STAT_FIELDS == len(pa.STAT_NAMES) == 10
    text = open(HEADER).read()
    doc = text[text.index("#define PA_STAT_FIELDS"):text.index("pa_get_step_stats(")]
    for f in range(nf):
        assert re.search(rf"\n \*\s+{f}\s", doc), f"field {f} undocumented"


def _create(n, row_ptr, col, w):
    h = ctypes.c_void_p()
    rp = np.ascontiguousarray(row_ptr, np.int32)
    c = np.ascontiguousarray(col, np.int32)
    ww = np.ascontiguousarray(w, np.int8)
    st = pa.lib().pa_create(ctypes.byref(h), n, rp.ctypes.data, c.ctypes.data, ww.ctypes.data)
    if st == 0:
        pa.lib().pa_destroy(h)
    return st


def test_create_accepts_valid_graph_and_reports_facts():
    g = W.torus(6, 3, signed=True)
    s = pa.Solver(g)
    info = s.info()
    assert info["n"] == 36 and info["nnz"] == 144 and info["dmax"] == 4
    assert info["w_tot"] == int(g.edges()[2].sum())


@pytest.mark.parametrize("case", ["asym", "self", "dup", "w0", "w2", "col", "rowptr", "rowptr0"])
def test_create_rejects_malformed_graph(case):
    g = W.cycle(5)
    rp, col, w = g.row_ptr.copy(), g.col.copy(), g.w.copy()
    if case == "asym":
        w[0] = -1
    elif case == "self":
        col[0] = 0
    elif case == "dup":
        col[1] = col[0]
    elif case == "w0":
        w[:] = 0
    elif case == "w2":
        w[3] = 2
    elif case == "col":
        col[2] = 99
    elif case == "rowptr":
        rp[2], rp[3] = rp[3], rp[2]
    elif case == "rowptr0":
        rp = rp + 1
    assert _create(5, rp, col, w) == pa.PA_EINVAL


def test_create_rejects_sizes():
    assert _create(1, [0, 0], [], []) == pa.PA_ERANGE
    assert _create(40000, np.zeros(40001, np.int32), [], []) == pa.PA_ERANGE


def _star(leaves):
    g = W.from_edges(leaves + 1, np.zeros(leaves, np.int64), np.arange(1, leaves + 1), None)
    return g.row_ptr, g.col, g.w


def test_size_limits_are_inclusive():
    """n <= 32767, degree <= 4096 and R <= 32768 are accepted at the limit and
    refused one past it."""
    assert _create(2, [0, 0, 0], [], []) == pa.PA_OK
    assert _create(32767, np.zeros(32768, np.int32), [], []) == pa.PA_OK
    assert _create(32768, np.zeros(32769, np.int32), [], []) == pa.PA_ERANGE
    assert _create(4097, *_star(4096)) == pa.PA_OK
    assert _create(4098, *_star(4097)) == pa.PA_ERANGE
    wl = W.workload("small800")
    s = pa.Solver(wl["graph"])
    assert s.workspace_bytes(pa.params_from_workload(wl, R=32768)) > 0
    with pytest.raises(pa.PAError) as e:
        s.workspace_bytes(pa.params_from_workload(wl, R=32769))
    assert e.value.status == pa.PA_ERANGE


def _bytes(s, p):
    return s.workspace_bytes(p)


def test_workspace_grows_with_population():
    wl = W.workload("small800")
    s = pa.Solver(wl["graph"])
    a = _bytes(s, pa.params_from_workload(wl, R=64))
    b = _bytes(s, pa.params_from_workload(wl, R=4096))
    assert 0 < a < b


@pytest.mark.parametrize("bad,status", [
    (dict(betas=[0.5, 0.4]), pa.PA_EINVAL),
    (dict(betas=[-0.1]), pa.PA_EINVAL),
    (dict(betas=[float("nan")]), pa.PA_EINVAL),
    (dict(betas=[float("inf")]), pa.PA_EINVAL),
    (dict(sweeps=0), pa.PA_ERANGE),
    (dict(sweeps=70000), pa.PA_ERANGE),
    (dict(R=0), pa.PA_ERANGE),
    (dict(R=40000), pa.PA_ERANGE),
    (dict(R=7, nl_period=2), pa.PA_EINVAL),
    (dict(tile_replicas=12), pa.PA_EINVAL),
    (dict(sweep_kernel=3), pa.PA_EINVAL),
    (dict(wg_threads=100), pa.PA_EINVAL),
    (dict(wg_threads=2048), pa.PA_EINVAL),
    (dict(as_enable=1, as_stall_steps=0), pa.PA_EINVAL),
    (dict(as_enable=1, as_max_level=16), pa.PA_ERANGE),
    (dict(as_enable=1, as_gamma=1.5), pa.PA_EINVAL),
    (dict(as_enable=1, as_frozen_inv=0), pa.PA_EINVAL),
    (dict(record=4), pa.PA_EINVAL),
    (dict(nl_kind=2, nl_period=2), pa.PA_EINVAL),
    (dict(beta_adapt=2), pa.PA_EINVAL),
    (dict(beta_adapt=1, adapt_jump=0), pa.PA_EINVAL),
    (dict(beta_adapt=1, adapt_jump=65), pa.PA_EINVAL),
    (dict(beta_adapt=1, adapt_num=3, adapt_den=2), pa.PA_EINVAL),
    (dict(beta_adapt=1, adapt_num=0, adapt_den=0), pa.PA_EINVAL),
    (dict(beta_adapt=1, adapt_num=1, adapt_den=70000), pa.PA_EINVAL),
    (dict(nl_kind=-1), pa.PA_EINVAL),
    (dict(field_bits=12), pa.PA_EINVAL),
    (dict(field_bits=-8), pa.PA_EINVAL),
])
def test_schedule_validation(bad, status):
    wl = W.workload("small800")
    s = pa.Solver(wl["graph"])
    with pytest.raises(pa.PAError) as e:
        _bytes(s, pa.params_from_workload(wl, **bad))
    assert e.value.status == status


def test_field_bits_checks_that_local_fields_fit():
    """field_bits 8 refuses a graph whose degree (the largest |h_i|) exceeds
    127 and accepts one up to 127; 16 accepts both (degree <= 4096); 0 checks
    nothing."""
    wl = W.workload("small800")
    small = pa.Solver(wl["graph"])
    assert small.info()["dmax"] <= 127
    for fb in (0, 8, 16):
        assert _bytes(small, pa.params_from_workload(wl, field_bits=fb)) > 0
    star = W.from_edges(200, np.zeros(199, dtype=np.int64), np.arange(1, 200), name="star200")
    big = pa.Solver(star)
    p = dict(wl, graph=star, order=W.natural_order(200))
    assert big.info()["dmax"] == 199
    for fb in (0, 16):
        assert _bytes(big, pa.params_from_workload(p, field_bits=fb)) > 0
    with pytest.raises(pa.PAError) as e:
        _bytes(big, pa.params_from_workload(p, field_bits=8))
    assert e.value.status == pa.PA_ERANGE


def test_adaptive_steps_need_an_evenly_spaced_grid():
    """A jump of j grid points is reweighted by beta_j - beta_0, the jump's own
    increase only on an evenly spaced grid: uneven grids are refused (here and
    by pa_build_tables), linear grids in FP64 are accepted, and without
    adaptive steps any non-decreasing schedule is fine."""
    wl = W.workload("small800")
    s = pa.Solver(wl["graph"])
    geo = 0.1 * 1.05 ** np.arange(60)
    for betas in (geo, np.r_[W.linear_betas(0.1, 3.0, 50), 3.2],
                  np.r_[0.0, 0.0, W.linear_betas(0.1, 1.0, 10)]):
        p = pa.params_from_workload(wl, betas=betas, beta_adapt=1)
        with pytest.raises(pa.PAError) as e:
            _bytes(s, p)
        assert e.value.status == pa.PA_EINVAL and "evenly spaced" in str(e.value)
        with pytest.raises(pa.PAError) as e:
            pa.build_tables(p, 4, 10)
        assert e.value.status == pa.PA_EINVAL
        assert _bytes(s, pa.params_from_workload(wl, betas=betas)) > 0
    for lo, hi, K in [(0.1, 5.0, 2000), (0.0, 1.5, 121), (0.2, 3.0, 41), (1e6, 1e6 + 1e-3, 300),
                      (0.7, 0.7, 9)]:
        assert _bytes(s, pa.params_from_workload(wl, betas=W.linear_betas(lo, hi, K), beta_adapt=1)) > 0


def test_single_replica_cluster_moves_take_odd_populations_and_more_scratch():
    """The pair move needs an even R; the single-replica update does not, and
    keeps one cluster bitmap per replica instead of per pair plus its bond
    thresholds."""
    wl = W.workload("small800")
    s = pa.Solver(wl["graph"])
    odd = _bytes(s, pa.params_from_workload(wl, R=7, nl_period=2, nl_kind=1))
    assert odd > 0
    pair = _bytes(s, pa.params_from_workload(wl, R=64, nl_period=2, nl_kind=0))
    single = _bytes(s, pa.params_from_workload(wl, R=64, nl_period=2, nl_kind=1))
    assert single > pair
    off = _bytes(s, pa.params_from_workload(wl, R=64, nl_period=0, nl_kind=1))
    assert off < pair


def test_order_must_be_permutation():
    wl = W.workload("small800")
    s = pa.Solver(wl["graph"])
    order = np.arange(800, dtype=np.int32)
    order[5] = 6
    with pytest.raises(pa.PAError) as e:
        _bytes(s, pa.params_from_workload(wl, order=order))
    assert e.value.status == pa.PA_EINVAL


def test_run_rejects_missing_or_misaligned_workspace_without_device_calls():
    wl = W.workload("small800")
    s = pa.Solver(wl["graph"])
    p = pa.params_from_workload(wl)
    sch, keep = s._schedule(p)
    L = pa.lib()
    st = L.pa_run(s._h, ctypes.byref(sch), p.R, p.seed, p.inst, None, 1 << 20, None)
    assert st == pa.PA_EWORKSPACE
    st = L.pa_run(s._h, ctypes.byref(sch), p.R, p.seed, p.inst, ctypes.c_void_p(4096 + 8),
                  1 << 20, None)
    assert st == pa.PA_EWORKSPACE
    st = L.pa_run(s._h, ctypes.byref(sch), p.R, p.seed, 70000, ctypes.c_void_p(4096), 1 << 20, None)
    assert st == pa.PA_ERANGE


def test_results_before_run_are_rejected():
    s = pa.Solver(W.cycle(8))
    for call in (s.best_cut, s.best_config, s.best_config_hex, s.population, s.step_stats,
                 s.launch_info):
        with pytest.raises(pa.PAError) as e:
            call()
        assert e.value.status == pa.PA_ESTATE
    assert "no completed pa_run" in pa.lib().pa_last_error().decode()


def test_auto_launch_choice_is_reported_in_workspace_plan():
    """Kernel 1 refuses graphs whose degree exceeds its byte counters."""
    g = W.complete(200)        # degree 199 > 127
    s = pa.Solver(g)
    wl = dict(W.workload("small800"), graph=g, order=None)
    with pytest.raises(pa.PAError) as e:
        _bytes(s, pa.params_from_workload(wl, sweep_kernel=1))
    assert e.value.status == pa.PA_EINVAL
    assert _bytes(s, pa.params_from_workload(wl)) > 0       # automatic choice falls back


def test_partially_saturated_threshold_row_needs_the_word_kernel():
    """beta = 1e-17: exp(-2 beta m) rounds to 1 for m = 1 but not for m = 20,
    which the 32-bit thresholds of kernel 1 cannot express."""
    wl = dict(W.workload("small800"), betas=[1e-17, 0.5])
    s = pa.Solver(wl["graph"])
    assert wl["graph"].degrees().max() == 20
    with pytest.raises(pa.PAError) as e:
        _bytes(s, pa.params_from_workload(wl, sweep_kernel=1))
    assert e.value.status == pa.PA_ERANGE
    assert _bytes(s, pa.params_from_workload(wl)) > 0          # automatic choice: kernel 2
    # a fully saturated row (every uphill threshold 2^32) stays on kernel 1
    assert _bytes(s, pa.params_from_workload(dict(wl, betas=[0.0, 1e-20, 0.5]), sweep_kernel=1)) > 0


def test_run_batch_rejects_bad_arguments_without_device_calls():
    L = pa.lib()
    s = pa.Solver(W.cycle(8))
    p = pa.params_from_workload(dict(W.workload("small800"), graph=s.graph, order=None))
    sch, keep = s._schedule(p)
    runs = (pa.BatchRun * 2)()
    runs[0] = pa.BatchRun(s._h.value, ctypes.pointer(sch), p.R, p.seed, 0, 4096, 1 << 20)
    runs[1] = pa.BatchRun(s._h.value, ctypes.pointer(sch), p.R, p.seed, 1, 8192, 1 << 20)
    streams = (ctypes.c_void_p * 1)(None)
    assert L.pa_run_batch(None, 1, streams, 1) == pa.PA_EINVAL
    assert L.pa_run_batch(runs, 0, streams, 1) == pa.PA_EINVAL
    assert L.pa_run_batch(runs, 1, streams, 0) == pa.PA_EINVAL
    assert L.pa_run_batch(runs, 2, streams, 1) == pa.PA_EINVAL          # same solver twice
    assert "two runs" in L.pa_last_error().decode()
    runs[0].workspace = 4096 + 8                                          # misaligned
    assert L.pa_run_batch(runs, 1, streams, 1) == pa.PA_EWORKSPACE
    assert "run 0" in L.pa_last_error().decode()


def test_batch_instance_mix_is_deterministic_and_in_range():
    a, b = W.batch_workloads(8), W.batch_workloads(8)
    for x, y in zip(a, b):
        assert x["graph"].n == y["graph"].n and x["R"] == y["R"]
        assert np.array_equal(x["graph"].col, y["graph"].col)
    for j, w in enumerate(a):
        assert 256 <= w["R"] <= 4096 and w["inst"] == j and len(w["betas"]) == 500
        if j % 2:
            assert w["graph"].degrees().max() == 4 and w["sweeps"] == 5
        else:
            assert 800 <= w["graph"].n <= 7000 and w["sweeps"] == 10


@pytest.mark.parametrize("name,over", [
    ("small800", {}),
    ("g63like", dict(betas=W.workload("g63like")["betas"][::50])),          # AS levels on
    ("torus100", dict(betas=np.array([0.0, 1e-20, 1e-17, 0.05, 2.0, 4.0]))),  # saturated rows
])
def test_run_tables_equal_oracle_tables(name, over):
    """The fixed-point tables a run uses (pa_build_tables) equal the oracle's,
    entry by entry: thresholds for every step and noise level, and weights."""
    from oracle import oracle as O
    wl = dict(W.workload(name), **over)
    p = pa.params_from_workload(wl)
    dmax, span = int(wl["graph"].degrees().max()), 400
    thr, wts = pa.build_tables(p, dmax, span)
    levels = p.as_max_level + 1 if p.as_enable else 1
    assert thr.shape == (len(p.betas), levels, dmax + 1) and wts.shape == (len(p.betas) - 1, span + 1)
    for k, b in enumerate(p.betas):
        for lv in range(levels):
            bl = O.level_beta(float(b), p.as_gamma, lv)
            assert int(thr[k, lv, 0]) == 1 << 32
            assert [int(v) for v in thr[k, lv, 1:]] == [O.threshold(bl, m) for m in range(1, dmax + 1)]
    for k in range(len(p.betas) - 1):
        db = float(p.betas[k + 1]) - float(p.betas[k])
        assert [int(v) for v in wts[k]] == [O.weight(db, n) for n in range(span + 1)]


@pytest.mark.parametrize("jump", [1, 5, 64])
def test_adaptive_weight_tables_equal_oracle(jump):
    """Adaptive steps use one weight table per jump j, for beta_j - beta_0."""
    from oracle import oracle as O
    wl = dict(W.workload("small800"), beta_adapt=1, adapt_jump=jump)
    p = pa.params_from_workload(wl)
    thr, wts = pa.build_tables(p, 12, 300)
    assert wts.shape == (min(jump, len(p.betas) - 1), 301)
    for j in range(1, wts.shape[0] + 1):
        db = float(p.betas[j]) - float(p.betas[0])
        assert [int(v) for v in wts[j - 1]] == [O.weight(db, n) for n in range(301)]


def test_build_tables_rejects_bad_input():
    wl = W.workload("small800")
    with pytest.raises(pa.PAError) as e:
        pa.build_tables(pa.params_from_workload(wl, betas=[0.5, 0.1]), 4, 10)
    assert e.value.status == pa.PA_EINVAL
    with pytest.raises(pa.PAError) as e:
        pa.build_tables(pa.params_from_workload(wl), 5000, 10)
    assert e.value.status == pa.PA_ERANGE


# ------------------------------------------------------------ checkpoints ----

def _sched_args(s, p):
    sch, keep = s._schedule(p)
    return sch, keep


def test_resume_and_checkpoint_errors_without_device_calls():
    """Continuing, saving or loading without a matching run fails before any
    device call."""
    wl = W.workload("small800")
    s = pa.Solver(wl["graph"])
    p = pa.params_from_workload(wl, R=64)
    sch, keep = _sched_args(s, p)
    L = pa.lib()
    n = ctypes.c_size_t()
    assert L.pa_checkpoint_bytes(s._h, ctypes.byref(n)) == pa.PA_ESTATE
    buf = ctypes.create_string_buffer(64)
    assert L.pa_checkpoint_save(s._h, buf, 64) == pa.PA_ESTATE
    ws = ctypes.c_void_p(256)     # never dereferenced: every call below fails first
    K = len(p.betas)
    assert L.pa_run_steps(s._h, ctypes.byref(sch), p.R, p.seed, p.inst, 3, K, ws, 1 << 30, None) == pa.PA_ESTATE
    assert L.pa_run_steps(s._h, ctypes.byref(sch), p.R, p.seed, p.inst, 0, K + 1, ws, 1 << 30, None) == pa.PA_EINVAL
    assert L.pa_run_steps(s._h, ctypes.byref(sch), p.R, p.seed, p.inst, 5, 4, ws, 1 << 30, None) == pa.PA_EINVAL
    for blob in (b"", b"x" * 100, b"PACKPT01" + bytes(200)):
        assert L.pa_checkpoint_load(s._h, ctypes.byref(sch), p.R, p.seed, p.inst, blob, len(blob),
                                    ws, 1 << 30, None) == pa.PA_EINVAL
    with pytest.raises(ValueError):
        pa.next_step(b"x" * 100)


def test_checkpoint_header_is_read_back():
    import struct
    hdr = b"PACKPT01" + struct.pack("<QQ8i", 1, 56, 800, 64, 50, 1, 25, 17, 0, 1)
    assert pa.next_step(hdr) == 17


def test_static_workspace_run_refuses_oversized_runs_without_device_calls():
    """pa_run_static works inside the library's fixed static workspace: a run
    needing more than PA_STATIC_SCRATCH_BYTES is refused before any device
    call, and so is a bad schedule."""
    L = pa.lib()
    text = open(HEADER).read()
    assert re.search(r"#define PA_STATIC_SCRATCH_BYTES \(64u << 20\)", text)
    assert pa.STATIC_SCRATCH_BYTES == 64 << 20
    wl = W.workload("torus100")
    s = pa.Solver(wl["graph"])
    p = pa.params_from_workload(wl, R=32768, betas=wl["betas"][:2])
    assert s.workspace_bytes(p) > pa.STATIC_SCRATCH_BYTES
    sch, keep = s._schedule(p)
    assert L.pa_run_static(s._h, ctypes.byref(sch), p.R, p.seed, p.inst, None) == pa.PA_EWORKSPACE
    assert "static workspace" in L.pa_last_error().decode()
    bad = pa.params_from_workload(wl, betas=[0.5, 0.4])
    sch, keep = s._schedule(bad)
    assert L.pa_run_static(s._h, ctypes.byref(sch), bad.R, bad.seed, bad.inst, None) == pa.PA_EINVAL
    assert L.pa_run_static(None, ctypes.byref(sch), 4, 0, 0, None) == pa.PA_EINVAL


def test_pool_admission_errors_without_device_calls():
    """pa_pool_*: the region must be aligned and hold more than the argument
    tables; submissions are validated (no cluster moves or adaptive steps, one
    run per solver, a run must fit the pool); cancel and release follow the
    run's state. No device work happens before the first advance."""
    L = pa.lib()
    h = ctypes.c_void_p()
    assert L.pa_pool_create(ctypes.byref(h), ctypes.c_void_p(4096 + 8), 1 << 30) == pa.PA_EWORKSPACE
    assert L.pa_pool_create(ctypes.byref(h), ctypes.c_void_p(4096), 1 << 20) == pa.PA_EWORKSPACE
    pool = pa.Pool(workspace=(1 << 20, 64 << 20))     # never dereferenced here
    wl = W.workload("small800")
    s = pa.Solver(wl["graph"])
    t = pool.submit(s, pa.params_from_workload(wl))
    assert pool.info()["waiting"] == 1
    with pytest.raises(pa.PAError) as e:
        pool.submit(s, pa.params_from_workload(wl))
    assert e.value.status == pa.PA_EINVAL
    s2 = pa.Solver(wl["graph"])
    for bad, status in [(dict(nl_period=2), pa.PA_EINVAL), (dict(beta_adapt=1), pa.PA_EINVAL),
                        (dict(R=32768, betas=wl["betas"]), pa.PA_EWORKSPACE)]:
        if status == pa.PA_EWORKSPACE:
            big = pa.Pool(workspace=(1 << 20, 16 << 20))
            with pytest.raises(pa.PAError) as e:
                big.submit(s2, pa.params_from_workload(wl, **bad))
            big.close()
        else:
            with pytest.raises(pa.PAError) as e:
                pool.submit(s2, pa.params_from_workload(wl, **bad))
        assert e.value.status == status
    with pytest.raises(pa.PAError) as e:
        pool.release(t)                         # waiting, not finished
    assert e.value.status == pa.PA_ESTATE
    pool.cancel(t)
    with pytest.raises(pa.PAError) as e:
        pool.cancel(t)
    assert e.value.status == pa.PA_ESTATE
    assert pool.info()["waiting"] == 0 and pool.poll() == []
    pool.close()


def test_timing_stride_validation():
    s = pa.Solver(W.cycle(10))
    s.set_timing(3)
    s.set_timing(0)
    with pytest.raises(pa.PAError) as e:
        s.set_timing(-1)
    assert e.value.status == pa.PA_EINVAL


def test_fault_step_validation_and_status_codes():
    """pa_set_fault_step takes -1 (off) or a step index; the binding's status
    codes equal the header's enum, PA_EABORTED included."""
    s = pa.Solver(W.cycle(10))
    s.set_fault_step(3).set_fault_step(0).set_fault_step(-1)
    with pytest.raises(pa.PAError) as e:
        s.set_fault_step(-2)
    assert e.value.status == pa.PA_EINVAL
    assert pa.lib().pa_set_fault_step(None, 1) == pa.PA_EINVAL
    prog = ('#include <stdio.h>\n#include "pa.h"\nint main(void){printf("%d %d %d %d %d %d %d\\n", '
            'PA_OK, PA_EINVAL, PA_ERANGE, PA_EWORKSPACE, PA_EDEVICE, PA_ESTATE, PA_EABORTED);return 0;}\n')
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "f.c")
        exe = os.path.join(d, "f")
        open(src, "w").write(prog)
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), src, "-o", exe])
        codes = [int(v) for v in subprocess.check_output([exe]).split()]
    assert codes == [pa.PA_OK, pa.PA_EINVAL, pa.PA_ERANGE, pa.PA_EWORKSPACE, pa.PA_EDEVICE,
                     pa.PA_ESTATE, pa.PA_EABORTED]
