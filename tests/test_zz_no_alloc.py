"""pa_run_static (the entry point for callers that cannot allocate device
memory) against pa_run, through the C ABI: two calls in a row, the second on
a smaller input, each equal to pa_run of the same inputs in every result."""
import sys

import numpy as np
import pytest

from paper_2510_21105_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[no-alloc] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pa():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_21105_amd import pa as _pa
    _pa.lib()
    return _pa


def _results(s):
    x, E = s.population()
    return dict(stats=s.step_stats(), x=x, E=E, info=s.best_info(), bx=s.best_config(),
                cut=s.best_cut(), counts=s.counts())


def _same(a, b):
    assert np.array_equal(a["stats"], b["stats"])
    assert np.array_equal(a["E"], b["E"]) and np.array_equal(a["x"], b["x"])
    assert a["info"] == b["info"] and a["cut"] == b["cut"]
    assert np.array_equal(a["bx"], b["bx"])
    assert np.array_equal(a["counts"][:-1], b["counts"][:-1])


def test_static_workspace_runs_equal_workspace_runs(pa):
    big = dict(W.workload("g63like"), R=2048, betas=W.workload("g63like")["betas"][:6],
               nl_period=2, as_stall_steps=1, as_frozen_inv=8)
    small = dict(W.workload("small800"), R=100, betas=W.workload("small800")["betas"][:9],
                 as_enable=1, as_stall_steps=1, nl_period=3)
    for wl in (big, small):                      # second call: smaller input
        p = pa.params_from_workload(wl, record=1)
        _say(f"{wl['graph'].name} R={p.R} K={len(p.betas)}")
        a = pa.Solver(wl["graph"])
        need = a.workspace_bytes(p)
        assert need <= pa.STATIC_SCRATCH_BYTES
        a.run_static(p)
        got = _results(a)
        want = _results(pa.Solver(wl["graph"]).run(p))
        _same(got, want)
        _say(f"  equal, best cut {got['cut']}")


def test_static_workspace_refuses_runs_that_do_not_fit(pa):
    wl = W.workload("torus100")
    p = pa.params_from_workload(wl, R=32768, betas=wl["betas"][:2])
    s = pa.Solver(wl["graph"])
    assert s.workspace_bytes(p) > pa.STATIC_SCRATCH_BYTES
    with pytest.raises(pa.PAError) as e:
        s.run_static(p)
    assert e.value.status == pa.PA_EWORKSPACE and "static workspace" in str(e.value)
