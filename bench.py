"""Throughput benchmark of the population-annealing engine on one MI355X.

One benchmark step is one complete solve -- every part of the hot path
(setup, tables, initial population, all sweeps, best tracking, adaptive
noise levels, cluster moves, reweighting and resampling) -- on the G63-shaped
workload: random graph with 7,000 nodes and 41,459 edges (paper section 1),
R = 4,096 replicas, 2,000 linear inverse-temperature steps 0.1 -> 5.0,
10 sweeps per step, natural order, adaptive stochasticity and cluster moves
every 10 steps. Inputs are synthetic (seeded generator) and resident on the
device before the timed region.

Prints one JSON line: spin-flip attempts/s (= R*N*S*K per solve / time per
solve), the sweep kernel's roofline figures and the CPU oracle baseline.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
TIMING_STRIDE = 7
SWEEP_SOURCE = os.path.join(ROOT, "paper_2510_21105_amd", "csrc", "pa_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sweep_kernel_hbm_traffic_{}.json")
INSTR_FILE = os.path.join(ROOT, "profiles", "sweep_kernel_instructions_{}.json")
# 32-bit vector ALU peak: 256 CUs x 128 lanes x 2.4 GHz = 7.86e13 lane-op/s,
# the lane rate of the 157.3 TFLOP/s FP32 vector figure (128 FMA lanes per
# CU per cycle). Measured on this MI355X: a chain of independent 32-bit
# xor/add instructions issues 0.45 wave64 instructions per SIMD per cycle
# (90 % of it); 32-bit multiplies issue at half that rate.
VALU_PEAK_LANE_OPS = 256 * 128 * 2.4e9


def kernel_source_hash() -> str:
    with open(SWEEP_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def algorithmic_bytes_per_attempt(accept_rate: float, mean_degree: float, s_x=1, s_h=2) -> float:
    """Bytes the sequential method must touch per attempt with int8 spins and
    int16 fields: read x_i and h_i; on acceptance write x_i and update the
    d fields of the neighbours (read + write)."""
    return (s_x + s_h) + accept_rate * (s_x + 2 * s_h * mean_degree)


def measured_traffic_per_launch(workload: str):
    """HBM bytes per sweep launch from the committed rocprofv3 counter summary
    of this workload, or None when it is absent or was taken on a different
    kernel source."""
    try:
        with open(TRAFFIC_FILE.format(workload)) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return t.get("bytes_per_launch")


def measured_valu_per_launch(workload: str):
    """VALU wave64 instructions per sweep launch from the committed rocprofv3
    instruction-count summary of this workload, or None when it is absent or
    was taken on a different kernel source."""
    try:
        with open(INSTR_FILE.format(workload)) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return t.get("valu_wave_instructions_per_launch")


def cpu_baseline(wl, sample_steps: int):
    """The oracle, built for this host (-O3 -march=native, OpenMP over
    replicas), on the first `sample_steps` steps of the workload with a
    quarter of its replicas (the oracle's cost is linear in the replica
    count), scaled to attempts/s; plus one thread on the first 2 steps. The
    first steps sweep at the hottest inverse temperatures, where the most
    moves are accepted, so the figure leans slow against the whole anneal."""
    from oracle import oracle as O
    O.use_native_build()
    betas = wl["betas"][:sample_steps]
    R = max(1, wl["R"] // 4)
    if wl.get("nl_period", 0) and wl.get("nl_kind", 0) == 0:
        R += R & 1
    cores = O.num_threads()       # before the one-thread sample below changes it
    t0 = time.perf_counter()
    O.run_workload(wl, betas=betas, R=R, want_population=False, want_counts=False)
    dt = time.perf_counter() - t0
    attempts = R * wl["graph"].n * wl["sweeps"] * len(betas)
    one = dict(wl, R=R, betas=wl["betas"][:2], nthreads=1)
    t1 = time.perf_counter()
    O.run_workload(one, want_population=False, want_counts=False)
    dt1 = time.perf_counter() - t1
    attempts1 = one["R"] * wl["graph"].n * wl["sweeps"] * 2
    return {"value": attempts / dt, "unit": "attempts/s", "cores": cores,
            "kind": "oracle",
            "sample": f"first {len(betas)} of {len(wl['betas'])} temperature steps of the same "
                      f"workload with R={R} of its {wl['R']} replicas (N={wl['graph'].n}, "
                      f"S={wl['sweeps']}), {dt:.1f} s on the host, oracle built -O3 -march=native; "
                      f"the whole solve at this rate: {wl['R'] * wl['graph'].n * wl['sweeps'] * len(wl['betas']) / (attempts / dt):.0f} s "
                      f"(a linear extrapolation)",
            "value_1thread": attempts1 / dt1,
            "sample_1thread": f"first 2 steps with R={one['R']} on one thread, {dt1:.1f} s"}


def batch_bench(args, count: int):
    """Instances/s of a mix of uneven runs: one after another, one launch
    sequence per instance on one stream (the baseline); the same runs over
    several streams (pa_run_batch); and as a fused batch sharing launches
    (pa_fused_*: autotuned shapes, step loop as a HIP graph), the reported
    value. Every instance's statistics, population and best record must be
    identical across the three."""
    import torch
    from paper_2510_21105_amd import pa, workloads as W

    wls = W.batch_workloads(count)
    params = [pa.params_from_workload(w) for w in wls]
    solvers = [pa.Solver(w["graph"]) for w in wls]
    fused_solvers = [pa.Solver(w["graph"]) for w in wls]
    attempts = sum(p.R * w["graph"].n * p.sweeps * len(p.betas) for w, p in zip(wls, params))
    streams = [torch.cuda.Stream() for _ in range(args.streams)]
    print(f"[bench] {count} instances, {attempts:.3e} attempts per batch, {args.streams} streams",
          file=sys.stderr, flush=True)
    fb = pa.FusedBatch(fused_solvers, params)
    t0 = time.perf_counter()
    shapes = fb.tune(probe_steps=3)
    tune_s = time.perf_counter() - t0
    print(f"[bench] fused batch tuned in {tune_s:.2f} s: {shapes}", file=sys.stderr, flush=True)
    for w in range(args.warmup):
        pa.run_batch(solvers, params, streams)
        fb.run()
        torch.cuda.synchronize()
        print(f"[bench] warmup {w + 1}/{args.warmup} done", file=sys.stderr, flush=True)

    def results(sv):
        return [(s.step_stats(), s.best_info(), s.population()[1]) for s in sv]

    def same(a, b):
        return all(np.array_equal(x[0], y[0]) and x[1] == y[1] and np.array_equal(x[2], y[2])
                   for x, y in zip(a, b))

    seq, bat, fus = [], [], []
    for step in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s, p in zip(solvers, params):
            s.run(p, stream=streams[0])
        torch.cuda.synchronize()
        seq.append(time.perf_counter() - t0)
        r_seq = results(solvers)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pa.run_batch(solvers, params, streams)
        torch.cuda.synchronize()
        bat.append(time.perf_counter() - t0)
        r_bat = results(solvers)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fb.run()
        torch.cuda.synchronize()
        fus.append(time.perf_counter() - t0)
        r_fus = results(fused_solvers)
        if not (same(r_seq, r_bat) and same(r_seq, r_fus)):
            raise RuntimeError("fused, streamed and sequential runs disagree")
        print(f"[bench] timed batch {step + 1}/{args.steps}: sequential {seq[-1]:.2f} s, "
              f"streams {bat[-1]:.2f} s, fused {fus[-1]:.2f} s", file=sys.stderr, flush=True)
    t_seq, t_str, t_bat = sum(seq) / len(seq), sum(bat) / len(bat), sum(fus) / len(fus)
    cuts_bat = [s.best_cut() for s in fused_solvers]
    out = {
        "metric": "instances/s",
        "value": count / t_bat,
        "unit": "instances/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_bat * 1000.0,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"batch{count}: {count} uneven instances (even: random "
                               "G(N, N d/2), d ~ U[4,12]; odd: +-1 torus), N ~ U[800,7000], "
                               "R ~ U[256,4096], K=500, plain population annealing; fused "
                               "launches, autotuned shapes, HIP-graph step loop",
                   "instances": count, "attempts_per_batch": attempts},
        "sequential_instances_per_s": count / t_seq,
        "streams_instances_per_s": count / t_str,
        "streams": args.streams,
        "speedup_vs_sequential": t_seq / t_bat,
        "attempts_per_s": attempts / t_bat,
        "fused_groups": shapes,
        "tune_s": tune_s,
        "best_cuts_first8": cuts_bat[:8],
    }
    print(json.dumps(out), flush=True)


def serve_bench(args, count: int):
    """Serving with continuous batching (the resident pool, pa_pool_*: each
    iteration one step of every admitted request in shared launches):
    capacity with every request present, then Poisson arrivals at 0.5x and
    0.9x that capacity (p50/p99 latency); beside it the stream-per-request
    server's capacity and FIFO sequential plain PA (one request at a time) at
    0.5x. Results must equal across all of them."""
    import torch
    from paper_2510_21105_amd import pa, serve as S, workloads as W

    reqs = W.serve_requests(count)
    span = reqs[-1]["arrival"]

    def requests(rate):
        return [S.Request(j, r["graph"], pa.params_from_workload(r),
                          0.0 if rate is None else r["arrival"] / rate * (count / span))
                for j, r in enumerate(reqs)]

    budget = int(args.hbm_budget_gb * (1 << 30))

    def run(rate, server):
        t0 = time.perf_counter()
        res = server.serve(requests(rate), realtime=rate is not None)
        torch.cuda.synchronize()
        span_s = time.perf_counter() - t0
        lat = [r.latency for r in res]
        cuts = {r.rid: r.best_cut for r in res}
        return dict(requests_per_s=count / span_s, p50_s=S.percentile(lat, 50),
                    p99_s=S.percentile(lat, 99), makespan_s=span_s), cuts

    pool = S.PoolServer(budget)
    print(f"[bench] serving {count} requests, pool of {args.hbm_budget_gb} GB", file=sys.stderr,
          flush=True)
    run(None, pool)                                           # warm-up (allocator, tables)
    cap, cuts0 = run(None, pool)
    print(f"[bench] pool capacity {cap['requests_per_s']:.2f} requests/s", file=sys.stderr, flush=True)
    out_loads = {}
    for f in (0.5, 0.9):
        m, cuts = run(f * cap["requests_per_s"], pool)
        if cuts != cuts0:
            raise RuntimeError("served results depend on the mix")
        out_loads[f"{f:.1f}x"] = m
        print(f"[bench] pool offered {f:.1f}x: {m}", file=sys.stderr, flush=True)
    streams_cap, cuts = run(None, S.Server(budget, n_streams=args.streams))
    if cuts != cuts0:
        raise RuntimeError("served results depend on the server")
    print(f"[bench] stream server capacity: {streams_cap}", file=sys.stderr, flush=True)
    seq_cap, cuts = run(None, S.Server(budget, n_streams=1))
    if cuts != cuts0:
        raise RuntimeError("served results depend on the server")
    print(f"[bench] sequential plain PA (one at a time) capacity: {seq_cap}", file=sys.stderr, flush=True)
    fifo, cuts = run(0.5 * cap["requests_per_s"], S.Server(budget, n_streams=1))
    if cuts != cuts0:
        raise RuntimeError("served results depend on the mix")
    print(f"[bench] FIFO one at a time at 0.5x: {fifo}", file=sys.stderr, flush=True)
    out = {
        "metric": "requests/s",
        "value": cap["requests_per_s"],
        "unit": "requests/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": cap["makespan_s"] * 1000.0,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"serve{count}: N log-uniform [800, 20000] (half random "
                               "G(N, N d/2) with d ~ U[2,12], half +-1 tori), R log-uniform "
                               "[512, 8192], K=500, S=5, Poisson arrivals; continuous batching "
                               "in a resident pool",
                   "requests": count, "hbm_budget_gb": args.hbm_budget_gb},
        "capacity": cap,
        "offered": out_loads,
        "stream_server_capacity": streams_cap,
        "streams": args.streams,
        "sequential_capacity": seq_cap,
        "speedup_vs_sequential": cap["requests_per_s"] / seq_cap["requests_per_s"],
        "fifo_one_at_a_time_0.5x": fifo,
    }
    print(json.dumps(out), flush=True)


def copy_bandwidth_gbs(nbytes: int = 1 << 30, reps: int = 5) -> float:
    """Achievable HBM rate of a plain device copy (read + write bytes per
    second), the practical ceiling beside the nominal peak."""
    import torch
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        b.copy_(a)
    t1.record()
    torch.cuda.synchronize()
    sec = t0.elapsed_time(t1) / 1e3 / reps
    del a, b
    return 2.0 * nbytes / sec / 1e9


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3, help="timed solves")
    ap.add_argument("--warmup", type=int, default=1, help="untimed solves")
    ap.add_argument("--workload", default="g63like",
                    help="g63like, g63color, g63wolff, torus100, small800, batchN (N uneven "
                         "instances) or serveN (N served requests)")
    ap.add_argument("--streams", type=int, default=8, help="streams for batchN / serveN (1..32)")
    ap.add_argument("--hbm-budget-gb", type=float, default=32.0,
                    help="workspace budget of concurrent runs for serveN")
    ap.add_argument("--sweep-kernel", type=int, default=0,
                    help="0 automatic, 1 node-per-lane byte records, 2 replica-per-lane bit words")
    ap.add_argument("--tile", type=int, default=0, help="replicas per workgroup (0 automatic)")
    ap.add_argument("--threads", type=int, default=0, help="threads per sweep workgroup (0 automatic)")
    ap.add_argument("--cpu-sample-steps", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain int32 elementwise kernel of known size "
                         "(for scaling HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the engine runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU design is replica sharding, not built)",
              file=sys.stderr)
        sys.exit(2)

    if args.workload.startswith(("batch", "serve")):
        # One hardware queue per stream (set before the HIP runtime starts).
        args.streams = max(1, min(32, args.streams))
        if int(os.environ.get("GPU_MAX_HW_QUEUES", "4")) < args.streams:
            os.environ["GPU_MAX_HW_QUEUES"] = str(args.streams)

    import torch
    from paper_2510_21105_amd import pa, workloads as W

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        src = torch.ones(64 << 20, dtype=torch.int32, device="cuda")   # 256 MiB
        dst = torch.empty_like(src)
        torch.add(src, 1, out=dst)
        torch.cuda.synchronize()
        print(f"[bench] calibration kernel: {src.numel() * 4} bytes read, "
              f"{dst.numel() * 4} bytes written", file=sys.stderr, flush=True)
        del src, dst

    if args.workload.startswith("batch"):
        batch_bench(args, int(args.workload[5:] or 64))
        return
    if args.workload.startswith("serve"):
        serve_bench(args, int(args.workload[5:] or 128))
        return
    wl = W.workload(args.workload)
    g = wl["graph"]
    params = pa.params_from_workload(wl, sweep_kernel=args.sweep_kernel, tile_replicas=args.tile,
                                     wg_threads=args.threads)
    solver = pa.Solver(g)
    K, S, R, N = len(params.betas), params.sweeps, params.R, g.n
    attempts = R * N * S * K
    print(f"[bench] workload {g.name}: N={N} edges={g.n_edges} R={R} K={K} S={S}",
          file=sys.stderr, flush=True)
    # HIP events around the sweep launch of every 7th step (7 is coprime to
    # the cluster-move period of 10, so every phase of it is sampled): the
    # average launch time for the roofline, with the events' own cost on a
    # seventh of the steps only.
    solver.set_timing(TIMING_STRIDE)
    for w in range(args.warmup):
        solver.run(params)
        torch.cuda.synchronize()
        print(f"[bench] warmup {w + 1}/{args.warmup} done", file=sys.stderr, flush=True)

    sweep_ms, sweep_launches = 0.0, 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for step in range(args.steps):
        solver.run(params)
        ms, nl = solver.sweep_time()          # synchronises the stream
        sweep_ms += ms
        sweep_launches += nl
        print(f"[bench] timed solve {step + 1}/{args.steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sec_per_step = (t1 - t0) / args.steps
    value = attempts / sec_per_step

    st = solver.step_stats()
    att_up = int(st[:, 2].sum())
    acc_up = int(st[:, 3].sum())
    accepts = attempts - att_up + acc_up
    a = accepts / attempts
    dbar = 2.0 * g.n_edges / N
    b_alg = algorithmic_bytes_per_attempt(a, dbar, s_h=wl.get("field_bytes", 2))
    per_launch_attempts = R * N * S
    avg_launch_s = sweep_ms / 1000.0 / max(sweep_launches, 1)
    achieved_gbs = b_alg * per_launch_attempts / avg_launch_s / 1e9
    traffic = measured_traffic_per_launch(args.workload)
    copy_gbs = copy_bandwidth_gbs()
    # The sweep keeps a step's spins in LDS and reads HBM only to load and
    # store the population once per step, so the roof above it is the
    # vector ALU (with LDS latency), not HBM. `achieved` counts the method's
    # own integer operations per attempt (algorithmic, whatever the
    # implementation packs into one instruction): one add per neighbour for
    # the local field, 6 for the test, flip, energy and counters, and a
    # quarter of a Philox4x32-10 call (10 rounds of 2 multiply-high, 2
    # multiply-low, 4 xor and 2 key adds: 25 operations per draw) for every
    # uphill attempt, the uphill fraction from the kernel's own counters;
    # times attempts per launch / the live average launch time. Beside it:
    # the issued VALU rate (rocprofv3 SQ_INSTS_VALU per launch, committed
    # under profiles/ and used only while the kernel source matches, x 64
    # lanes), the measured HBM bytes per launch, and the streaming model of
    # a design that streams int8 spins and int16 local fields from HBM.
    f_up = att_up / attempts
    alg_ops = dbar + 6.0 + 25.0 * f_up
    alg_rate = alg_ops * per_launch_attempts / avg_launch_s
    roof = {"bound": "alu", "achieved": float(f"{alg_rate:.4g}"), "peak": VALU_PEAK_LANE_OPS,
            "unit": "int32 lane-op/s", "frac": round(alg_rate / VALU_PEAK_LANE_OPS, 4),
            "traffic": traffic,
            "ops_per_attempt": round(alg_ops, 2), "uphill_fraction": round(f_up, 4),
            "issued": None,
            "hbm_model": {"achieved_gbs": round(achieved_gbs, 1), "peak_gbs": HBM_PEAK_GBS,
                          "frac": round(achieved_gbs / HBM_PEAK_GBS, 4),
                          "bytes_per_attempt": round(b_alg, 3),
                          "measured_copy_gbs": round(copy_gbs, 1),
                          "measured_gbs": (round(traffic / avg_launch_s / 1e9, 1)
                                           if traffic is not None else None)}}
    valu = measured_valu_per_launch(args.workload)
    if valu is not None:
        lane_ops = valu * 64 / avg_launch_s
        roof["issued"] = {"achieved": float(f"{lane_ops:.4g}"),
                          "frac": round(lane_ops / VALU_PEAK_LANE_OPS, 4),
                          "ops_per_attempt": round(valu * 64 / per_launch_attempts, 2),
                          "basis": "rocprofv3 SQ_INSTS_VALU per launch x 64 lanes / live launch time"}

    out = {
        "metric": "spin-flip attempts/s",
        "value": value,
        "unit": "attempts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec_per_step * 1000.0,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {wl['desc']}",
                   "nodes": N, "edges": g.n_edges, "replicas": R, "temperature_steps": K,
                   "sweeps_per_step": S, "attempts_per_solve": attempts},
        "roofline": roof,
        "sweep_kernel": {"avg_launch_ms": avg_launch_s * 1e3, "launches": sweep_launches,
                         "attempts_per_launch": per_launch_attempts,
                         "attempts_per_s": per_launch_attempts / avg_launch_s,
                         "accept_rate": a, "alg_bytes_per_attempt": b_alg,
                         "launch": solver.launch_info()},
        "best_cut": solver.best_cut(),
    }
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_sample_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
