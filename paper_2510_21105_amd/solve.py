"""Command-line Max-Cut solve of a G-set file on one MI355X.

    python -m paper_2510_21105_amd.solve --gset G63.txt --hex-out best.hex
    python -m paper_2510_21105_amd.solve --gset G63.txt --check-hex config.hex
    python -m paper_2510_21105_amd.solve --gset G63.txt --checkpoint run.ckpt --checkpoint-every 100
    python -m paper_2510_21105_amd.solve --gset G63.txt --resume run.ckpt

The first form runs population annealing (linear inverse-temperature steps,
adaptive stochasticity and cluster moves on by default) and prints one JSON
line with the best cut (eq. (1)) and its configuration in the paper's
hexadecimal format (section 3). The second evaluates eq. (1) for a given
configuration without solving. With --checkpoint the run's state is written
to a file every --checkpoint-every steps (and at the end); --resume continues
such a file with the same flags and gives the result of the uninterrupted
run. Every annealing step runs in the library's kernels; this module only
parses arguments and files.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

from . import gset, hexcfg
from . import workloads as W


def _args(argv):
    ap = argparse.ArgumentParser(prog="python -m paper_2510_21105_amd.solve")
    ap.add_argument("--gset", required=True, help="G-set file: 'N M' then M lines 'i j w'")
    ap.add_argument("--check-hex", help="evaluate the cut of this hex configuration and exit")
    ap.add_argument("--replicas", type=int, default=4096)
    ap.add_argument("--steps", type=int, default=2000, help="temperature steps K")
    ap.add_argument("--sweeps", type=int, default=10, help="sweeps per step S")
    ap.add_argument("--beta", type=float, nargs=2, default=(0.1, 5.0), metavar=("BETA0", "BETA1"))
    ap.add_argument("--order", choices=("natural", "coloring"), default="natural")
    ap.add_argument("--no-as", action="store_true", help="adaptive stochasticity off")
    ap.add_argument("--nl-period", type=int, default=10, help="cluster move every P steps (0 off)")
    ap.add_argument("--nl-kind", type=int, choices=(0, 1), default=0,
                    help="0: cluster moves on replica pairs; 1: single-replica cluster updates")
    ap.add_argument("--adaptive", type=int, nargs=3, metavar=("JUMP", "NUM", "DEN"),
                    help="adaptive steps over the --steps grid: jumps of up to JUMP grid points "
                         "while the reweighted population keeps NUM/DEN of its effective size")
    ap.add_argument("--seed", type=int, default=42)
    ap.add_argument("--instance", type=int, default=0)
    ap.add_argument("--hex-out", help="write the best configuration here")
    ap.add_argument("--checkpoint", help="write the run's state to this file")
    ap.add_argument("--checkpoint-every", type=int, default=100, help="steps between checkpoints")
    ap.add_argument("--resume", help="continue the run saved in this checkpoint file")
    return ap.parse_args(argv)


def main(argv=None) -> dict:
    a = _args(sys.argv[1:] if argv is None else argv)
    g = gset.load(a.gset)
    if a.check_hex:
        with open(a.check_hex) as f:
            x = hexcfg.hex_to_config(f.read(), g.n)
        out = dict(graph=g.name, n=g.n, edges=g.n_edges, cut=gset.cut_value(g, x),
                   ones=int((x > 0).sum()))
        print(json.dumps(out), flush=True)
        return out

    import torch
    from . import pa

    order = W.natural_order(g.n) if a.order == "natural" else W.coloring_order(g)
    wl = dict(graph=g, betas=W.linear_betas(a.beta[0], a.beta[1], a.steps), sweeps=a.sweeps,
              order=order, R=a.replicas, seed=a.seed, inst=a.instance,
              as_enable=0 if a.no_as else 1, as_stall_steps=20, as_max_level=4,
              as_frozen_inv=256, as_gamma=0.8, nl_period=a.nl_period, nl_kind=a.nl_kind)
    if a.adaptive:
        wl.update(beta_adapt=1, adapt_jump=a.adaptive[0], adapt_num=a.adaptive[1],
                  adapt_den=a.adaptive[2])
    s = pa.Solver(g)
    p = pa.params_from_workload(wl)
    t0 = time.perf_counter()
    k = 0
    if a.resume:
        with open(a.resume, "rb") as f:
            blob = f.read()
        s.restore(p, blob)
        k = pa.next_step(blob)
    every = a.steps if not a.checkpoint else max(1, a.checkpoint_every)
    while k < a.steps:
        k1 = min(a.steps, k + every)
        s.run_steps(p, k, k1)
        k = k1
        if a.checkpoint:
            blob = s.checkpoint()
            with open(a.checkpoint + ".tmp", "wb") as f:
                f.write(blob)
            os.replace(a.checkpoint + ".tmp", a.checkpoint)
    cut = s.best_cut()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    hx = s.best_config_hex()
    info = s.best_info()
    if a.hex_out:
        with open(a.hex_out, "w") as f:
            f.write(hx + "\n")
    out = dict(graph=g.name, n=g.n, edges=g.n_edges, best_cut=cut, best_energy=info["E"],
               found_at_step=info.get("step"), seconds=dt, hex=hx)
    print(json.dumps(out), flush=True)
    s.close()
    return out


if __name__ == "__main__":
    main()
