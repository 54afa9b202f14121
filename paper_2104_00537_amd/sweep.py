"""Throughput against problem size on one GPU (the paper's Section 5.3 plots
GPIPS, 10^9 particle interactions per second, against the particle count).

The 3-D dam break (1.6 x 0.6 x 0.6 m box, 0.6 x 0.6 x 0.3 m block) is built at
the spacing that gives each requested fluid particle count, advanced a few
warm-up steps, then timed over --steps symplectic steps (all state resident
in HBM, cells of h split in 4 along x).  One JSON line per size on stdout.

  python -m paper_2104_00537_amd.sweep [--sizes 0.1,0.3,1,3,10,30,64] [--steps 10] [--graph]

Sizes are in millions of fluid particles.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import torch

from . import cases
from .runner import Simulation


def measure(n_fluid: float, steps: int, warmup: int, integrator: str = "symplectic",
            graph: bool = False) -> dict:
    dp = (0.6 * 0.6 * 0.3 / n_fluid) ** (1.0 / 3.0)
    t0 = time.perf_counter()
    case = cases.dam_break_3d(dp=dp, cell_div=2, x_sub=4)
    build_s = time.perf_counter() - t0
    sim = Simulation(case, "cuda:0", integrator=integrator)
    for _ in range(warmup):
        sim.step()
    if graph:  # two steps per HIP graph (the state buffers alternate)
        if steps % 2:
            raise SystemExit("--graph needs an even --steps")
        sim.capture(2)
        sim.replay(1)
    torch.cuda.synchronize()
    i0 = sim.interaction_count()
    t0 = time.perf_counter()
    if graph:
        sim.replay(steps // 2)
    else:
        for _ in range(steps):
            sim.step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    err = sim.error()
    pairs = sim.interaction_count() - i0
    out = {"n_fluid": case.n_fluid, "n": case.n, "dp": dp, "cells": case.params.ncell_total(),
           "integrator": integrator, "steps": steps, "ms_per_step": el / steps * 1e3,
           "interactions_per_s": pairs / el, "gpips": pairs / el / 1e9,
           "interactions_per_particle_step": pairs / steps / case.n, "error_word": err,
           "case_build_s": build_s, "graph": graph}
    del sim
    torch.cuda.empty_cache()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes", default="0.1,0.3,1,3,10,30,64")
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--integrator", default="symplectic")
    ap.add_argument("--graph", action="store_true",
                    help="replay the timed steps from HIP graphs (as the serving path does)")
    args = ap.parse_args(argv)
    for s in args.sizes.split(","):
        r = measure(float(s) * 1e6, args.steps, args.warmup, args.integrator, args.graph)
        print(json.dumps(r), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
