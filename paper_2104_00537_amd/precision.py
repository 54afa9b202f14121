"""Precision study of Section 5.1 on the GPU.

The 3-D dam break is advanced in four arms:

  all_f64     all FP64: velocities and densities held and advanced in FP64,
              every pair in FP64 from the FP64 positions, FP64 rates
              (SPH_INTERACT_F64_STATE) -- the reference of the long run;
  f64         every pair in FP64 (SPH_INTERACT_F64), with the production
              state (FP32 velocities and densities, FP32 rates);
  offset_f32  the production pass: FP32 arithmetic on short offsets
              (fixed-point x modulo 8 cells, cell-relative y and z);
  abs_f32     FP32 arithmetic on positions rounded to FP32 as absolute
              coordinates (SPH_INTERACT_ABS_F32).

Positions are FP64 in every arm.  The front x_f = max x over fluid particles
is recorded every `--every` steps.  Usage:

  python -m paper_2104_00537_amd.precision [--steps 20000] [--every 1000]
                                           [--workload dam_break_3d_1m]

One JSON line per arm goes to stdout, then a summary line.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import cases
from . import sph as S
from .runner import Simulation

ARMS = {"all_f64": S.SPH_INTERACT_F64_STATE, "f64": S.SPH_INTERACT_F64, "offset_f32": 0,
        "abs_f32": S.SPH_INTERACT_ABS_F32}


def _case(name):
    if name == "dam_break_3d_1m":
        return cases.dam_break_3d(cell_div=2, x_sub=4)
    if name == "dam_break_3d_0p5m":
        return cases.dam_break_3d(dp=0.006, cell_div=2, x_sub=4)
    if name == "dam_break_2d":
        return cases.dam_break_2d(cell_div=2, x_sub=4)
    raise SystemExit(f"unknown workload {name}")


def _front(sim):
    st = sim.state
    fl = st.type == cases.FLUID  # excluded particles carry an extra bit
    return float(st.pos[0][fl].max().item())


def run_arm(name, flags, steps, every):
    case = _case(name)
    f64s = flags == S.SPH_INTERACT_F64_STATE
    sim = Simulation(case, "cuda:0", flags=flags, f64_state=f64s)
    fronts = [(0, 0.0, _front(sim))]
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        k = min(every, steps - done)
        sim.run(k)
        done += k
        torch.cuda.synchronize()
        # a particle leaving the grid (a splash over the open top) is excluded
        # and counted; any other error ends the run
        if sim.error() & ~S.SPH_ERR_EXCLUDED:
            raise RuntimeError(f"device error word {sim.error()} at step {done}")
        fronts.append((done, sim.time(), _front(sim)))
        print(f"[precision] flags={flags} step {done}/{steps} t={sim.time():.4f} "
              f"front={fronts[-1][2]:.6f} ({time.perf_counter() - t0:.1f} s)",
              file=sys.stderr, flush=True)
    el = time.perf_counter() - t0
    st = sim.host_state()
    excluded = int(np.count_nonzero(st["type"] & cases.EXCLUDED))
    return dict(fronts=fronts, seconds=el, ms_per_step=el / steps * 1e3,
                interactions=sim.interaction_count(), state=st, excluded=excluded)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--every", type=int, default=1000)
    ap.add_argument("--workload", default="dam_break_3d_1m")
    ap.add_argument("--arms", default="all_f64,f64,offset_f32,abs_f32")
    args = ap.parse_args(argv)
    out = {}
    for arm in args.arms.split(","):
        r = run_arm(args.workload, ARMS[arm], args.steps, args.every)
        out[arm] = r
        print(json.dumps({"arm": arm, "workload": args.workload, "steps": args.steps,
                          "ms_per_step": r["ms_per_step"], "excluded": r["excluded"],
                          "fronts": r["fronts"]}), flush=True)
    refname = "all_f64" if "all_f64" in out else ("f64" if "f64" in out else None)
    if refname:
        ref = out[refname]
        summary = {"workload": args.workload, "steps": args.steps, "reference": refname}
        for arm, r in out.items():
            if arm == refname:
                continue
            d_front = [abs(a[2] - b[2]) for a, b in zip(r["fronts"], ref["fronts"])]
            # particle-wise differences of the final state against the FP64 arm
            dpos = np.abs(r["state"]["pos"] - ref["state"]["pos"]).max(axis=0)
            drho = np.abs(r["state"]["rho"].astype(np.float64)
                          - ref["state"]["rho"].astype(np.float64))
            fl = (ref["state"]["type"] == cases.FLUID) & (r["state"]["type"] == cases.FLUID)
            summary[arm] = {"max_front_diff_m": max(d_front), "final_front_diff_m": d_front[-1],
                            "median_pos_diff_m": float(np.median(dpos[fl])),
                            "p99_pos_diff_m": float(np.quantile(dpos[fl], 0.99)),
                            "median_rho_diff": float(np.median(drho[fl])),
                            "p99_rho_diff": float(np.quantile(drho[fl], 0.99))}
        print(json.dumps({"summary": summary}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
