"""Benchmark: particle interactions/s of the WCSPH hot path on one MI355X.

A step is one full symplectic step of the hot path (two neighbour lists, two
interaction passes, the time step, predictor and corrector) on the 3-D dam
break with 1.0M fluid particles (plus 0.32M wall particles), all state
resident in HBM.  The JSON line reports:

  value      particle interactions (ordered pairs evaluated, the paper's PIPS
             count) per second over the K timed steps, counted on the device;
  roofline   the interaction kernel (the dominant one): algorithmic FP32
             flops per launch / its average duration from HIP events on the
             launch stream, against the FP32 vector peak;
  cpu_baseline  the CPU FP64 oracle on a bounded sample of the same pass.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "particle interactions/s at 3D 1M particles; batched solves/s + p50/p99 latency"

# Algorithmic FP32 flops per evaluated pair (FMA = 2, sqrt and division = 1):
# fluid target: kernel gradient 15, relative velocity and v.r 8, volume 1,
# continuity 3, pressure term 3, viscosity mu 3 and Pi 4, coefficient 3,
# momentum update 6, density diffusion 4  -> 50;
# wall target (continuity of Eq. 36 only): 15 + 8 + 1 + 3 -> 27.
FLOPS_FLUID_PAIR = 50
FLOPS_WALL_PAIR = 27
# FP32 vector issue peak without packed-FP32 instructions (the build disables
# them): 256 CUs x 4 SIMD x 16 lanes x 2 flops (FMA) x 2.4 GHz.
PEAK_FP32_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
PEAK_HBM_GBS = 8000.0


def measured_traffic(kernel, workload_name):
    """HBM bytes per launch of the interaction kernel from the committed
    counter summary (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when
    the kernel sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}__{workload_name}.md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and line.split(":")[0] in ("traffic_bytes_per_launch",
                                                  "kernel_source_sha256", "kernel_sources"):
            k, v = line.split(":", 1)
            fields[k] = v.strip()
    if len(fields) != 3:
        return None
    h = hashlib.sha256()
    for src in fields["kernel_sources"].split():
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != fields["kernel_source_sha256"]:
        return None
    return int(fields["traffic_bytes_per_launch"])


def workload(name, cell_div, x_sub):
    from paper_2104_00537_amd import cases
    kw = dict(cell_div=cell_div, x_sub=x_sub)
    if name == "dam_break_3d_1m":
        return cases.dam_break_3d(**kw)
    if name == "dam_break_3d_0p5m":
        return cases.dam_break_3d(dp=0.006, **kw)
    if name == "dam_break_2d":
        return cases.dam_break_2d(**kw)
    if name == "sloshing_3d_64m":
        return cases.sloshing_3d(**kw)
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(case, sim, seconds):
    """The oracle (brute force, FP64) on a random sample of targets of the
    benchmarked state; interactions/s over the sampled targets."""
    import numpy as np
    import oracle
    st = sim.host_state()
    rng = np.random.default_rng(1234)
    n = case.n
    cp = case.params
    args = (cp, st["pos"], st["vel"].astype(np.float64), st["rho"].astype(np.float64), st["type"])
    oracle.interact(*args, targets=rng.choice(n, size=min(n, 16), replace=False))  # warm-up
    # random targets in chunks until about `seconds` of CPU work is done
    order = rng.permutation(n)
    done, pairs, el, chunk = 0, 0, 0.0, 256
    while done < n and el < seconds:
        tg = order[done:done + chunk]
        t0 = time.perf_counter()
        _, _, _, nbr = oracle.interact(*args, targets=tg)
        dt = time.perf_counter() - t0
        el += dt
        pairs += int(nbr.astype(np.int64).sum())
        done += len(tg)
        chunk = int(min(max(chunk, len(tg) * max(seconds - el, 0.0) / max(dt, 1e-6) / 4), 1 << 16))
        chunk = max(chunk, 64)
    k = done
    try:
        aff = len(os.sched_getaffinity(0))
    except AttributeError:
        aff = os.cpu_count() or 1
    omp = os.environ.get("OMP_NUM_THREADS")
    cores = min(aff, int(omp)) if omp and omp.isdigit() else aff
    return {"value": float(pairs / el), "unit": "interactions/s",
            "cores": cores, "kind": "oracle", "cpu": cpu_model(),
            "sample": f"one interaction pass for {k} random targets of {n} particles "
                      f"(all {n} as candidate neighbours, brute force FP64), {el:.1f} s"}


def verlet_leg(case, steps, warmup):
    """The same workload advanced with the Verlet scheme (Eq. 30-31, one
    interaction per step, Eq. 31 every 40 steps): steps/s and interactions/s."""
    import torch
    from paper_2104_00537_amd.runner import Simulation
    sim = Simulation(case, "cuda:0", integrator="verlet", verlet_ns=40)
    for _ in range(warmup):
        sim.step()
    torch.cuda.synchronize()
    i0 = sim.interaction_count()
    t0 = time.perf_counter()
    for _ in range(steps):
        sim.step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    if sim.error() != 0:
        raise SystemExit(f"device error word {sim.error()} in the Verlet leg")
    pairs = sim.interaction_count() - i0
    return {"steps": steps, "ms_per_step": el / steps * 1e3, "steps_per_s": steps / el,
            "interactions_per_s": pairs / el, "ns": 40}


def case_leg(case, steps=20, warmup=5):
    """Whole symplectic steps of another case: ms per step, interactions/s
    and the mean time of each call (HIP events on the launch stream, 3 extra
    steps)."""
    import numpy as np
    import torch
    from paper_2104_00537_amd.runner import Simulation
    sim = Simulation(case, "cuda:0")
    for _ in range(warmup):
        sim.step()
    torch.cuda.synchronize()
    i0 = sim.interaction_count()
    t0 = time.perf_counter()
    for _ in range(steps):
        sim.step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    pairs = sim.interaction_count() - i0
    timing = {}
    for _ in range(3):
        sim.step(timing=timing)
    torch.cuda.synchronize()
    if sim.error() != 0:
        raise SystemExit(f"device error word {sim.error()} in the {case.params.name} leg")
    phase_ms = {k: float(np.mean([a.elapsed_time(b) for a, b in v])) for k, v in timing.items()}
    return sim, {"n_particles": case.n, "steps": steps, "ms_per_step": el / steps * 1e3,
                 "interactions_per_s": pairs / el, "phase_ms_per_call": phase_ms}


def periodic_leg(args):
    """A 3-D channel periodic along x and y (Section 2.7): 1.6 x 0.6 m in
    plan, 0.3 m deep between a bottom and a top wall, at the workload's
    resolution (cells of a whole number of particle spacings), with a mean
    flow of 1 m/s along x driven by a body force of 2 m/s^2."""
    from paper_2104_00537_amd import cases
    dp = 0.6 / 126
    g = (2.0, 0.0, -cases.GRAVITY)
    case = cases.periodic_box(3, shape=(336, 126, 63), dp=dp, periodic=(0, 1), walls=True,
                              gravity=g, cell_div=args.cell_div, x_sub=args.x_sub)
    case.vel[0, case.type == cases.FLUID] = 1.0
    _, res = case_leg(case)
    res["workload"] = "periodic_channel_3d"
    res["n_fluid"] = case.n_fluid
    return res


def shifting_leg(args):
    """The workload itself with particle shifting (Section 2.8: A_s = 2,
    tangential shift where C < 0.9) after every corrector."""
    import dataclasses
    from paper_2104_00537_amd import cases
    case = workload(args.workload, args.cell_div, args.x_sub)
    case = cases.Case(dataclasses.replace(case.params, shift_coef=2.0, shift_fs=0.9), case.pos,
                      case.vel, case.rho, case.type, dict(case.meta), case.normal)
    _, res = case_leg(case)
    res["workload"] = args.workload + "+shifting"
    return res


def floating_leg(args, steps=20, warmup=5):
    """A floating box (Section 3.2) at the workload's resolution: the 3-D
    dam-break block released into a tank holding a 0.06 m water layer, with
    a 0.12 x 0.12 x 0.08 m box of density 500 kg/m^3 floating on the layer
    at x = 1.0 m.  Steps/s, interactions/s and the cost of the rigid-body
    calls (HIP events on the launch stream)."""
    import numpy as np
    import torch
    from paper_2104_00537_amd import cases
    from paper_2104_00537_amd.runner import Simulation
    case = cases.floating_box(3, dp=0.6 / 126, tank=(1.6, 0.6, 0.6), column=(0.6, 0.6, 0.3),
                              layer=0.06, box=(0.12, 0.12, 0.08), box_x=1.0,
                              cell_div=args.cell_div, x_sub=args.x_sub)
    sim = Simulation(case, "cuda:0")
    for _ in range(warmup):
        sim.step()
    torch.cuda.synchronize()
    i0 = sim.interaction_count()
    t0 = time.perf_counter()
    for _ in range(steps):
        sim.step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    timing = {}
    for _ in range(3):
        sim.step(timing=timing)
    torch.cuda.synchronize()
    if sim.error() != 0:
        raise SystemExit(f"device error word {sim.error()} in the floating-body leg")
    pairs = sim.interaction_count() - i0
    steps_all = steps + 3
    phase_ms = {k: float(np.mean([a.elapsed_time(b) for a, b in v])) for k, v in timing.items()}
    b = sim.body_state()[0]
    return {"workload": "floating_box_3d", "n_particles": case.n,
            "n_floating": case.bodies[0]["count"], "steps": steps,
            "ms_per_step": el / steps * 1e3, "interactions_per_s": pairs / (el * steps_all / steps),
            "ms_floating_call": phase_ms["floating"], "ms_interact": phase_ms["interact"],
            "body_velocity": [float(v) for v in b["vel"]]}


VARIANTS = {"default": {}, "cubic_spline": dict(kernel=1),
            "laminar_viscosity": dict(viscosity=1, visc_nu=1e-6), "fourtakas_ddt": dict(ddt=2),
            "all_three": dict(kernel=1, viscosity=1, visc_nu=1e-6, ddt=2)}


def variants_leg(case, launches=10):
    """One interaction pass per formulation option on the binned initial
    state: ms per pass and interactions/s (HIP events on the launch stream)."""
    import dataclasses
    import torch
    from paper_2104_00537_amd import sph as S
    n, dim = case.n, case.params.dim
    P0 = S.make_params(case.params)
    src = S.DeviceState.from_case(case, "cuda:0", with_normal=True)
    dst = S.DeviceState.empty(dim, n, "cuda:0", with_normal=True)
    key = torch.empty(n, dtype=torch.int32, device="cuda:0")
    perm = torch.empty_like(key)
    start = torch.empty(case.params.ncell_total() + 1, dtype=torch.int32, device="cuda:0")
    ws = torch.zeros(S.sph_workspace_bytes(P0, n), dtype=torch.uint8, device="cuda:0")
    ace = torch.empty((dim, n), dtype=torch.float32, device="cuda:0")
    arho = torch.empty(n, dtype=torch.float32, device="cuda:0")
    S.sph_bin_cells(P0, n, src, dst, key, perm, start, ws)
    out = {}
    for name, kw in VARIANTS.items():
        P = S.make_params(dataclasses.replace(case.params, **kw))
        inter = torch.zeros(2, dtype=torch.int64, device="cuda:0")
        dt = torch.zeros(1, dtype=torch.float64, device="cuda:0")
        S.sph_interact(P, n, dst, key, start, ace, arho, ws)  # warm-up
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(launches):
            S.sph_interact(P, n, dst, key, start, ace, arho, ws)
        e1.record()
        S.sph_reduce_dt(P, n, dt, ws, interactions=inter)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / launches
        out[name] = {"ms_per_pass": ms, "interactions_per_s": int(inter[0].item()) / (ms * 1e-3)}
    # modified DBC (last: it rewrites the wall entries of the state and view):
    # the wall pass, then the interaction, which skips wall targets
    P = S.make_params(dataclasses.replace(case.params, boundary=1))
    S.sph_mdbc(P, n, dst, key, start, ws)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record()
    for _ in range(launches):
        S.sph_mdbc(P, n, dst, key, start, ws)
    ev[1].record()
    for _ in range(launches):
        S.sph_interact(P, n, dst, key, start, ace, arho, ws)
    ev[2].record()
    inter = torch.zeros(2, dtype=torch.int64, device="cuda:0")
    dt = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    S.sph_reduce_dt(P, n, dt, ws, interactions=inter)
    torch.cuda.synchronize()
    ms_m = ev[0].elapsed_time(ev[1]) / launches
    ms_i = ev[1].elapsed_time(ev[2]) / launches
    out["modified_dbc"] = {"ms_mdbc": ms_m, "ms_per_pass": ms_i,
                           "interactions_per_s": int(inter[0].item()) / ((ms_m + ms_i) * 1e-3)}
    return out


def serving(args):
    """The request stream through the batched engine and the plain
    one-case-at-a-time path (same seeded trace, same GPU)."""
    import numpy as np
    import torch
    from paper_2104_00537_amd import serve as V
    kw = dict(n_min=args.serve_n_min, n_max=args.serve_n_max, steps_min=1000, steps_max=5000,
              steps_scale=args.serve_steps_scale)
    out = {"stream": dict(requests=args.serve_requests, rate_per_s=args.serve_rate,
                          n_range=[args.serve_n_min, args.serve_n_max],
                          steps="uniform 1000-5000 x %g" % args.serve_steps_scale, seed=7)}
    reqs = V.make_stream(args.serve_requests, args.serve_rate, seed=7, **kw)
    out["stream"]["particles_mean"] = float(np.mean([r.n for r in reqs]))
    out["stream"]["steps_mean"] = float(np.mean([r.steps for r in reqs]))
    cap_n = max(4 * max(r.n for r in reqs), args.serve_cap_particles)
    eng = V.BatchEngine(cap_particles=cap_n, cap_cells=args.serve_cap_cells,
                        max_slots=args.serve_slots, device="cuda:0",
                        four_lanes=args.serve_four_lanes)
    out["stream"]["four_lanes"] = bool(args.serve_four_lanes)
    # warm-up of the code paths (first kernel launches, graph capture)
    warm = V.make_stream(2, 1e6, seed=99, n_min=2000, n_max=3000, steps_min=4, steps_max=4)
    V.serve_batched(warm, eng)
    V.serve_plain(V.make_stream(1, 1e6, seed=98, n_min=2000, n_max=3000, steps_min=4,
                                steps_max=4))
    torch.cuda.synchronize()
    if args.serve_legs in ("both", "batched"):
        print("[bench] serving: batched engine", file=sys.stderr, flush=True)
        out["batched"] = V.serve_batched(reqs, eng)
    if args.serve_legs in ("both", "plain"):
        print("[bench] serving: plain path", file=sys.stderr, flush=True)
        reqs2 = V.make_stream(args.serve_requests, args.serve_rate, seed=7, **kw)
        out["plain"] = V.serve_plain(reqs2)
        # offered load: arrival rate x the mean service time of the plain
        # path (above 1 the stream queues on that path)
        svc = [r.finish - r.start for r in reqs2]
        out["stream"]["plain_mean_service_s"] = float(np.mean(svc))
        out["stream"]["offered_load_plain"] = float(args.serve_rate * np.mean(svc))
    if "batched" in out and "plain" in out:
        out["speedup_solves_per_s"] = out["batched"]["solves_per_s"] / out["plain"]["solves_per_s"]
        out["p50_ratio_plain_over_batched"] = (out["plain"]["p50_latency_s"]
                                               / out["batched"]["p50_latency_s"])
        out["p99_ratio_plain_over_batched"] = (out["plain"]["p99_latency_s"]
                                               / out["batched"]["p99_latency_s"])
    return out


def profile_mode(args):
    """Kernel-only modes for counter runs: 'interact' bins the workload once
    and launches the interaction kernel --steps times; 'copy' copies a 1 GiB
    buffer --steps times (the reference for the HBM byte counters)."""
    import torch
    if args.mode == "copy":
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(args.steps):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "copy", "bytes_read_per_launch": x.numel() * 4,
                          "bytes_written_per_launch": y.numel() * 4}), flush=True)
        return 0
    from paper_2104_00537_amd import sph as S
    case = workload(args.workload, args.cell_div, args.x_sub)
    P = S.make_params(case.params)
    n = case.n
    src = S.DeviceState.from_case(case, "cuda:0")
    dst = S.DeviceState.empty(case.params.dim, n, "cuda:0")
    key = torch.empty(n, dtype=torch.int32, device="cuda:0")
    perm = torch.empty_like(key)
    start = torch.empty(case.params.ncell_total() + 1, dtype=torch.int32, device="cuda:0")
    ws = torch.zeros(S.sph_workspace_bytes(P, n), dtype=torch.uint8, device="cuda:0")
    ace = torch.empty((case.params.dim, n), dtype=torch.float32, device="cuda:0")
    arho = torch.empty(n, dtype=torch.float32, device="cuda:0")
    S.sph_bin_cells(P, n, src, dst, key, perm, start, ws)
    inter = torch.zeros(2, dtype=torch.int64, device="cuda:0")
    dt = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        S.sph_interact(P, n, dst, key, start, ace, arho, ws)
    e1.record()
    S.sph_reduce_dt(P, n, dt, ws, interactions=inter)
    torch.cuda.synchronize()
    print(json.dumps({"mode": "interact", "workload": args.workload, "n": n,
                      "pairs_per_launch": int(inter[0].item()),
                      "wall_pairs_per_launch": int(inter[1].item()),
                      "ms_per_launch": e0.elapsed_time(e1) / max(args.steps, 1)}), flush=True)
    return 0


def _front(sim, case):
    """Largest x over fluid particles, relative to the tank length (the
    dam-break front) and its value in metres."""
    import numpy as np
    st = sim.state
    fl = (st.type == 0)
    x = float(st.pos[0][fl].max().item())
    x0 = float(case.pos[0].min())
    return x, (x - x0)


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), or the platform's."""
    import platform
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def run_mode(args):
    """A whole run of a workload from its initial state: every one of
    --steps steps is timed (no warm-up beyond the kernels' first launch on a
    copy of the case), with the interactions counted on the device.  For the
    2-D dam break, --oracle also runs the CPU oracle over the same steps
    (timed, on the host cores) and compares the fronts."""
    import numpy as np
    import torch
    from paper_2104_00537_amd.runner import Simulation
    case = workload(args.workload, args.cell_div, args.x_sub)
    print(f"[bench] run {args.workload}: n={case.n} fluid={case.n_fluid} "
          f"cells={case.params.ncell} steps={args.steps}", file=sys.stderr, flush=True)
    # first launches (module load, code paths) on a throw-away copy of a
    # small case of the same kind, so that the timed run starts warm
    warm = workload("dam_break_2d", args.cell_div, args.x_sub)
    w = Simulation(warm, "cuda:0")
    for _ in range(4):
        w.step()
    del w
    sim = Simulation(case, "cuda:0")
    torch.cuda.synchronize()
    # every step is timed; the device is synchronised after every chunk of
    # steps (a few microseconds per chunk) to record how the cost per step
    # evolves with the flow
    t0 = time.perf_counter()
    last = t0
    done = 0
    chunk = max(1, min(args.steps, args.run_chunk))
    by_chunk = []
    i_prev, c_prev = 0, t0
    while done < args.steps:
        k = min(chunk, args.steps - done)
        for _ in range(k):
            sim.step()
        done += k
        torch.cuda.synchronize()
        now = time.perf_counter()
        i_now = int(sim.interactions[0].item())
        by_chunk.append({"steps": k, "ms_per_step": (now - c_prev) / k * 1e3,
                         "interactions_per_s": (i_now - i_prev) / (now - c_prev),
                         "t_end_s": sim.time(), "dt": float(sim.dt.item())})
        i_prev, c_prev = i_now, time.perf_counter()
        if now - last > 20.0 or done == args.steps:
            last = now
            print(f"[bench] step {done}/{args.steps} t={sim.time():.5f} s", file=sys.stderr,
                  flush=True)
    el = time.perf_counter() - t0
    err = sim.error()
    if err != 0:
        raise SystemExit(f"device error word {err} during the run")
    d_inter = sim.interactions.cpu().numpy().astype(np.int64)
    xf, front = _front(sim, case)
    length = float(case.meta.get("tank", (1.0,))[0])
    res = {"mode": "run", "workload": args.workload, "n_particles": case.n,
           "n_fluid": case.n_fluid, "steps": args.steps, "seconds": el,
           "ms_per_step": el / args.steps * 1e3, "steps_per_s": args.steps / el,
           "interactions": int(d_inter[0]), "interactions_per_s": float(d_inter[0]) / el,
           "sim_time_s": sim.time(), "dt_last": float(sim.dt.item()),
           "front_x_m": xf, "front_over_length": front / length,
           "cell_div": args.cell_div, "x_sub": args.x_sub, "by_chunk": by_chunk}
    if args.oracle:
        import oracle
        if case.n > 20000:
            raise SystemExit("--oracle runs the brute-force oracle: small cases only")
        gpu = sim.host_state()
        cp = case.params
        print(f"[bench] oracle: {args.steps} steps on the host", file=sys.stderr, flush=True)
        t1 = time.perf_counter()
        out = oracle.run(cp, case.pos, case.vel.astype(np.float64),
                         case.rho.astype(np.float64), case.type, args.steps)
        el_o = time.perf_counter() - t1
        pos, t_end = out["pos"], out["t"]
        fl = case.type == 0
        xo = float(pos[0][fl].max())
        try:
            aff = len(os.sched_getaffinity(0))
        except AttributeError:
            aff = os.cpu_count() or 1
        omp = os.environ.get("OMP_NUM_THREADS")
        cores = min(aff, int(omp)) if omp and omp.isdigit() else aff
        res["oracle"] = {"seconds": el_o, "ms_per_step": el_o / args.steps * 1e3,
                         "cores": cores, "cpu": cpu_model(), "sim_time_s": float(t_end),
                         "front_x_m": xo,
                         "front_diff_over_length": abs(xo - float(gpu["pos"][0][fl].max())) / length,
                         "max_pos_diff_m": float(np.abs(pos - gpu["pos"]).max()),
                         "interactions": int(out["interactions"]), "status": int(out["status"]),
                         "gpu_speedup": el_o / el}
    print(json.dumps(res), flush=True)
    return 0


def serve_mode(args):
    """The serving stream alone (both paths, same seeded trace)."""
    res = {"mode": "serve", "serving": serving(args)}
    print(json.dumps(res), flush=True)
    return 0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="dam_break_3d_1m")
    ap.add_argument("--cell-div", type=int, default=2)
    ap.add_argument("--x-sub", type=int, default=4)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--mode", choices=["step", "interact", "copy", "run", "serve"],
                    default="step",
                    help="step: the benchmark; interact/copy: kernel-only runs for counters; "
                         "run: a whole run of --steps steps from t = 0; serve: the serving "
                         "stream alone")
    ap.add_argument("--run-chunk", type=int, default=100,
                    help="run mode: steps between synchronisations (cost per chunk reported)")
    ap.add_argument("--oracle", action="store_true",
                    help="run mode: also run the CPU oracle over the same steps (2-D case)")
    ap.add_argument("--neighbour-list", action="store_true",
                    help="step mode: both passes replay per-target neighbour lists "
                         "(sph_build_list / sph_interact_list) instead of walking the cells")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-verlet", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-floating", action="store_true")
    ap.add_argument("--no-periodic", action="store_true")
    ap.add_argument("--no-shifting", action="store_true")
    ap.add_argument("--timing", choices=["all", "interact", "none"], default="interact",
                    help="calls bracketed by HIP events inside the timed steps")
    ap.add_argument("--graph-steps", type=int, default=0,
                    help="> 0: replay the timed steps as HIP graphs of this many steps")
    ap.add_argument("--serve-requests", type=int, default=24)
    ap.add_argument("--serve-legs", choices=["both", "batched", "plain"], default="both")
    ap.add_argument("--serve-rate", type=float, default=4.0)
    ap.add_argument("--serve-steps-scale", type=float, default=1.0)
    ap.add_argument("--serve-n-min", type=int, default=2000)
    ap.add_argument("--serve-n-max", type=int, default=500_000)
    ap.add_argument("--serve-slots", type=int, default=256)
    ap.add_argument("--serve-four-lanes", action="store_true",
                    help="batched leg: four lanes per target for slots of at most 131,072 "
                         "particles (SPH_BATCH_FOUR_LANES)")
    ap.add_argument("--serve-cap-particles", type=int, default=6_000_000)
    ap.add_argument("--serve-cap-cells", type=int, default=120_000_000)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: this path has no multi-GPU mode "
              f"(asked for --gpus {args.gpus})", file=sys.stderr)
        return 2

    if args.mode == "run":
        return run_mode(args)
    if args.mode == "serve":
        return serve_mode(args)
    if args.mode != "step":
        return profile_mode(args)

    import numpy as np
    import torch
    from paper_2104_00537_amd.runner import Simulation

    case = workload(args.workload, args.cell_div, args.x_sub)
    sim = Simulation(case, "cuda:0", neighbour_list=args.neighbour_list)
    print(f"[bench] {args.workload}: n={case.n} fluid={case.n_fluid} cells={case.params.ncell}",
          file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        sim.step()
    torch.cuda.synchronize()
    if sim.error() != 0:
        raise SystemExit(f"device error word {sim.error()} after warm-up")
    inter0 = sim.interactions.clone()
    timing = {}
    if args.timing == "interact":
        sim.timed_calls = ("interact",)
    if args.graph_steps > 0:
        if args.steps % args.graph_steps:
            raise SystemExit("--steps must be a multiple of --graph-steps")
        sim.capture(args.graph_steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if args.graph_steps > 0:
        sim.replay(args.steps // args.graph_steps)
    else:
        for _ in range(args.steps):
            sim.step(timing=None if args.timing == "none" else timing)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    err = sim.error()
    if err != 0:
        raise SystemExit(f"device error word {err} during the timed steps")
    d_inter = (sim.interactions - inter0).cpu().numpy().astype(np.int64)
    pairs, wall_pairs = int(d_inter[0]), int(d_inter[1])
    launches = 2 * args.steps  # two interaction passes per symplectic step
    phase_src = "timed steps"
    if not timing or set(timing) == {"interact"}:
        # the other calls' durations from 5 extra steps after the timed region
        extra = {}
        sim.timed_calls = None
        for _ in range(5):
            sim.step(timing=extra)
        torch.cuda.synchronize()
        for k, v in extra.items():
            if k not in timing:
                timing[k] = v
        phase_src = "timed steps (interact)" if "interact" in timing and \
            len(timing["interact"]) == launches else "5 steps after the timed region"
        if not args.graph_steps and args.timing == "none":
            phase_src = "5 steps after the timed region"
    phase_ms = {k: float(np.mean([a.elapsed_time(b) for a, b in v])) for k, v in timing.items()}
    phase_med = {k: float(np.median([a.elapsed_time(b) for a, b in v]))
                 for k, v in timing.items()}
    phase_n = {k: len(v) for k, v in timing.items()}
    graph_ms = None
    if args.graph_steps == 0 and not args.neighbour_list:
        # the whole step replayed from a HIP graph (two steps per graph: the
        # state buffers alternate), after the timed region
        sim.capture(2)
        sim.replay(2)
        torch.cuda.synchronize()
        g0 = time.perf_counter()
        sim.replay(10)
        torch.cuda.synchronize()
        graph_ms = (time.perf_counter() - g0) / 20 * 1e3
        if sim.error() != 0:
            raise SystemExit(f"device error word {sim.error()} in the graph replay")
    t_int = phase_ms["interact"] * 1e-3
    flops = (FLOPS_FLUID_PAIR * (pairs - wall_pairs) + FLOPS_WALL_PAIR * wall_pairs) / launches
    achieved = flops / t_int / 1e12
    # algorithmic bytes of one interaction launch: per particle the view read
    # (2 x 16 B), ace + arho written (4 x 4 B), key and cell range reads (8 B)
    bytes_per_launch = case.n * (32 + 16 + 8)
    kernel = "k_interact_list" if args.neighbour_list else "k_interact_gather"
    traffic = (measured_traffic(kernel, args.workload)
               if (args.cell_div, args.x_sub) == (2, 4) and not args.neighbour_list else None)
    res = {
        "metric": METRIC,
        "value": pairs / el,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n_particles": case.n, "n_fluid": case.n_fluid,
                   "dp": case.params.dp, "h": case.params.h, "cell_div": args.cell_div,
                   "x_sub": args.x_sub, "neighbour_list": args.neighbour_list,
                   "parallelism": "single GPU", "positions": "fp64 state; fp32 offsets (fixed-point x, cell-relative y, z)"},
        "steps_per_s": args.steps / el,
        "interactions_per_step": pairs / args.steps,
        "phase_ms_per_call": phase_ms,
        "phase_ms_source": phase_src,
        "phase_ms_median": phase_med,
        "phase_calls_timed": phase_n,
        "graph_replay_ms_per_step": graph_ms,
        "timing_mode": {"events": args.timing, "graph_steps": args.graph_steps},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS, "traffic": traffic,
                     "traffic_unit": "bytes/launch", "kernel": kernel,
                     "flops_per_launch": flops, "avg_launch_ms": phase_ms["interact"],
                     "algorithmic_bytes_per_launch": bytes_per_launch,
                     "hbm_algorithmic_GBs": bytes_per_launch / t_int / 1e9,
                     "hbm_frac": bytes_per_launch / t_int / 8e12,
                     "hbm_measured_frac": (traffic / t_int / 8e12) if traffic else None},
    }
    print(f"[bench] timed {args.steps} steps: {pairs / el:.4g} interactions/s", file=sys.stderr,
          flush=True)
    if not args.no_verlet:
        res["verlet"] = verlet_leg(case, args.steps, args.warmup)
    if not args.no_variants:
        res["variants"] = variants_leg(case)
    if not args.no_floating:
        res["floating"] = floating_leg(args)
    if not args.no_periodic:
        res["periodic"] = periodic_leg(args)
    if not args.no_shifting:
        res["shifting"] = shifting_leg(args)
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(case, sim, args.cpu_seconds)
    if not args.no_serve:
        del sim
        torch.cuda.empty_cache()
        res["serving"] = serving(args)
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
