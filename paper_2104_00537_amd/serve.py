"""Continuous-batching serving of SPH cases over the libsph batch ABI.

Requests (SPH cases with a step count) arrive over time.  The batched engine
keeps every admitted case's particle state and cell lists resident on the
GPU, packed into one set of arrays (one "slot" per case), and advances all of
them together each step through the ``sph_batch_*`` calls: one binning, one
interaction launch and one update for the whole batch, each case with its own
dt and t.  Cases are admitted when a slot and HBM are free (footprint
admission) and retired as soon as their steps are done; the batch is then
repacked and its step re-captured as a HIP graph.  The plain path runs the
same requests one at a time, in arrival order, with the single-case calls.

Both report per-request completion latency (arrival to results on the host),
solves/s and particle interactions/s.
"""
from __future__ import annotations

import time
from dataclasses import dataclass
from typing import List, Optional

import numpy as np
import torch

from . import cases as K
from . import sph as S
from .runner import Simulation

# bytes of device memory per particle held by the batched engine (two
# states, two saved states, key, perm, rates, views and sort buffers)
BYTES_PER_PARTICLE = 2 * (24 + 12 + 4 + 1 + 4) + 2 * (24 + 12 + 4) + 8 + 16 + 32 + 16 + 16


@dataclass
class Request:
    rid: int
    case: K.Case
    steps: int
    arrival: float                   # seconds after the stream starts
    start: Optional[float] = None    # admitted (batched) / started (plain)
    finish: Optional[float] = None   # results on the host
    interactions: int = 0
    result: Optional[dict] = None    # final state (original particle order)
    error: int = 0

    @property
    def n(self) -> int:
        return self.case.n

    @property
    def latency(self) -> float:
        return self.finish - self.arrival


def to_3d(case: K.Case):
    """A case's arrays in the batch's 3-component layout ((x, 0, z) in 2-D)."""
    if case.params.dim == 3:
        return case.pos, case.vel
    n = case.n
    pos = np.zeros((3, n), np.float64)
    vel = np.zeros((3, n), np.float32)
    pos[0], pos[2] = case.pos[0], case.pos[1]
    vel[0], vel[2] = case.vel[0], case.vel[1]
    return pos, vel


def from_3d(dim, pos, vel):
    if dim == 3:
        return pos, vel
    return pos[[0, 2]], vel[[0, 2]]


class _Flat:
    """A flat device buffer viewed as [c][n] for the current batch size."""

    def __init__(self, comps, cap, dtype, device):
        self.comps = comps
        self.buf = torch.zeros(comps * cap, dtype=dtype, device=device)

    def view(self, n):
        v = self.buf[: self.comps * n]
        return v.view(self.comps, n) if self.comps > 1 else v


# Each slot's particle range is padded to a whole number of wavefronts with
# excluded particles, so that no wavefront holds targets of two slots (the
# batch's SPH_BATCH_WAVE_ALIGNED kernels).
WAVE = 64


def padded(n: int, pad: bool = True) -> int:
    return -(-n // WAVE) * WAVE if pad else n


class BatchEngine:
    """Packed multi-case state on one GPU, stepped by the batch ABI."""

    def __init__(self, cap_particles: int, cap_cells: int, max_slots: int = 256,
                 device="cuda", use_graph: bool = True, cell_div: int = 1,
                 reuse_cells: bool = True, pad_slots: bool = True, four_lanes: bool = False):
        """four_lanes: slots of at most 131,072 particles take four lanes per
        target in the interaction (SPH_BATCH_FOUR_LANES).  Off by default: on
        a queued stream the batch fills the GPU, and one lane per target is
        then faster (512-request stream: 3.26 against 3.08 solves/s)."""
        self.dev = torch.device(device)
        # one binning per step: the n+1/2 interaction reuses the cells of
        # state n (sph_batch_refresh_view, SPH_INTERACT_REUSE_CELLS); the
        # state then alternates between the two buffers, `cur` holding it
        self.reuse = bool(reuse_cells)
        self.pad = bool(pad_slots)
        self.four_lanes = bool(four_lanes)
        self.shifting = False
        self.cur = 0
        self.cap_n = int(cap_particles)
        self.cap_cells = int(cap_cells)
        self.max_slots = int(max_slots)
        self.cell_div = int(cell_div)
        self.use_graph = use_graph
        d = self.dev
        mk = lambda c, t: _Flat(c, self.cap_n, t, d)  # noqa: E731
        self._state = [dict(pos=mk(3, torch.float64), vel=mk(3, torch.float32),
                            rho=mk(1, torch.float32), type=mk(1, torch.uint8),
                            id=mk(1, torch.int32)) for _ in range(2)]
        self._saved = [dict(pos=mk(3, torch.float64), vel=mk(3, torch.float32),
                            rho=mk(1, torch.float32)) for _ in range(2)]
        self._key = mk(1, torch.int32)
        self._perm = mk(1, torch.int32)
        self._ace = mk(3, torch.float32)
        self._arho = mk(1, torch.float32)
        self.cell_start = torch.zeros(self.cap_cells + 1, dtype=torch.int32, device=d)
        self.dt = torch.zeros(self.max_slots, dtype=torch.float64, device=d)
        self.dt_half = torch.zeros(self.max_slots, dtype=torch.float64, device=d)
        self.t = torch.zeros(self.max_slots, dtype=torch.float64, device=d)
        self.inter = torch.zeros((self.max_slots, 2), dtype=torch.int64, device=d)
        self.table = torch.zeros(S.lib.sph_batch_table_bytes(self.max_slots), dtype=torch.uint8,
                                 device=d)
        # workspace sized for the largest batch: the layout grows with both
        # the particle and the slot count
        self.ws = None
        self.slots: List[Request] = []
        self.offsets = [0]
        self.batch: Optional[S.SphBatch] = None
        self.graphs = {}   # captured step per buffer holding the current state
        self.steps_run = 0
        self.repacks = 0
        self.repack_s = 0.0    # host time spent repacking (copies, table upload)
        self.capture_s = 0.0   # host time spent capturing step graphs

    # ------------------------------------------------------------ capacity
    def fits(self, slots: List[Request], req: Request) -> bool:
        """Footprint admission: a free slot, particle capacity (HBM) and cell
        capacity for `slots` plus `req`."""
        n_after = sum(padded(r.n, self.pad) for r in slots) + padded(req.n, self.pad)
        cells_after = sum(r.case.params.ncell_total() + 1 for r in slots + [req])
        return (len(slots) + 1 <= self.max_slots and n_after <= self.cap_n
                and cells_after <= self.cap_cells)

    # -------------------------------------------------------------- layout
    def _dev_state(self, idx, n) -> S.DeviceState:
        st = self._state[idx]
        return S.DeviceState(pos=st["pos"].view(n), vel=st["vel"].view(n), rho=st["rho"].view(n),
                             type=st["type"].view(n), id=st["id"].view(n))

    def _dev_saved(self, idx, n) -> S.DeviceState:
        st = self._saved[idx]
        return S.DeviceState(pos=st["pos"].view(n), vel=st["vel"].view(n), rho=st["rho"].view(n))

    def repack(self, keep: List[Request], add: List[Request]):
        """New composition: surviving slots (their current state) followed by
        the new cases (uploaded).  Per-slot t carries over."""
        t0 = time.perf_counter()
        try:
            self._repack(keep, add)
        finally:
            self.repack_s += time.perf_counter() - t0

    def _repack(self, keep: List[Request], add: List[Request]):
        old_n = self.offsets[-1]
        old_index = {id(r): k for k, r in enumerate(self.slots)}
        src = self._dev_state(self.cur, old_n) if old_n > 0 else None
        t_old = self.t[: len(self.slots)].clone()
        new_slots = keep + add
        offsets = [0]
        for r in new_slots:
            offsets.append(offsets[-1] + padded(r.n, self.pad))
        n = offsets[-1]
        if n > self.cap_n:
            raise S.SphError(f"batch of {n} particles (slots padded to whole wavefronts) "
                             f"exceeds the particle capacity {self.cap_n}")
        dst = self._dev_state(1 - self.cur, n)
        t_new = torch.zeros(len(new_slots), dtype=torch.float64, device=self.dev)
        for k, r in enumerate(new_slots):
            o0, o1 = offsets[k], offsets[k + 1]
            if id(r) in old_index:
                j = old_index[id(r)]
                s0, s1 = self.offsets[j], self.offsets[j + 1]
                dst.pos[:, o0:o1] = src.pos[:, s0:s1]
                dst.vel[:, o0:o1] = src.vel[:, s0:s1]
                dst.rho[o0:o1] = src.rho[s0:s1]
                dst.type[o0:o1] = src.type[s0:s1]
                dst.id[o0:o1] = src.id[s0:s1]
                t_new[k] = t_old[j]
            else:
                pos, vel = to_3d(r.case)
                o2 = o0 + r.n  # the case's particles, then excluded padding
                dst.pos[:, o0:o2] = torch.from_numpy(pos).to(self.dev)
                dst.vel[:, o0:o2] = torch.from_numpy(vel).to(self.dev)
                dst.rho[o0:o2] = torch.from_numpy(r.case.rho).to(self.dev)
                dst.type[o0:o2] = torch.from_numpy(r.case.type).to(self.dev)
                dst.pos[:, o2:o1] = 0.0
                dst.vel[:, o2:o1] = 0.0
                dst.rho[o2:o1] = float(r.case.params.rho0)
                dst.type[o2:o1] = K.EXCLUDED
                dst.id[o0:o1] = torch.arange(o1 - o0, dtype=torch.int32, device=self.dev)
        self.cur = 1 - self.cur
        self.slots = new_slots
        self.offsets = offsets
        ns = len(new_slots)
        self.t[:ns] = t_new
        self.inter[:ns] = 0
        self.graphs = {}
        self.repacks += 1
        if ns == 0:
            self.batch = None
            return
        params = [S.make_params(r.case.params) for r in new_slots]
        # particle shifting after each corrector when some slot takes it
        self.shifting = any(float(getattr(r.case.params, "shift_coef", 0.0)) > 0.0
                            for r in new_slots)
        b, host = S.sph_batch_describe(params, offsets, four_lanes=self.four_lanes)
        if b.key_cells + 1 > self.cell_start.numel():
            raise S.SphError("batch exceeds the cell capacity")
        self.table[: host.size] = torch.from_numpy(host).to(self.dev)
        b.table = self.table.data_ptr()
        need = S.sph_batch_workspace_bytes(b)
        if self.ws is None or self.ws.numel() < need:
            cap = S.SphBatch(self.max_slots, b.cell_div, self.cap_n, self.cap_cells, None)
            self.ws = torch.zeros(max(need, S.sph_batch_workspace_bytes(cap)), dtype=torch.uint8,
                                  device=self.dev)
        self.batch = b
        # per-slot error words are indexed by slot: start the composition clean
        S.sph_batch_clear_errors(b, self.ws)

    # ---------------------------------------------------------------- step
    def _step(self, cur: int):
        """One symplectic step of every slot from the state in buffer `cur`;
        returns the buffer that holds the result."""
        b = self.batch
        n = b.n_total
        a, bb = self._dev_state(cur, n), self._dev_state(1 - cur, n)
        s0, s1 = self._dev_saved(0, n), self._dev_saved(1, n)
        key, perm = self._key.view(n), self._perm.view(n)
        ace, arho = self._ace.view(n), self._arho.view(n)
        ns = b.n_slots
        dt, dth, t, inter = self.dt[:ns], self.dt_half[:ns], self.t[:ns], self.inter[:ns]
        S.sph_batch_bin_cells(b, a, bb, key, perm, self.cell_start, self.ws)
        S.sph_batch_interact(b, bb, key, self.cell_start, ace, arho, self.ws)
        S.sph_batch_reduce_dt(b, dt, self.ws, interactions=inter)
        S.sph_batch_symplectic_step(b, 0, dt, t, s0, bb, ace, arho, self.ws)
        if self.reuse:
            S.sph_batch_refresh_view(b, bb, key, self.ws)
            S.sph_batch_interact(b, bb, key, self.cell_start, ace, arho, self.ws,
                                 flags=S.SPH_INTERACT_REUSE_CELLS)
            S.sph_batch_reduce_dt(b, dth, self.ws, interactions=inter)
            S.sph_batch_symplectic_step(b, 1, dt, t, s0, bb, ace, arho, self.ws)
            if self.shifting:
                S.sph_batch_shifting(b, bb, key, self.cell_start, dt, self.ws,
                                     flags=S.SPH_INTERACT_REUSE_CELLS)
            return 1 - cur
        S.sph_batch_bin_cells(b, bb, a, key, perm, self.cell_start, self.ws, carry_in=s0,
                              carry_out=s1)
        S.sph_batch_interact(b, a, key, self.cell_start, ace, arho, self.ws)
        S.sph_batch_reduce_dt(b, dth, self.ws, interactions=inter)
        S.sph_batch_symplectic_step(b, 1, dt, t, s1, a, ace, arho, self.ws)
        if self.shifting:
            S.sph_batch_shifting(b, a, key, self.cell_start, dt, self.ws)
        return cur

    def run(self, k: int):
        if self.batch is None or k <= 0:
            return
        for _ in range(k):
            if not self.use_graph:
                self.cur = self._step(self.cur)
                continue
            entry = self.graphs.get(self.cur)
            if entry is None:
                t0 = time.perf_counter()
                torch.cuda.synchronize()
                g = torch.cuda.CUDAGraph()
                with torch.cuda.graph(g):
                    nxt = self._step(self.cur)
                entry = self.graphs[self.cur] = (g, nxt)
                self.capture_s += time.perf_counter() - t0
            entry[0].replay()
            self.cur = entry[1]
        self.steps_run += k

    # ------------------------------------------------------------- results
    def harvest(self, done: List[int], keep_results: bool):
        """After the stream has finished: adds every slot's pair count to its
        request (the counters restart at the next repack) and collects error
        words and, if asked, final states of the slots in `done`."""
        torch.cuda.synchronize()
        ns = len(self.slots)
        errs = S.sph_batch_read_errors(self.batch, self.ws)
        inter = self.inter[:ns].cpu().numpy()
        for k, r in enumerate(self.slots):
            r.interactions += int(inter[k, 0])
        for k in done:
            r = self.slots[k]
            r.error = int(errs[k])
            if keep_results:
                r.result = self.slot_result(k)

    def slot_result(self, k: int) -> dict:
        """Final state of slot k in the case's original particle order."""
        r = self.slots[k]
        o0, o1 = self.offsets[k], self.offsets[k + 1]
        st = self._dev_state(self.cur, self.offsets[-1])
        ids = st.id[o0:o1].cpu().numpy().view(np.uint32).astype(np.int64)
        inv = np.empty_like(ids)
        inv[ids] = np.arange(ids.shape[0])
        inv = inv[: r.n]  # the padding's ids follow the case's
        pos = st.pos[:, o0:o1].cpu().numpy()[:, inv]
        vel = st.vel[:, o0:o1].cpu().numpy()[:, inv]
        pos, vel = from_3d(r.case.params.dim, pos, vel)
        return dict(pos=pos, vel=vel, rho=st.rho[o0:o1].cpu().numpy()[inv],
                    type=st.type[o0:o1].cpu().numpy()[inv], t=float(self.t[k].item()))


# ----------------------------------------------------------------- drivers
def make_stream(n_requests: int, rate: float, seed: int = 0, n_min=2000, n_max=500_000,
                steps_min=1000, steps_max=5000, steps_scale: float = 1.0) -> List[Request]:
    """The seeded request stream: Poisson arrivals at `rate`/s; each request a
    2-D or 3-D dam break or sloshing case with a log-uniform particle count and
    a uniform step count (scaled by steps_scale)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for rid in range(n_requests):
        t += rng.exponential(1.0 / rate)
        case = K.random_serving_case(rng, n_min=n_min, n_max=n_max)
        steps = int(rng.integers(steps_min, steps_max + 1))
        steps = max(1, int(round(steps * steps_scale)))
        out.append(Request(rid=rid, case=case, steps=steps, arrival=t))
    return out


class _Progress:
    """A line on stderr at most every `every` seconds (long streams)."""

    def __init__(self, label: str, total: int, every: float = 30.0):
        self.label, self.total, self.every = label, total, every
        self.last = time.perf_counter()

    def __call__(self, done: int, now: float):
        if self.every > 0 and time.perf_counter() - self.last >= self.every:
            self.last = time.perf_counter()
            import sys
            print(f"[serve] {self.label}: {done}/{self.total} requests done at {now:.1f} s",
                  file=sys.stderr, flush=True)


def serve_batched(reqs: List[Request], engine: BatchEngine, max_chunk: int = 64,
                  keep_results: bool = False, progress_s: float = 30.0) -> dict:
    """Continuous batching: admit arrived requests whenever a slot and memory
    are free, run the batch until the next case finishes (at most max_chunk
    steps, so that arrivals wait briefly), retire finished cases, repeat."""
    pending = sorted(reqs, key=lambda r: r.arrival)
    left = {}
    prog = _Progress("batched", len(reqs), progress_s)
    t0 = time.perf_counter()
    while pending or engine.slots:
        now = time.perf_counter() - t0
        prog(sum(1 for r in reqs if r.finish is not None), now)
        done = [k for k, r in enumerate(engine.slots) if left[r.rid] == 0]
        keep = [r for r in engine.slots if left[r.rid] > 0]
        add = []
        while pending and pending[0].arrival <= now and engine.fits(keep + add, pending[0]):
            r = pending.pop(0)
            r.start = now
            left[r.rid] = r.steps
            add.append(r)
        if done or add:
            if engine.slots:
                engine.harvest(done, keep_results)
                fin = time.perf_counter() - t0
                for k in done:
                    engine.slots[k].finish = fin
            engine.repack(keep, add)
        if not engine.slots:
            if pending:
                wait = pending[0].arrival - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(wait)
            continue
        k = min(min(left[r.rid] for r in engine.slots), max_chunk)
        engine.run(k)
        for r in engine.slots:
            left[r.rid] -= k
        torch.cuda.synchronize()
    makespan = time.perf_counter() - t0
    inter_total = sum(r.interactions for r in reqs)
    return _summary(reqs, makespan, inter_total, dict(repacks=engine.repacks,
                                                      batch_steps=engine.steps_run,
                                                      repack_s=engine.repack_s,
                                                      capture_s=engine.capture_s))


def serve_plain(reqs: List[Request], device="cuda", use_graph: bool = True,
                keep_results: bool = False, progress_s: float = 30.0) -> dict:
    """One case at a time, in arrival order, with the single-case calls."""
    prog = _Progress("plain", len(reqs), progress_s)
    t0 = time.perf_counter()
    inter_total = 0
    for k, r in enumerate(sorted(reqs, key=lambda x: x.arrival)):
        now = time.perf_counter() - t0
        prog(k, now)
        if r.arrival > now:
            time.sleep(r.arrival - now)
        r.start = time.perf_counter() - t0
        sim = Simulation(r.case, device)
        if use_graph and r.steps > 2:
            sim.step()
            k = 2 if sim.reuse_cells else 1  # (the buffers alternate per step)
            sim.capture(k)
            reps = (r.steps - 1) // k
            sim.replay(reps)
            sim.run(r.steps - 1 - reps * k)
        else:
            sim.run(r.steps)
        torch.cuda.synchronize()
        r.error = sim.error()
        r.interactions = sim.interaction_count()
        if keep_results:
            r.result = sim.host_state()
        r.finish = time.perf_counter() - t0
        inter_total += r.interactions
        del sim
    makespan = time.perf_counter() - t0
    return _summary(reqs, makespan, inter_total, {})


def _summary(reqs, makespan, inter_total, extra) -> dict:
    lat = np.array([r.latency for r in reqs])
    return dict(requests=len(reqs), makespan_s=makespan, solves_per_s=len(reqs) / makespan,
                interactions_per_s=inter_total / makespan,
                p50_latency_s=float(np.percentile(lat, 50)),
                p99_latency_s=float(np.percentile(lat, 99)),
                mean_latency_s=float(lat.mean()),
                errors=int(sum(1 for r in reqs if r.error)),
                error_bits={str(r.rid): int(r.error) for r in reqs if r.error}, **extra)
