"""One-case step loop over the libsph C ABI (NL -> PI -> SU, Section 5.1).

A symplectic step (Section 2.5.2) is
    bin(n) -> interact(n) -> reduce_dt -> predictor -> bin(n+1/2, carrying the
    saved state n) -> interact(n+1/2) -> corrector (t += dt)
with dt and t kept in device memory, so a step enqueues no host work and can
be captured once in a HIP graph and replayed.  With reuse_cells (the default
where it applies) the second binning is replaced by a refresh of the
interaction view on the cells of the first, and the second interaction
searches one cell further with the cut widened by the largest displacement
since the binning: the same pairs, one sort and one reorder fewer per step;
the state then alternates between the two buffers from step to step.
"""
from __future__ import annotations

from typing import Optional

import numpy as np
import torch

from . import sph as S


class Simulation:
    def __init__(self, case, device="cuda", cell_div: Optional[int] = None, flags: int = 0,
                 integrator: str = "symplectic", verlet_ns: int = 40,
                 reuse_cells: Optional[bool] = None, f64_state: bool = False,
                 neighbour_list: bool = False, list_skin: Optional[float] = None):
        """f64_state: the all-FP64 arm of the precision study -- velocities
        and densities held and advanced in FP64, every pair evaluated in FP64
        (SPH_INTERACT_F64_STATE), FP64 rates."""
        cp = case.params
        self.f64 = bool(f64_state)
        if self.f64:
            if flags not in (0, S.SPH_INTERACT_F64_STATE) or integrator != "symplectic":
                raise ValueError("the all-FP64 state takes its own interaction arm and the "
                                 "symplectic integrator")
            flags = S.SPH_INTERACT_F64_STATE
        if cell_div is not None and cell_div != cp.cell_div:
            raise ValueError("cell_div is fixed by the case's grid")
        self.case = case
        self.cp = cp
        self.params = S.make_params(cp)
        self.dim = int(cp.dim)
        self.n = n = case.n
        dev = torch.device(device)
        self.device = dev
        # modified DBC needs the wall ghost vectors, carried through the sorts
        self.mdbc = int(getattr(cp, "boundary", 0)) == 1
        if self.f64 and (self.mdbc or getattr(case, "bodies", None)
                         or float(getattr(cp, "shift_coef", 0.0)) > 0.0):
            raise ValueError("the all-FP64 state takes DBC walls, no floating bodies and no "
                             "shifting")
        self.states = [S.DeviceState.from_case(case, dev, with_normal=self.mdbc, f64=self.f64),
                       S.DeviceState.empty(self.dim, n, dev, with_normal=self.mdbc,
                                           f64=self.f64)]
        self.saved = [S.DeviceState.empty(self.dim, n, dev, with_type=False, with_id=False,
                                          f64=self.f64)
                      for _ in range(2)]
        self.key = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
        self.perm = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
        self.cell_start = torch.empty(cp.ncell_total() + 1, dtype=torch.int32, device=dev)
        rate = torch.float64 if self.f64 else torch.float32
        self.ace = torch.zeros((self.dim, max(n, 1)), dtype=rate, device=dev)
        self.arho = torch.zeros(max(n, 1), dtype=rate, device=dev)
        self.ws = torch.zeros(S.sph_workspace_bytes(self.params, n), dtype=torch.uint8, device=dev)
        self.dt = torch.zeros(1, dtype=torch.float64, device=dev)
        self.t = torch.zeros(1, dtype=torch.float64, device=dev)
        self.dt_half = torch.zeros(1, dtype=torch.float64, device=dev)
        self.interactions = torch.zeros(2, dtype=torch.int64, device=dev)
        self.steps_done = 0
        self.graph = None
        # with `timing`, record events around these calls only (None: all)
        self.timed_calls = None
        # sph_interact flags: 0 for the production pass, or a precision-study
        # arm (S.SPH_INTERACT_F64 / S.SPH_INTERACT_ABS_F32)
        self.flags = int(flags)
        # "symplectic" (Eq. 33-34, two interactions per step) or "verlet"
        # (Eq. 30, with the Eq. 31 step first and every verlet_ns steps)
        if integrator not in ("symplectic", "verlet"):
            raise ValueError(f"unknown integrator {integrator}")
        if integrator == "verlet" and verlet_ns < 1:
            raise ValueError("verlet_ns must be >= 1")
        self.integrator = integrator
        self.verlet_ns = int(verlet_ns)
        # floating bodies (Section 3.2): the device body table, advanced by
        # sph_floating_step after each symplectic phase
        # particle shifting (Section 2.8) after each corrector
        self.shifting = float(getattr(cp, "shift_coef", 0.0)) > 0.0
        if self.shifting and integrator != "symplectic":
            raise ValueError("particle shifting takes the symplectic integrator")
        # the second interaction of a step (and shifting) on the cells of the
        # first (not with modified DBC or a precision-study arm, whose passes
        # search the cells without a displacement margin)
        # (a periodic component needs 2 (cell_div + 1) + 1 cells for the
        # longer walk on reused cells)
        per_cells = [cp.ncell[k] // (cp.x_sub if k == 0 else 1) for k in range(cp.dim)
                     if cp.period[k] > 0]
        can_reuse = (integrator == "symplectic" and not self.mdbc
                     and (self.flags & ~S.SPH_INTERACT_ONE_LANE) in (0, S.SPH_DIAG_COUNT_F64)
                     and all(c >= 2 * (cp.cell_div + 1) + 1 for c in per_cells))
        if reuse_cells and not can_reuse:
            raise ValueError("reuse_cells needs the symplectic integrator, DBC walls, no "
                             "precision-study arm and periodic components of at least "
                             "2 (cell_div + 1) + 1 cells")
        self.reuse_cells = can_reuse if reuse_cells is None else bool(reuse_cells)
        # neighbour lists (sph_build_list / sph_interact_list) for both passes
        # of a reused-cells step: default formulation, DBC walls, no floating
        # bodies, shifting or periodic components, one lane per target.  Off
        # unless asked for: on the 1.32M-particle dam break a step with lists
        # (build 0.37 ms, passes 0.53 and 0.59 ms) is slower than the cell
        # walk (passes 0.46 and 0.47 ms)
        list_ok = (self.reuse_cells and (self.flags & ~S.SPH_INTERACT_ONE_LANE) in
                   (0, S.SPH_DIAG_COUNT_F64) and int(getattr(cp, "kernel", 0)) == 0
                   and int(getattr(cp, "viscosity", 0)) == 0 and int(cp.ddt) != 2
                   and int(getattr(cp, "floating", 0)) == 0 and not per_cells
                   and not getattr(case, "bodies", None)
                   and float(getattr(cp, "shift_coef", 0.0)) == 0.0)
        if neighbour_list and not list_ok:
            raise ValueError("neighbour lists need the reused-cells step with the default "
                             "formulation, DBC walls and no floating bodies, shifting or "
                             "periodic components")
        self.neighbour_list = bool(neighbour_list)
        self.list = None
        if self.neighbour_list:
            self.list = torch.empty(S.sph_list_bytes(self.params, n), dtype=torch.uint8,
                                    device=dev)
            # the smallest skin; each step takes at least 1.5 times twice the
            # last step's largest half-step displacement (SPH_LIST_ADAPTIVE_SKIN)
            self.list_skin = 0.01 * float(cp.h) if list_skin is None else float(list_skin)
        self.bodies = None
        if getattr(case, "bodies", None):
            if integrator != "symplectic":
                raise ValueError("floating bodies take the symplectic integrator")
            if int(getattr(cp, "floating", 0)) != 1:
                raise ValueError("a case with bodies needs params.floating = 1")
            self.bodies = S.bodies_to_device(case.bodies, dev)

    # ------------------------------------------------------------------ step
    @property
    def state(self) -> S.DeviceState:
        return self.states[0]

    def step(self, stream=None, timing: Optional[dict] = None):
        """One symplectic step.  With `timing` (a dict), HIP events are
        recorded on the stream around each call, appended to
        timing[name] as (start, end) pairs."""
        if self.integrator == "verlet":
            return self._step_verlet(stream, timing)
        if self.reuse_cells:
            return self._step_reuse(stream, timing)
        P, n = self.params, self.n
        a, b = self.states
        s0, s1 = self.saved

        def call(name, fn, *args, **kw):
            if timing is None or (self.timed_calls and name not in self.timed_calls):
                fn(*args, **kw)
                return
            st = stream if stream is not None else torch.cuda.current_stream()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(st)
            fn(*args, **kw)
            e1.record(st)
            timing.setdefault(name, []).append((e0, e1))

        call("bin_cells", S.sph_bin_cells, P, n, a, b, self.key, self.perm, self.cell_start,
             self.ws, stream=stream)
        if self.mdbc:
            call("mdbc", S.sph_mdbc, P, n, b, self.key, self.cell_start, self.ws, stream=stream)
        call("interact", S.sph_interact, P, n, b, self.key, self.cell_start, self.ace, self.arho,
             self.ws, flags=self.flags, stream=stream)
        call("reduce_dt", S.sph_reduce_dt, P, n, self.dt, self.ws,
             interactions=self.interactions, stream=stream)
        call("symplectic", S.sph_symplectic_step, P, n, 0, self.dt, self.t, s0, b, self.ace,
             self.arho, self.ws, stream=stream)
        if self.bodies is not None:
            call("floating", S.sph_floating_step, P, n, 0, self.dt, self.bodies, s0, b, self.ace,
                 self.ws, stream=stream)
        call("bin_cells", S.sph_bin_cells, P, n, b, a, self.key, self.perm, self.cell_start,
             self.ws, carry_in=s0, carry_out=s1, stream=stream)
        if self.mdbc:
            call("mdbc", S.sph_mdbc, P, n, a, self.key, self.cell_start, self.ws, stream=stream)
        call("interact", S.sph_interact, P, n, a, self.key, self.cell_start, self.ace, self.arho,
             self.ws, flags=self.flags, stream=stream)
        # pair count of the second pass (its dt is not used: Eq. 35 is taken
        # at state n for both half steps)
        call("reduce_dt", S.sph_reduce_dt, P, n, self.dt_half, self.ws,
             interactions=self.interactions, stream=stream)
        call("symplectic", S.sph_symplectic_step, P, n, 1, self.dt, self.t, s1, a, self.ace,
             self.arho, self.ws, stream=stream)
        if self.bodies is not None:
            call("floating", S.sph_floating_step, P, n, 1, self.dt, self.bodies, s1, a, self.ace,
                 self.ws, stream=stream)
        if self.shifting:
            call("shifting", S.sph_shifting, P, n, a, self.key, self.cell_start, self.dt, self.ws,
                 stream=stream)
        self.steps_done += 1

    def _call(self, stream, timing):
        def call(name, fn, *args, **kw):
            if timing is None or (self.timed_calls and name not in self.timed_calls):
                fn(*args, **kw)
                return
            st = stream if stream is not None else torch.cuda.current_stream()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(st)
            fn(*args, **kw)
            e1.record(st)
            timing.setdefault(name, []).append((e0, e1))
        return call

    def _step_reuse(self, stream, timing):
        """A symplectic step with one binning: the n+1/2 interaction reuses
        the cells of state n (sph_refresh_view, SPH_INTERACT_REUSE_CELLS);
        the saved state n needs no carrying, and the result stays in the
        other buffer (the two swap roles every step)."""
        P, n = self.params, self.n
        a, b = self.states
        s0 = self.saved[0]
        call = self._call(stream, timing)
        call("bin_cells", S.sph_bin_cells, P, n, a, b, self.key, self.perm, self.cell_start,
             self.ws, stream=stream)
        if self.neighbour_list:
            call("build_list", S.sph_build_list, P, n, b, self.key, self.cell_start,
                 self.list_skin, self.list, self.ws, flags=S.SPH_LIST_ADAPTIVE_SKIN,
                 stream=stream)
            call("interact", S.sph_interact_list, P, n, b, self.key, self.cell_start, self.list,
                 self.ace, self.arho, self.ws, flags=self.flags, stream=stream)
        else:
            call("interact", S.sph_interact, P, n, b, self.key, self.cell_start, self.ace,
                 self.arho, self.ws, flags=self.flags, stream=stream)
        call("reduce_dt", S.sph_reduce_dt, P, n, self.dt, self.ws,
             interactions=self.interactions, stream=stream)
        call("symplectic", S.sph_symplectic_step, P, n, 0, self.dt, self.t, s0, b, self.ace,
             self.arho, self.ws, stream=stream)
        if self.bodies is not None:
            call("floating", S.sph_floating_step, P, n, 0, self.dt, self.bodies, s0, b, self.ace,
                 self.ws, stream=stream)
        call("refresh_view", S.sph_refresh_view, P, n, b, self.key, self.ws, stream=stream)
        if self.neighbour_list:
            call("interact", S.sph_interact_list, P, n, b, self.key, self.cell_start, self.list,
                 self.ace, self.arho, self.ws, flags=self.flags | S.SPH_INTERACT_REUSE_CELLS,
                 stream=stream)
        else:
            call("interact", S.sph_interact, P, n, b, self.key, self.cell_start, self.ace,
                 self.arho, self.ws, flags=self.flags | S.SPH_INTERACT_REUSE_CELLS,
                 stream=stream)
        call("reduce_dt", S.sph_reduce_dt, P, n, self.dt_half, self.ws,
             interactions=self.interactions, stream=stream)
        call("symplectic", S.sph_symplectic_step, P, n, 1, self.dt, self.t, s0, b, self.ace,
             self.arho, self.ws, stream=stream)
        if self.bodies is not None:
            call("floating", S.sph_floating_step, P, n, 1, self.dt, self.bodies, s0, b, self.ace,
                 self.ws, stream=stream)
        if self.shifting:
            call("shifting", S.sph_shifting, P, n, b, self.key, self.cell_start, self.dt, self.ws,
                 flags=S.SPH_INTERACT_REUSE_CELLS, stream=stream)
        self.states = [b, a]
        self.steps_done += 1

    def _step_verlet(self, stream, timing):
        """One Verlet step: NL (carrying step n-1's velocity and density),
        PI, dt, update; the result becomes the next step's input."""
        P, n = self.params, self.n
        a, b = self.states
        s0, s1 = self.saved

        def call(name, fn, *args, **kw):
            if timing is None or (self.timed_calls and name not in self.timed_calls):
                fn(*args, **kw)
                return
            st = stream if stream is not None else torch.cuda.current_stream()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(st)
            fn(*args, **kw)
            e1.record(st)
            timing.setdefault(name, []).append((e0, e1))

        mode = 1 if self.steps_done % self.verlet_ns == 0 else 0
        call("bin_cells", S.sph_bin_cells, P, n, a, b, self.key, self.perm, self.cell_start,
             self.ws, carry_in=s0, carry_out=s1, stream=stream)
        if self.mdbc:
            call("mdbc", S.sph_mdbc, P, n, b, self.key, self.cell_start, self.ws, stream=stream)
        call("interact", S.sph_interact, P, n, b, self.key, self.cell_start, self.ace, self.arho,
             self.ws, flags=self.flags, stream=stream)
        call("reduce_dt", S.sph_reduce_dt, P, n, self.dt, self.ws,
             interactions=self.interactions, stream=stream)
        call("verlet", S.sph_verlet_step, P, n, mode, self.dt, self.t, s1, b, self.ace,
             self.arho, self.ws, stream=stream)
        self.states = [b, a]
        self.saved = [s1, s0]
        self.steps_done += 1

    def run(self, nsteps: int):
        for _ in range(int(nsteps)):
            self.step()

    # ----------------------------------------------------------- HIP graphs
    def capture(self, steps_per_graph: int = 1):
        """Captures `steps_per_graph` steps in one HIP graph (warm up first).
        With Verlet the graph must start on an Eq. 31 step and span whole
        periods of verlet_ns steps and an even number of steps (the state
        buffers alternate every step)."""
        if self.integrator == "verlet":
            k = int(steps_per_graph)
            if self.steps_done % self.verlet_ns or k % self.verlet_ns or k % 2:
                raise ValueError("a Verlet graph must start at a multiple of verlet_ns and "
                                 "span an even multiple of it")
        if self.reuse_cells and int(steps_per_graph) % 2:
            raise ValueError("with reuse_cells the state buffers alternate every step: a graph "
                             "must span an even number of steps")
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for _ in range(steps_per_graph):
                self.step()
        self.steps_done -= steps_per_graph  # capture does not execute
        self.graph = (g, steps_per_graph)
        return g

    def replay(self, times: int = 1):
        g, k = self.graph
        for _ in range(times):
            g.replay()
        self.steps_done += k * times

    # ------------------------------------------------------------- readback
    def error(self) -> int:
        return S.sph_read_error(self.ws)

    def time(self) -> float:
        return float(self.t.item())

    def host_state(self) -> dict:
        """State in the case's original particle order (numpy, FP64/FP32)."""
        st = self.state
        ids = st.id.cpu().numpy().view(np.uint32).astype(np.int64)
        inv = np.empty_like(ids)
        inv[ids] = np.arange(ids.shape[0])
        vel = st.vel64 if st.vel64 is not None else st.vel
        rho = st.rho64 if st.rho64 is not None else st.rho
        return dict(pos=st.pos.cpu().numpy()[:, inv], vel=vel.cpu().numpy()[:, inv],
                    rho=rho.cpu().numpy()[inv], type=st.type.cpu().numpy()[inv],
                    t=self.time())

    def body_state(self) -> list:
        """The floating bodies' current state (host dicts)."""
        return [] if self.bodies is None else S.bodies_from_device(self.bodies)

    def interaction_count(self) -> int:
        return int(self.interactions[0].item())
