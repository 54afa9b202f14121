"""Thin ctypes binding of libsph (include/sph.h).

Argument marshalling only: every step of the path runs in the HIP kernels of
``libsph.so``.  PyTorch supplies device memory and streams.  Importing this
module fails loudly if the library has not been built (there is no CPU
fallback).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsph.so")

SPH_OK, SPH_E_ARG, SPH_E_WORKSPACE, SPH_E_HIP = 0, -1, -2, -3
SPH_FLUID, SPH_BOUND_FIXED, SPH_BOUND_MOVING, SPH_FLOATING, SPH_EXCLUDED = 0, 1, 2, 3, 0x80
SPH_ERR_NONFINITE, SPH_ERR_EXCLUDED, SPH_ERR_DT_FLOOR, SPH_ERR_FLOATING = 1, 2, 4, 8
SPH_ERR_MARGIN = 16
SPH_ERR_LIST = 32
SPH_LIST_ADAPTIVE_SKIN = 1
SPH_MAX_BODIES = 64
SPH_DIAG_COUNT_F64 = 1
SPH_INTERACT_F64 = 2
SPH_INTERACT_ABS_F32 = 4
SPH_INTERACT_REUSE_CELLS = 8
SPH_INTERACT_ONE_LANE = 16
SPH_INTERACT_F64_STATE = 32

EXPORTS = ("sph_workspace_bytes", "sph_bin_cells", "sph_refresh_view", "sph_interact",
           "sph_interact_noalloc", "sph_list_bytes", "sph_build_list", "sph_interact_list",
           "sph_list_walks", "sph_reduce_dt",
           "sph_symplectic_step", "sph_verlet_step", "sph_mdbc", "sph_floating_step",
           "sph_shifting",
           "sph_read_error", "sph_clear_error", "sph_strerror",
           "sph_batch_table_bytes", "sph_batch_describe", "sph_batch_workspace_bytes",
           "sph_batch_bin_cells", "sph_batch_interact", "sph_batch_refresh_view",
           "sph_batch_reduce_dt",
           "sph_batch_symplectic_step", "sph_batch_shifting", "sph_batch_read_errors",
           "sph_batch_clear_errors")
SPH_BATCH_MAX_SLOTS = 4096
SPH_BATCH_WAVE_ALIGNED = 1
SPH_BATCH_FOUR_LANES = 2
SPH_BATCH_GENERAL = 4
SPH_BATCH_PERIODIC = 8
SPH_NOALLOC_MAX_N = 2097152


class SphParams(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("cell_div", C.c_int32), ("ddt", C.c_int32),
        ("ncell", C.c_int32 * 3), ("x_sub", C.c_int32), ("boundary", C.c_int32),
        ("origin", C.c_double * 3),
        ("cell_size", C.c_double), ("inv_cell_size", C.c_double),
        ("h", C.c_double), ("rho0", C.c_double), ("gamma", C.c_double),
        ("c0", C.c_double), ("alpha", C.c_double), ("delta", C.c_double),
        ("eta2", C.c_double), ("cfl", C.c_double), ("mass_fluid", C.c_double),
        ("mass_bound", C.c_double), ("gravity", C.c_double * 3),
        ("motion_amp", C.c_double), ("motion_omega", C.c_double),
        ("dt_floor", C.c_double), ("kernel", C.c_int32), ("viscosity", C.c_int32),
        ("visc_nu", C.c_double), ("floating", C.c_int32), ("pad0", C.c_int32),
        ("period", C.c_double * 3), ("shift_coef", C.c_double), ("shift_fs", C.c_double),
    ]


class SphBody(C.Structure):
    _fields_ = [("id_first", C.c_int64), ("count", C.c_int64), ("mass", C.c_double),
                ("center", C.c_double * 3), ("vel", C.c_double * 3), ("omega", C.c_double * 3),
                ("center_n", C.c_double * 3), ("vel_n", C.c_double * 3),
                ("omega_n", C.c_double * 3), ("force", C.c_double * 3),
                ("torque", C.c_double * 3)]


class SphState(C.Structure):
    _fields_ = [("pos", C.c_void_p), ("vel", C.c_void_p), ("rho", C.c_void_p),
                ("type", C.c_void_p), ("id", C.c_void_p), ("normal", C.c_void_p),
                ("vel64", C.c_void_p), ("rho64", C.c_void_p)]


class SphBatch(C.Structure):
    _fields_ = [("n_slots", C.c_int32), ("cell_div", C.c_int32), ("n_total", C.c_int64),
                ("key_cells", C.c_int64), ("table", C.c_void_p), ("flags", C.c_uint32),
                ("lanes", C.c_uint32)]


class SphError(RuntimeError):
    pass


def _load() -> C.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"libsph.so not found at {LIB_PATH}: build it with "
            "`python -m paper_2104_00537_amd.build` (there is no CPU fallback)")
    L = C.CDLL(LIB_PATH)
    P, VP = C.POINTER, C.c_void_p
    L.sph_workspace_bytes.restype = C.c_size_t
    L.sph_workspace_bytes.argtypes = [P(SphParams), C.c_int64]
    L.sph_bin_cells.restype = C.c_int32
    L.sph_bin_cells.argtypes = [P(SphParams), C.c_int64, P(SphState), P(SphState),
                                P(SphState), P(SphState), VP, VP, VP, VP, C.c_size_t, VP]
    L.sph_interact.restype = C.c_int32
    L.sph_interact.argtypes = [P(SphParams), C.c_int64, P(SphState), VP, VP, VP, VP, VP, VP,
                               C.c_uint32, VP, C.c_size_t, VP]
    L.sph_interact_noalloc.restype = C.c_int32
    L.sph_interact_noalloc.argtypes = [P(SphParams), C.c_int64, P(SphState), VP, VP, VP, VP, VP,
                                       VP, C.c_uint32, VP]
    L.sph_list_bytes.restype = C.c_size_t
    L.sph_list_bytes.argtypes = [P(SphParams), C.c_int64]
    L.sph_build_list.restype = C.c_int32
    L.sph_build_list.argtypes = [P(SphParams), C.c_int64, P(SphState), VP, VP, C.c_double,
                                 C.c_uint32, VP, C.c_size_t, VP, C.c_size_t, VP]
    L.sph_interact_list.restype = C.c_int32
    L.sph_interact_list.argtypes = [P(SphParams), C.c_int64, P(SphState), VP, VP, VP, C.c_size_t,
                                    VP, VP, VP, VP, C.c_uint32, VP, C.c_size_t, VP]
    L.sph_list_walks.restype = C.c_int64
    L.sph_list_walks.argtypes = [VP]
    L.sph_refresh_view.restype = C.c_int32
    L.sph_refresh_view.argtypes = [P(SphParams), C.c_int64, P(SphState), VP, VP, C.c_size_t, VP]
    L.sph_reduce_dt.restype = C.c_int32
    L.sph_reduce_dt.argtypes = [P(SphParams), C.c_int64, VP, VP, VP, VP, C.c_size_t, VP]
    L.sph_symplectic_step.restype = C.c_int32
    L.sph_symplectic_step.argtypes = [P(SphParams), C.c_int64, C.c_int32, VP, VP,
                                      P(SphState), P(SphState), VP, VP, VP, C.c_size_t, VP]
    L.sph_verlet_step.restype = C.c_int32
    L.sph_verlet_step.argtypes = [P(SphParams), C.c_int64, C.c_int32, VP, VP,
                                  P(SphState), P(SphState), VP, VP, VP, C.c_size_t, VP]
    L.sph_mdbc.restype = C.c_int32
    L.sph_mdbc.argtypes = [P(SphParams), C.c_int64, P(SphState), VP, VP, VP, C.c_size_t, VP]
    L.sph_floating_step.restype = C.c_int32
    L.sph_floating_step.argtypes = [P(SphParams), C.c_int64, C.c_int32, VP, VP, C.c_int32,
                                    P(SphState), P(SphState), VP, VP, C.c_size_t, VP]
    L.sph_shifting.restype = C.c_int32
    L.sph_shifting.argtypes = [P(SphParams), C.c_int64, P(SphState), VP, VP, VP, VP, VP,
                               C.c_uint32, VP, C.c_size_t, VP]
    L.sph_read_error.restype = C.c_int32
    L.sph_read_error.argtypes = [VP]
    L.sph_clear_error.restype = C.c_int32
    L.sph_clear_error.argtypes = [VP, VP]
    L.sph_strerror.restype = C.c_char_p
    L.sph_strerror.argtypes = [C.c_int32]
    L.sph_batch_table_bytes.restype = C.c_size_t
    L.sph_batch_table_bytes.argtypes = [C.c_int32]
    L.sph_batch_describe.restype = C.c_int32
    L.sph_batch_describe.argtypes = [P(SphParams), P(C.c_int64), C.c_int32, C.c_uint32, VP,
                                     C.c_size_t, P(SphBatch)]
    L.sph_batch_workspace_bytes.restype = C.c_size_t
    L.sph_batch_workspace_bytes.argtypes = [P(SphBatch)]
    L.sph_batch_bin_cells.restype = C.c_int32
    L.sph_batch_bin_cells.argtypes = [P(SphBatch), P(SphState), P(SphState), P(SphState),
                                      P(SphState), VP, VP, VP, VP, C.c_size_t, VP]
    L.sph_batch_interact.restype = C.c_int32
    L.sph_batch_interact.argtypes = [P(SphBatch), P(SphState), VP, VP, VP, VP, VP, VP,
                                     C.c_uint32, VP, C.c_size_t, VP]
    L.sph_batch_refresh_view.restype = C.c_int32
    L.sph_batch_refresh_view.argtypes = [P(SphBatch), P(SphState), VP, VP, C.c_size_t, VP]
    L.sph_batch_reduce_dt.restype = C.c_int32
    L.sph_batch_reduce_dt.argtypes = [P(SphBatch), VP, VP, VP, C.c_size_t, VP]
    L.sph_batch_symplectic_step.restype = C.c_int32
    L.sph_batch_symplectic_step.argtypes = [P(SphBatch), C.c_int32, VP, VP, P(SphState),
                                            P(SphState), VP, VP, VP, C.c_size_t, VP]
    L.sph_batch_shifting.restype = C.c_int32
    L.sph_batch_shifting.argtypes = [P(SphBatch), P(SphState), VP, VP, VP, VP, VP, C.c_uint32, VP,
                                     C.c_size_t, VP]
    L.sph_batch_read_errors.restype = C.c_int32
    L.sph_batch_read_errors.argtypes = [P(SphBatch), VP, VP]
    L.sph_batch_clear_errors.restype = C.c_int32
    L.sph_batch_clear_errors.argtypes = [P(SphBatch), VP, VP]
    return L


lib = _load()


def _check(st: int, what: str):
    if st != SPH_OK:
        raise SphError(f"{what}: {lib.sph_strerror(st).decode()} ({st})")


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream) -> Optional[C.c_void_p]:
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def make_params(cp) -> SphParams:
    """SphParams from a ``cases.CaseParams``."""
    p = SphParams()
    p.dim, p.cell_div, p.ddt = int(cp.dim), int(cp.cell_div), int(cp.ddt)
    p.x_sub = int(getattr(cp, "x_sub", 1))
    p.boundary = int(getattr(cp, "boundary", 0))
    p.kernel = int(getattr(cp, "kernel", 0))
    p.viscosity = int(getattr(cp, "viscosity", 0))
    p.visc_nu = float(getattr(cp, "visc_nu", 0.0))
    p.floating = int(getattr(cp, "floating", 0))
    period = getattr(cp, "period", (0.0, 0.0, 0.0))
    for k in range(3):
        p.period[k] = float(period[k])
    p.shift_coef = float(getattr(cp, "shift_coef", 0.0))
    p.shift_fs = float(getattr(cp, "shift_fs", 0.0))
    for k in range(3):
        p.ncell[k] = int(cp.ncell[k])
        p.origin[k] = float(cp.origin[k])
        p.gravity[k] = float(cp.gravity[k])
    for name in ("cell_size", "inv_cell_size", "h", "rho0", "gamma", "c0", "alpha", "delta",
                 "eta2", "cfl", "mass_fluid", "mass_bound", "motion_amp", "motion_omega",
                 "dt_floor"):
        setattr(p, name, float(getattr(cp, name)))
    return p


@dataclass
class DeviceState:
    """SoA particle state in device memory (torch tensors)."""
    pos: torch.Tensor            # (dim, n) float64
    vel: torch.Tensor            # (dim, n) float32
    rho: torch.Tensor            # (n,) float32
    type: Optional[torch.Tensor] = None  # (n,) uint8
    id: Optional[torch.Tensor] = None    # (n,) int32 (bit pattern of uint32)
    normal: Optional[torch.Tensor] = None  # (dim, n) float32 wall ghost vectors
    vel64: Optional[torch.Tensor] = None   # (dim, n) float64: an all-FP64 state
    rho64: Optional[torch.Tensor] = None   # (n,) float64

    @staticmethod
    def empty(dim: int, n: int, device, with_type=True, with_id=True,
              with_normal=False, f64=False) -> "DeviceState":
        return DeviceState(
            pos=torch.empty((dim, n), dtype=torch.float64, device=device),
            vel=torch.empty((dim, n), dtype=torch.float32, device=device),
            rho=torch.empty((n,), dtype=torch.float32, device=device),
            type=torch.empty((n,), dtype=torch.uint8, device=device) if with_type else None,
            id=torch.empty((n,), dtype=torch.int32, device=device) if with_id else None,
            normal=(torch.empty((dim, n), dtype=torch.float32, device=device)
                    if with_normal else None),
            vel64=torch.empty((dim, n), dtype=torch.float64, device=device) if f64 else None,
            rho64=torch.empty((n,), dtype=torch.float64, device=device) if f64 else None)

    @staticmethod
    def from_case(case, device, with_normal=False, f64=False) -> "DeviceState":
        """The case's initial state; with f64, also FP64 copies of its
        velocities and densities (an all-FP64 state)."""
        n = case.n
        normal = None
        if with_normal:
            if case.normal is None:
                raise ValueError("the case has no wall ghost vectors")
            normal = torch.from_numpy(np.ascontiguousarray(case.normal)).to(device)
        return DeviceState(
            pos=torch.from_numpy(case.pos).to(device),
            vel=torch.from_numpy(case.vel).to(device),
            rho=torch.from_numpy(case.rho).to(device),
            type=torch.from_numpy(case.type).to(device),
            id=torch.arange(n, dtype=torch.int32, device=device), normal=normal,
            vel64=(torch.from_numpy(case.vel.astype(np.float64)).to(device) if f64 else None),
            rho64=(torch.from_numpy(case.rho.astype(np.float64)).to(device) if f64 else None))

    def c(self) -> SphState:
        opt = lambda t: None if t is None else t.data_ptr()  # noqa: E731
        return SphState(self.pos.data_ptr(), self.vel.data_ptr(), self.rho.data_ptr(),
                        opt(self.type), opt(self.id), opt(self.normal), opt(self.vel64),
                        opt(self.rho64))

    @property
    def n(self) -> int:
        return int(self.rho.shape[0])


def sph_workspace_bytes(params: SphParams, n: int) -> int:
    return int(lib.sph_workspace_bytes(C.byref(params), int(n)))


def sph_bin_cells(params: SphParams, n: int, src: DeviceState, dst: DeviceState,
                  key: torch.Tensor, perm: torch.Tensor, cell_start: torch.Tensor,
                  ws: torch.Tensor, carry_in: Optional[DeviceState] = None,
                  carry_out: Optional[DeviceState] = None, stream=None):
    ci = C.byref(carry_in.c()) if carry_in is not None else None
    co = C.byref(carry_out.c()) if carry_out is not None else None
    _check(lib.sph_bin_cells(C.byref(params), int(n), C.byref(src.c()), C.byref(dst.c()), ci, co,
                             _ptr(key), _ptr(perm), _ptr(cell_start), _ptr(ws), ws.numel(),
                             _stream(stream)), "sph_bin_cells")


def sph_interact(params: SphParams, n: int, s: DeviceState, key: torch.Tensor,
                 cell_start: torch.Tensor, ace: torch.Tensor, arho: torch.Tensor,
                 ws: torch.Tensor, visc: Optional[torch.Tensor] = None,
                 nbr: Optional[torch.Tensor] = None, flags: int = 0, stream=None):
    _check(lib.sph_interact(C.byref(params), int(n), C.byref(s.c()), _ptr(key), _ptr(cell_start),
                            _ptr(ace), _ptr(arho), _ptr(visc), _ptr(nbr), int(flags), _ptr(ws),
                            ws.numel(), _stream(stream)), "sph_interact")


def sph_interact_noalloc(params: SphParams, n: int, s: DeviceState, key: torch.Tensor,
                         cell_start: torch.Tensor, ace: torch.Tensor, arho: torch.Tensor,
                         visc: Optional[torch.Tensor] = None, nbr: Optional[torch.Tensor] = None,
                         flags: int = 0, stream=None):
    _check(lib.sph_interact_noalloc(C.byref(params), int(n), C.byref(s.c()), _ptr(key),
                                    _ptr(cell_start), _ptr(ace), _ptr(arho), _ptr(visc), _ptr(nbr),
                                    int(flags), _stream(stream)), "sph_interact_noalloc")


def sph_list_bytes(params: SphParams, n: int) -> int:
    return int(lib.sph_list_bytes(C.byref(params), int(n)))


def sph_build_list(params: SphParams, n: int, s: DeviceState, key: torch.Tensor,
                   cell_start: torch.Tensor, skin: float, lst: torch.Tensor, ws: torch.Tensor,
                   flags: int = 0, stream=None):
    _check(lib.sph_build_list(C.byref(params), int(n), C.byref(s.c()), _ptr(key),
                              _ptr(cell_start), float(skin), int(flags), _ptr(lst), lst.numel(),
                              _ptr(ws), ws.numel(), _stream(stream)), "sph_build_list")


def sph_interact_list(params: SphParams, n: int, s: DeviceState, key: torch.Tensor,
                      cell_start: torch.Tensor, lst: torch.Tensor, ace: torch.Tensor,
                      arho: torch.Tensor, ws: torch.Tensor, visc: Optional[torch.Tensor] = None,
                      nbr: Optional[torch.Tensor] = None, flags: int = 0, stream=None):
    _check(lib.sph_interact_list(C.byref(params), int(n), C.byref(s.c()), _ptr(key),
                                 _ptr(cell_start), _ptr(lst), lst.numel(), _ptr(ace), _ptr(arho),
                                 _ptr(visc), _ptr(nbr), int(flags), _ptr(ws), ws.numel(),
                                 _stream(stream)), "sph_interact_list")


def sph_list_walks(ws: torch.Tensor) -> int:
    v = int(lib.sph_list_walks(_ptr(ws)))
    if v < 0:
        _check(v, "sph_list_walks")
    return v


def sph_refresh_view(params: SphParams, n: int, s: DeviceState, key: torch.Tensor,
                     ws: torch.Tensor, stream=None):
    _check(lib.sph_refresh_view(C.byref(params), int(n), C.byref(s.c()), _ptr(key), _ptr(ws),
                                ws.numel(), _stream(stream)), "sph_refresh_view")


def sph_reduce_dt(params: SphParams, n: int, dt: torch.Tensor, ws: torch.Tensor,
                  interactions: Optional[torch.Tensor] = None,
                  maxima: Optional[torch.Tensor] = None, stream=None):
    _check(lib.sph_reduce_dt(C.byref(params), int(n), _ptr(dt), _ptr(interactions), _ptr(maxima),
                             _ptr(ws), ws.numel(), _stream(stream)), "sph_reduce_dt")


def sph_symplectic_step(params: SphParams, n: int, phase: int, dt: torch.Tensor,
                        t: torch.Tensor, saved: DeviceState, s: DeviceState, ace: torch.Tensor,
                        arho: torch.Tensor, ws: torch.Tensor, stream=None):
    _check(lib.sph_symplectic_step(C.byref(params), int(n), int(phase), _ptr(dt), _ptr(t),
                                   C.byref(saved.c()), C.byref(s.c()), _ptr(ace), _ptr(arho),
                                   _ptr(ws), ws.numel(), _stream(stream)), "sph_symplectic_step")


def sph_verlet_step(params: SphParams, n: int, mode: int, dt: torch.Tensor, t: torch.Tensor,
                    prev: DeviceState, s: DeviceState, ace: torch.Tensor, arho: torch.Tensor,
                    ws: torch.Tensor, stream=None):
    _check(lib.sph_verlet_step(C.byref(params), int(n), int(mode), _ptr(dt), _ptr(t),
                               C.byref(prev.c()), C.byref(s.c()), _ptr(ace), _ptr(arho),
                               _ptr(ws), ws.numel(), _stream(stream)), "sph_verlet_step")


def sph_mdbc(params: SphParams, n: int, s: DeviceState, key: torch.Tensor,
             cell_start: torch.Tensor, ws: torch.Tensor, stream=None):
    _check(lib.sph_mdbc(C.byref(params), int(n), C.byref(s.c()), _ptr(key), _ptr(cell_start),
                        _ptr(ws), ws.numel(), _stream(stream)), "sph_mdbc")


def bodies_to_device(bodies, device) -> torch.Tensor:
    """The sph_body table of `bodies` (dicts with id_first, count, mass,
    center, vel, omega) as a uint8 device tensor."""
    arr = (SphBody * len(bodies))()
    for k, b in enumerate(bodies):
        arr[k].id_first, arr[k].count, arr[k].mass = int(b["id_first"]), int(b["count"]), \
            float(b["mass"])
        for d in range(3):
            arr[k].center[d] = float(b["center"][d])
            arr[k].vel[d] = float(b.get("vel", (0.0,) * 3)[d])
            arr[k].omega[d] = float(b.get("omega", (0.0,) * 3)[d])
    raw = np.frombuffer(bytes(arr), dtype=np.uint8).copy()
    return torch.from_numpy(raw).to(device)


def bodies_from_device(table: torch.Tensor) -> list:
    """The body table read back as dicts (numpy arrays of 3 components)."""
    raw = table.cpu().numpy().tobytes()
    nb = len(raw) // C.sizeof(SphBody)
    arr = (SphBody * nb).from_buffer_copy(raw)
    out = []
    for b in arr:
        d = dict(id_first=int(b.id_first), count=int(b.count), mass=float(b.mass))
        for name in ("center", "vel", "omega", "center_n", "vel_n", "omega_n", "force",
                     "torque"):
            d[name] = np.array(getattr(b, name)[:])
        out.append(d)
    return out


def sph_floating_step(params: SphParams, n: int, phase: int, dt: torch.Tensor,
                      bodies: torch.Tensor, saved: DeviceState, s: DeviceState,
                      ace: torch.Tensor, ws: torch.Tensor, stream=None):
    nb = bodies.numel() // C.sizeof(SphBody)
    _check(lib.sph_floating_step(C.byref(params), int(n), int(phase), _ptr(dt), _ptr(bodies),
                                 int(nb), C.byref(saved.c()), C.byref(s.c()), _ptr(ace),
                                 _ptr(ws), ws.numel(), _stream(stream)), "sph_floating_step")


def sph_shifting(params: SphParams, n: int, s: DeviceState, key: torch.Tensor,
                 cell_start: torch.Tensor, dt: torch.Tensor, ws: torch.Tensor,
                 conc: Optional[torch.Tensor] = None, shift: Optional[torch.Tensor] = None,
                 flags: int = 0, stream=None):
    _check(lib.sph_shifting(C.byref(params), int(n), C.byref(s.c()), _ptr(key), _ptr(cell_start),
                            _ptr(dt), _ptr(conc), _ptr(shift), int(flags), _ptr(ws), ws.numel(),
                            _stream(stream)), "sph_shifting")


def sph_read_error(ws: torch.Tensor) -> int:
    v = int(lib.sph_read_error(_ptr(ws)))
    if v < 0:
        _check(v, "sph_read_error")
    return v


def sph_clear_error(ws: torch.Tensor, stream=None):
    _check(lib.sph_clear_error(_ptr(ws), _stream(stream)), "sph_clear_error")


# ------------------------------------------------------------------ batches
def sph_batch_describe(params_list, offsets, four_lanes: bool = False):
    """Host-side slot table of a batch (four_lanes: SPH_BATCH_FOUR_LANES).
    Returns (SphBatch without table, table bytes as a uint8 numpy array)."""
    import numpy as np
    ns = len(params_list)
    arr = (SphParams * ns)(*params_list)
    offs = (C.c_int64 * (ns + 1))(*[int(o) for o in offsets])
    nbytes = int(lib.sph_batch_table_bytes(ns))
    if nbytes == 0:
        raise SphError(f"sph_batch_table_bytes: bad slot count {ns}")
    host = np.zeros(nbytes, np.uint8)
    b = SphBatch()
    opts = SPH_BATCH_FOUR_LANES if four_lanes else 0
    _check(lib.sph_batch_describe(arr, offs, ns, opts, host.ctypes.data_as(C.c_void_p), nbytes,
                                  C.byref(b)), "sph_batch_describe")
    return b, host


def sph_batch_workspace_bytes(batch: SphBatch) -> int:
    return int(lib.sph_batch_workspace_bytes(C.byref(batch)))


def sph_batch_bin_cells(batch: SphBatch, src: DeviceState, dst: DeviceState, key, perm,
                        cell_start, ws, carry_in=None, carry_out=None, stream=None):
    ci = C.byref(carry_in.c()) if carry_in is not None else None
    co = C.byref(carry_out.c()) if carry_out is not None else None
    _check(lib.sph_batch_bin_cells(C.byref(batch), C.byref(src.c()), C.byref(dst.c()), ci, co,
                                   _ptr(key), _ptr(perm), _ptr(cell_start), _ptr(ws), ws.numel(),
                                   _stream(stream)), "sph_batch_bin_cells")


def sph_batch_interact(batch: SphBatch, s: DeviceState, key, cell_start, ace, arho, ws,
                       visc=None, nbr=None, flags: int = 0, stream=None):
    _check(lib.sph_batch_interact(C.byref(batch), C.byref(s.c()), _ptr(key), _ptr(cell_start),
                                  _ptr(ace), _ptr(arho), _ptr(visc), _ptr(nbr), int(flags),
                                  _ptr(ws), ws.numel(), _stream(stream)), "sph_batch_interact")


def sph_batch_refresh_view(batch: SphBatch, s: DeviceState, key, ws, stream=None):
    _check(lib.sph_batch_refresh_view(C.byref(batch), C.byref(s.c()), _ptr(key), _ptr(ws),
                                      ws.numel(), _stream(stream)), "sph_batch_refresh_view")


def sph_batch_reduce_dt(batch: SphBatch, dt, ws, interactions=None, stream=None):
    _check(lib.sph_batch_reduce_dt(C.byref(batch), _ptr(dt), _ptr(interactions), _ptr(ws),
                                   ws.numel(), _stream(stream)), "sph_batch_reduce_dt")


def sph_batch_symplectic_step(batch: SphBatch, phase, dt, t, saved: DeviceState, s: DeviceState,
                              ace, arho, ws, stream=None):
    _check(lib.sph_batch_symplectic_step(C.byref(batch), int(phase), _ptr(dt), _ptr(t),
                                         C.byref(saved.c()), C.byref(s.c()), _ptr(ace),
                                         _ptr(arho), _ptr(ws), ws.numel(), _stream(stream)),
           "sph_batch_symplectic_step")


def sph_batch_shifting(batch: SphBatch, s: DeviceState, key, cell_start, dt, ws,
                       conc: Optional[torch.Tensor] = None, shift: Optional[torch.Tensor] = None,
                       flags: int = 0, stream=None):
    _check(lib.sph_batch_shifting(C.byref(batch), C.byref(s.c()), _ptr(key), _ptr(cell_start),
                                  _ptr(dt), _ptr(conc), _ptr(shift), int(flags), _ptr(ws),
                                  ws.numel(), _stream(stream)), "sph_batch_shifting")


def sph_batch_read_errors(batch: SphBatch, ws):
    import numpy as np
    out = np.zeros(batch.n_slots, np.uint32)
    _check(lib.sph_batch_read_errors(C.byref(batch), _ptr(ws), out.ctypes.data_as(C.c_void_p)),
           "sph_batch_read_errors")
    return out


def sph_batch_clear_errors(batch: SphBatch, ws, stream=None):
    _check(lib.sph_batch_clear_errors(C.byref(batch), _ptr(ws), _stream(stream)),
           "sph_batch_clear_errors")
