"""CPU FP64 oracle of the WCSPH particle-interaction step (test infrastructure).

A plain, slow, brute-force implementation (``sph_oracle.c``) of Section 2 and
Section 5.1 of the DualSPHysics v5.0 paper, wrapped with ctypes for numpy
arrays.  Only the tests, the smoke check and the CPU-baseline leg of the
benchmark use it; the product path never imports it.

Every function is pinned by tests in ``tests/test_oracle_*.py`` against what
the paper and the mathematics fix (closed forms, invariants, brute-force
lattice counts, exact special cases).  Long multi-step trajectories are
"parity unpinned" beyond those pins: the paper's experimental comparisons
need datasets that are not available.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "sph_oracle.c")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, no contraction, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", "-D_GNU_SOURCE",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class OrcParams(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("ddt", C.c_int32), ("ncell", C.c_int32 * 3),
        ("x_sub", C.c_int32), ("origin", C.c_double * 3),
        ("inv_cell_size", C.c_double), ("h", C.c_double), ("rho0", C.c_double),
        ("gamma", C.c_double), ("c0", C.c_double), ("alpha", C.c_double),
        ("delta", C.c_double), ("eta2", C.c_double), ("cfl", C.c_double),
        ("mass_fluid", C.c_double), ("mass_bound", C.c_double),
        ("gravity", C.c_double * 3), ("motion_amp", C.c_double),
        ("motion_omega", C.c_double), ("kernel", C.c_int32), ("viscosity", C.c_int32),
        ("visc_nu", C.c_double), ("boundary", C.c_int32), ("pad2", C.c_int32),
        ("period", C.c_double * 3), ("shift_coef", C.c_double), ("shift_fs", C.c_double),
    ]


class OrcBody(C.Structure):
    _fields_ = [
        ("first", C.c_int64), ("count", C.c_int64), ("mass", C.c_double),
        ("center", C.c_double * 3), ("vel", C.c_double * 3), ("omega", C.c_double * 3),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB_PATH)
        P = C.POINTER
        L.orc_wendland_w.restype = C.c_double
        L.orc_wendland_w.argtypes = [C.c_double, C.c_double, C.c_int32]
        L.orc_wendland_fab.restype = C.c_double
        L.orc_wendland_fab.argtypes = [C.c_double, C.c_double, C.c_int32]
        for name in ("orc_cubic_w", "orc_cubic_fab"):
            getattr(L, name).restype = C.c_double
            getattr(L, name).argtypes = [C.c_double, C.c_double, C.c_int32]
        L.orc_pressure.restype = C.c_double
        L.orc_pressure.argtypes = [P(OrcParams), C.c_double]
        L.orc_cell_keys.argtypes = [P(OrcParams), C.c_int64, C.c_void_p, C.c_void_p]
        L.orc_wrap.argtypes = [P(OrcParams), C.c_int64, C.c_void_p, C.c_void_p]
        L.orc_sort_perm.argtypes = [C.c_int64, C.c_void_p, C.c_void_p]
        L.orc_cell_start.argtypes = [C.c_int64, C.c_void_p, C.c_int64, C.c_void_p]
        L.orc_interact.argtypes = [P(OrcParams), C.c_int64, C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                   C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_time_step.restype = C.c_double
        L.orc_time_step.argtypes = [P(OrcParams), C.c_int64, C.c_void_p, C.c_void_p,
                                    C.c_void_p]
        for name in ("orc_predictor", "orc_corrector"):
            getattr(L, name).argtypes = [P(OrcParams), C.c_int64, C.c_double,
                                         C.c_double] + [C.c_void_p] * 9
        L.orc_verlet.argtypes = [P(OrcParams), C.c_int64, C.c_double, C.c_double,
                                 C.c_int32] + [C.c_void_p] * 8
        L.orc_run_verlet.restype = C.c_int32
        L.orc_run_verlet.argtypes = [P(OrcParams), C.c_int64, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                                     P(C.c_double), C.c_void_p, P(C.c_uint64)]
        L.orc_run.restype = C.c_int32
        L.orc_run.argtypes = [P(OrcParams), C.c_int64, C.c_void_p, C.c_void_p,
                              C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, P(C.c_double),
                              C.c_void_p, P(C.c_uint64), C.c_void_p, C.c_int32]
        L.orc_body_forces.argtypes = [P(OrcParams), C.c_int64, C.c_void_p, C.c_void_p,
                                      P(OrcBody), C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_body_step.restype = C.c_int32
        L.orc_body_step.argtypes = [P(OrcParams), C.c_int64, C.c_int32, C.c_double,
                                    P(OrcBody), P(OrcBody)] + [C.c_void_p] * 7
        L.orc_mdbc.argtypes = [P(OrcParams), C.c_int64] + [C.c_void_p] * 7
        L.orc_shift.argtypes = [P(OrcParams), C.c_int64] + [C.c_void_p] * 4 + \
            [C.c_double] + [C.c_void_p] * 3
        _lib = L
    return _lib


def params(cp) -> OrcParams:
    """OrcParams from a ``cases.CaseParams`` (or any object with its fields)."""
    p = OrcParams()
    p.dim = int(cp.dim)
    p.ddt = int(cp.ddt)
    for k in range(3):
        p.ncell[k] = int(cp.ncell[k])
        p.origin[k] = float(cp.origin[k])
        p.gravity[k] = float(cp.gravity[k])
    p.inv_cell_size = float(cp.inv_cell_size)
    p.x_sub = int(getattr(cp, "x_sub", 1))
    p.kernel = int(getattr(cp, "kernel", 0))
    p.viscosity = int(getattr(cp, "viscosity", 0))
    p.visc_nu = float(getattr(cp, "visc_nu", 0.0))
    p.boundary = int(getattr(cp, "boundary", 0))
    period = getattr(cp, "period", (0.0, 0.0, 0.0))
    for k in range(3):
        p.period[k] = float(period[k])
    p.shift_coef = float(getattr(cp, "shift_coef", 0.0))
    p.shift_fs = float(getattr(cp, "shift_fs", 0.0))
    for name in ("h", "rho0", "gamma", "c0", "alpha", "delta", "eta2", "cfl",
                 "mass_fluid", "mass_bound", "motion_amp", "motion_omega"):
        setattr(p, name, float(getattr(cp, name)))
    return p


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def wendland_w(r, h, dim):
    return float(lib().orc_wendland_w(float(r), float(h), int(dim)))


def wendland_fab(r, h, dim):
    return float(lib().orc_wendland_fab(float(r), float(h), int(dim)))


def cubic_w(r, h, dim):
    return float(lib().orc_cubic_w(float(r), float(h), int(dim)))


def cubic_fab(r, h, dim):
    return float(lib().orc_cubic_fab(float(r), float(h), int(dim)))


def pressure(cp, rho):
    p = params(cp)
    return float(lib().orc_pressure(C.byref(p), float(rho)))


def cell_keys(cp, pos):
    pos = _f64(pos)
    n = pos.shape[1]
    key = np.zeros(n, np.uint32)
    p = params(cp)
    lib().orc_cell_keys(C.byref(p), n, _ptr(pos), _ptr(key))
    return key


def wrap(cp, pos, ptype=None):
    """Positions brought back into [origin, origin + period) along periodic
    components (Section 2.7)."""
    pos = _f64(pos).copy()
    p = params(cp)
    tp = None if ptype is None else np.ascontiguousarray(ptype, dtype=np.uint8)
    lib().orc_wrap(C.byref(p), pos.shape[1], _ptr(pos), None if tp is None else _ptr(tp))
    return pos


def sort_perm(key):
    key = np.ascontiguousarray(key, dtype=np.uint32)
    perm = np.zeros(key.shape[0], np.uint32)
    lib().orc_sort_perm(key.shape[0], _ptr(key), _ptr(perm))
    return perm


def cell_start(sorted_key, ncell_total):
    sk = np.ascontiguousarray(sorted_key, dtype=np.uint32)
    start = np.zeros(int(ncell_total) + 1, np.uint32)
    lib().orc_cell_start(sk.shape[0], _ptr(sk), int(ncell_total), _ptr(start))
    return start


def interact(cp, pos, vel, rho, ptype, targets=None):
    """Brute-force PI for ``targets`` (indices; None = all).  Returns
    (ace [dim, nt], arho [nt], visc [nt], nbr [nt])."""
    pos, vel, rho = _f64(pos), _f64(vel), _f64(rho)
    ptype = np.ascontiguousarray(ptype, dtype=np.uint8)
    n = rho.shape[0]
    dim = int(cp.dim)
    if targets is None:
        nt, tptr, tarr = n, None, None
    else:
        tarr = np.ascontiguousarray(targets, dtype=np.int64)
        nt, tptr = tarr.shape[0], _ptr(tarr)
    ace = np.zeros((dim, nt), np.float64)
    arho = np.zeros(nt, np.float64)
    visc = np.zeros(nt, np.float64)
    nbr = np.zeros(nt, np.uint32)
    p = params(cp)
    lib().orc_interact(C.byref(p), n, _ptr(pos), _ptr(vel), _ptr(rho), _ptr(ptype),
                       nt, tptr, _ptr(ace), _ptr(arho), _ptr(visc), _ptr(nbr))
    return ace, arho, visc, nbr


def time_step(cp, ptype, ace, visc):
    ptype = np.ascontiguousarray(ptype, dtype=np.uint8)
    ace, visc = _f64(ace), _f64(visc)
    p = params(cp)
    return float(lib().orc_time_step(C.byref(p), ptype.shape[0], _ptr(ptype),
                                     _ptr(ace), _ptr(visc)))


def predictor(cp, dt, t, pos, vel, rho, ptype, ace, arho):
    """Returns (pos, vel, rho) at n+1/2 and the saved (pos_n, vel_n, rho_n)."""
    pos, vel, rho = _f64(pos).copy(), _f64(vel).copy(), _f64(rho).copy()
    ptype = np.ascontiguousarray(ptype, dtype=np.uint8)
    ace, arho = _f64(ace), _f64(arho)
    pn, vn, rn = np.zeros_like(pos), np.zeros_like(vel), np.zeros_like(rho)
    p = params(cp)
    lib().orc_predictor(C.byref(p), rho.shape[0], float(dt), float(t), _ptr(pos),
                        _ptr(vel), _ptr(rho), _ptr(ptype), _ptr(ace), _ptr(arho),
                        _ptr(pn), _ptr(vn), _ptr(rn))
    return (pos, vel, rho), (pn, vn, rn)


def corrector(cp, dt, t, half, saved, ptype, ace, arho):
    pos, vel, rho = (_f64(a).copy() for a in half)
    pn, vn, rn = (_f64(a) for a in saved)
    ptype = np.ascontiguousarray(ptype, dtype=np.uint8)
    ace, arho = _f64(ace), _f64(arho)
    p = params(cp)
    lib().orc_corrector(C.byref(p), rho.shape[0], float(dt), float(t), _ptr(pos),
                        _ptr(vel), _ptr(rho), _ptr(ptype), _ptr(ace), _ptr(arho),
                        _ptr(pn), _ptr(vn), _ptr(rn))
    return pos, vel, rho


def _normal_arg(cp, normal, n):
    if int(getattr(cp, "boundary", 0)) == 1:
        if normal is None:
            raise ValueError("modified DBC needs the wall particles' ghost vectors")
        return _f64(normal).reshape(int(cp.dim), n)
    return None


def body(first, count, mass, center, vel=(0.0, 0.0, 0.0), omega=(0.0, 0.0, 0.0)) -> OrcBody:
    """A floating body over particles [first, first + count) (Section 3.2)."""
    b = OrcBody()
    b.first, b.count, b.mass = int(first), int(count), float(mass)
    for k in range(3):
        b.center[k] = float(center[k]) if k < len(center) else 0.0
        b.vel[k] = float(vel[k]) if k < len(vel) else 0.0
        b.omega[k] = float(omega[k]) if k < len(omega) else 0.0
    return b


def body_dict(b: OrcBody) -> dict:
    return dict(first=int(b.first), count=int(b.count), mass=float(b.mass),
                center=np.array(b.center[:]), vel=np.array(b.vel[:]),
                omega=np.array(b.omega[:]))


def _bodies_arg(bodies):
    if not bodies:
        return None, 0
    arr = (OrcBody * len(bodies))()
    for k, b in enumerate(bodies):
        arr[k] = b if isinstance(b, OrcBody) else body(**b)
    return arr, len(bodies)


def body_forces(cp, pos, ace, b):
    """(force [3], torque [3], inertia [3, 3]) of body b (Eq. 48-49): the
    fluid force sum_k m_B dv_k/dt, its torque about the centre and the
    inertia tensor about the centre (2-D: torque[0], inertia[0, 0])."""
    pos, ace = _f64(pos), _f64(ace)
    f, tq, inertia = np.zeros(3), np.zeros(3), np.zeros(9)
    bb = b if isinstance(b, OrcBody) else body(**b)
    p = params(cp)
    lib().orc_body_forces(C.byref(p), pos.shape[1], _ptr(pos), _ptr(ace), C.byref(bb),
                          _ptr(f), _ptr(tq), _ptr(inertia))
    return f, tq, inertia.reshape(3, 3)


def body_step(cp, phase, dt, b, b_n, pos_n, pos, vel, ptype, ace):
    """One phase of a floating body's symplectic update (orc_body_step).
    b, b_n: OrcBody (updated in place; phase 0 writes b_n).  Returns
    (pos, vel, force, torque, status) with the body's particles moved."""
    pos_n = _f64(pos_n)
    pos, vel = _f64(pos).copy(), _f64(vel).copy()
    ptype = np.ascontiguousarray(ptype, dtype=np.uint8)
    ace = _f64(ace)
    f, tq = np.zeros(3), np.zeros(3)
    p = params(cp)
    st = lib().orc_body_step(C.byref(p), pos.shape[1], int(phase), float(dt), C.byref(b),
                             C.byref(b_n), _ptr(pos_n), _ptr(pos), _ptr(vel), _ptr(ptype),
                             _ptr(ace), _ptr(f), _ptr(tq))
    return pos, vel, f, tq, int(st)


def run(cp, pos, vel, rho, ptype, nsteps, t0=0.0, normal=None, bodies=None):
    """nsteps full symplectic steps.  Returns dict with pos, vel, rho, type,
    t, dt history, interaction count, status and the bodies' final states.
    normal: ghost vectors of the wall particles (needed with modified DBC);
    bodies: floating bodies (OrcBody or body() keyword dicts)."""
    pos, vel, rho = _f64(pos).copy(), _f64(vel).copy(), _f64(rho).copy()
    ptype = np.ascontiguousarray(ptype, dtype=np.uint8).copy()
    t = C.c_double(float(t0))
    dts = np.zeros(max(int(nsteps), 1), np.float64)
    inter = C.c_uint64(0)
    p = params(cp)
    nrm = _normal_arg(cp, normal, rho.shape[0])
    barr, nb = _bodies_arg(bodies)
    st = lib().orc_run(C.byref(p), rho.shape[0], _ptr(pos), _ptr(vel), _ptr(rho),
                       _ptr(ptype), _ptr(nrm) if nrm is not None else None, int(nsteps),
                       C.byref(t), _ptr(dts), C.byref(inter),
                       C.cast(barr, C.c_void_p) if nb else None, nb)
    return dict(pos=pos, vel=vel, rho=rho, type=ptype, t=t.value,
                dt=dts[: int(nsteps)], interactions=int(inter.value), status=int(st),
                bodies=[body_dict(barr[k]) for k in range(nb)])


def verlet(cp, dt, t, mode, pos, vel, rho, vel_prev, rho_prev, ptype, ace, arho):
    """One Verlet update (Section 2.5.1; mode 0: Eq. 30, mode 1: Eq. 31).
    Returns (pos, vel, rho) at n+1 and (vel_prev, rho_prev) = state n."""
    pos, vel, rho = _f64(pos).copy(), _f64(vel).copy(), _f64(rho).copy()
    vp, rp = _f64(vel_prev).copy(), _f64(rho_prev).copy()
    ptype = np.ascontiguousarray(ptype, dtype=np.uint8)
    ace, arho = _f64(ace), _f64(arho)
    p = params(cp)
    lib().orc_verlet(C.byref(p), rho.shape[0], float(dt), float(t), int(mode), _ptr(pos),
                     _ptr(vel), _ptr(rho), _ptr(vp), _ptr(rp), _ptr(ptype), _ptr(ace),
                     _ptr(arho))
    return (pos, vel, rho), (vp, rp)


def run_verlet(cp, pos, vel, rho, ptype, nsteps, ns=40, t0=0.0, normal=None):
    """nsteps Verlet steps (Eq. 31 on the first step and every ns-th).
    Returns the same dict as run()."""
    pos, vel, rho = _f64(pos).copy(), _f64(vel).copy(), _f64(rho).copy()
    ptype = np.ascontiguousarray(ptype, dtype=np.uint8).copy()
    t = C.c_double(float(t0))
    dts = np.zeros(max(int(nsteps), 1), np.float64)
    inter = C.c_uint64(0)
    p = params(cp)
    nrm = _normal_arg(cp, normal, rho.shape[0])
    st = lib().orc_run_verlet(C.byref(p), rho.shape[0], _ptr(pos), _ptr(vel), _ptr(rho),
                              _ptr(ptype), _ptr(nrm) if nrm is not None else None, int(nsteps),
                              int(ns), C.byref(t), _ptr(dts), C.byref(inter))
    return dict(pos=pos, vel=vel, rho=rho, type=ptype, t=t.value,
                dt=dts[: int(nsteps)], interactions=int(inter.value), status=int(st))


def shift(cp, pos, vel, rho, ptype, dt):
    """Particle shifting (Section 2.8, Eq. 40-41, 53): returns (C [n],
    grad C [dim, n], dr [dim, n]) for the given state and time step."""
    pos, vel, rho = _f64(pos), _f64(vel), _f64(rho)
    n = rho.shape[0]
    ptype = np.ascontiguousarray(ptype, dtype=np.uint8)
    dim = int(cp.dim)
    conc, grad, dr = np.zeros(n), np.zeros((dim, n)), np.zeros((dim, n))
    p = params(cp)
    lib().orc_shift(C.byref(p), n, _ptr(pos), _ptr(vel), _ptr(rho), _ptr(ptype), float(dt),
                    _ptr(conc), _ptr(grad), _ptr(dr))
    return conc, grad, dr


def mdbc(cp, pos, vel, rho, ptype, normal):
    """Modified DBC (Section 2.6.2, Eq. 38-39): returns (rho, vel) with the
    wall particles' density and velocity from their ghost nodes."""
    pos, vel, rho = _f64(pos), _f64(vel), _f64(rho)
    n = rho.shape[0]
    ptype = np.ascontiguousarray(ptype, dtype=np.uint8)
    normal = _f64(normal).reshape(int(cp.dim), n)
    ro, vo = np.zeros_like(rho), np.zeros_like(vel)
    p = params(cp)
    lib().orc_mdbc(C.byref(p), n, _ptr(pos), _ptr(vel), _ptr(rho), _ptr(ptype), _ptr(normal),
                   _ptr(ro), _ptr(vo))
    return ro, vo

