"""Seeded synthetic SPH cases: dam breaks (2-D, 3-D) and a sloshing tank.

This module only builds inputs.  It holds none of the solver's arithmetic
(no kernel, equation of state, interaction sum or time integrator), so both
the HIP path and the CPU oracle can take their inputs from it.

Geometry conventions
--------------------
* Components are ordered (x, [y,] z) with the vertical axis last; a 2-D case
  stores (x, z).
* Fluid and wall particles sit on one Cartesian lattice of spacing ``dp``
  (cell centres at ``(i + 0.5) dp``), as a case generator does for the
  paper's dynamic boundary condition (Section 2.6.1): two layers of wall
  particles outside every wall.
* Every coordinate gets a seeded uniform jitter of +-1e-4 dp.
* Mass is ``rho0 dp^d`` for every particle; the initial density is the
  hydrostatic one for the fluid column height H, so that the Tait pressure
  of Eq. 28 equals rho0 g (H - z) at t = 0 (walls above the free surface
  start at rho0).  Velocities start at zero.
* The numerical speed of sound is ``c0 = 10 sqrt(g H)`` (Section 2.4).
* The cell grid covers the tank plus a margin (open tanks: head room up to
  2.5 times the initial fluid height for run-up); cell size is ``2h/cell_div``
  (Section 5.1 uses 2h; Section 5.3 reports cells of size h).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict
from typing import Optional, Tuple

import numpy as np

FLUID, BOUND_FIXED, BOUND_MOVING, FLOATING = 0, 1, 2, 3
EXCLUDED = 0x80
GRAVITY = 9.81

__all__ = ["CaseParams", "Case", "dam_break_2d", "dam_break_3d", "sloshing_3d",
           "block_case", "random_serving_case", "floating_box", "periodic_box", "FLUID",
           "BOUND_FIXED",
           "BOUND_MOVING", "FLOATING", "EXCLUDED", "GRAVITY"]


@dataclass
class CaseParams:
    """Scalar constants of one case (plain floats; mirrored by the C ABI)."""
    name: str
    dim: int
    dp: float
    h: float
    rho0: float = 1000.0
    gamma: float = 7.0
    c0: float = 0.0
    alpha: float = 0.01
    delta: float = 0.1
    eta2: float = 0.0
    cfl: float = 0.2
    mass_fluid: float = 0.0
    mass_bound: float = 0.0
    gravity: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    ddt: int = 1          # 0 none, 1 Molteni-Colagrossi (Eq. 18), 2 Fourtakas (Eq. 19-20)
    kernel: int = 0       # 0 Wendland C2 (Eq. 11), 1 cubic spline (Eq. 10)
    boundary: int = 0     # 0 DBC (Eq. 36), 1 modified DBC (Eq. 38-39)
    floating: int = 0     # 1: the case has floating bodies (Section 3.2)
    # periodic length per component (Section 2.7), 0 = open; a periodic
    # component's grid starts at the periodic boundary and spans the period
    period: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    # particle shifting (Section 2.8): A_s of Eq. 41 (0 = off) and the
    # concentration below which only the tangential shift is kept (0 = none)
    shift_coef: float = 0.0
    shift_fs: float = 0.0
    viscosity: int = 0    # 0 artificial (Eq. 21), 1 laminar (Eq. 23)
    visc_nu: float = 1e-6  # kinematic viscosity of the laminar term (water)
    cell_div: int = 1
    x_sub: int = 1
    origin: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    cell_size: float = 0.0
    inv_cell_size: float = 0.0
    ncell: Tuple[int, int, int] = (1, 1, 1)
    motion_amp: float = 0.0
    motion_omega: float = 0.0
    dt_floor: float = 1e-12
    fluid_height: float = 0.0

    def ncell_total(self) -> int:
        return int(self.ncell[0]) * int(self.ncell[1]) * int(self.ncell[2])

    def to_dict(self) -> dict:
        return asdict(self)


@dataclass
class Case:
    params: CaseParams
    pos: np.ndarray   # (dim, n) float64
    vel: np.ndarray   # (dim, n) float32
    rho: np.ndarray   # (n,) float32
    type: np.ndarray  # (n,) uint8
    meta: dict = field(default_factory=dict)
    # (dim, n) float32: for wall particles the vector from the particle to its
    # ghost node (its mirror image across the wall face, Section 2.6.2);
    # zero for fluid particles
    normal: Optional[np.ndarray] = None
    # floating bodies (Section 3.2): dicts with id_first, count (the body owns
    # particles [id_first, id_first + count), of type FLOATING), mass, center,
    # vel, omega (3 components each; 2-D uses omega[0])
    bodies: Optional[list] = None

    @property
    def n(self) -> int:
        return int(self.rho.shape[0])

    @property
    def n_fluid(self) -> int:
        return int(np.count_nonzero(self.type == FLUID))


# ----------------------------------------------------------------------------
# lattice helpers
# ----------------------------------------------------------------------------
def _grid(*ranges):
    """Integer lattice indices for the given half-open per-axis ranges."""
    axes = [np.arange(lo, hi, dtype=np.int64) for lo, hi in ranges]
    mesh = np.meshgrid(*axes, indexing="ij")
    return np.stack([m.reshape(-1) for m in mesh], axis=0)


def _walls(dim, nx_tank, ny_tank, nz_tank, closed_top):
    """Lattice indices of two wall layers around a tank of nx*ny*nz cells.

    The bottom (and the lid of a closed tank) spans the full footprint
    including the wall thickness; side walls span the tank height.
    """
    parts = []
    if dim == 2:
        parts.append(_grid((-2, nx_tank + 2), (-2, 0)))                 # bottom
        if closed_top:
            parts.append(_grid((-2, nx_tank + 2), (nz_tank, nz_tank + 2)))
        parts.append(_grid((-2, 0), (0, nz_tank)))                      # x walls
        parts.append(_grid((nx_tank, nx_tank + 2), (0, nz_tank)))
    else:
        parts.append(_grid((-2, nx_tank + 2), (-2, ny_tank + 2), (-2, 0)))
        if closed_top:
            parts.append(_grid((-2, nx_tank + 2), (-2, ny_tank + 2),
                               (nz_tank, nz_tank + 2)))
        parts.append(_grid((-2, 0), (-2, ny_tank + 2), (0, nz_tank)))
        parts.append(_grid((nx_tank, nx_tank + 2), (-2, ny_tank + 2), (0, nz_tank)))
        parts.append(_grid((0, nx_tank), (-2, 0), (0, nz_tank)))
        parts.append(_grid((0, nx_tank), (ny_tank, ny_tank + 2), (0, nz_tank)))
    return np.concatenate(parts, axis=1)


def _ghost_vectors(idx, tank, dp):
    """Per wall particle (lattice indices idx, tank interior [0, tank[k]) in
    cells of dp per axis), the vector to its mirror image across the wall
    faces it lies outside of: 2 (face - centre) along each such axis."""
    out = np.zeros(idx.shape, np.float64)
    for k, nk in enumerate(tank):
        c = idx[k].astype(np.float64) + 0.5
        out[k] = np.where(idx[k] < 0, -2.0 * c, np.where(idx[k] >= nk, 2.0 * (nk - c), 0.0))
    return (out * dp).astype(np.float32)


def _finish(name, dim, dp, fluid_idx, wall_idx, fluid_height, lo, hi, seed,
            cell_div=1, x_sub=1, wall_type=BOUND_FIXED, motion_amp=0.0,
            motion_omega=0.0, h_factor=1.0, meta=None, tank=None) -> Case:
    rng = np.random.default_rng(seed)
    idx = np.concatenate([fluid_idx, wall_idx], axis=1)
    n = idx.shape[1]
    pos = (idx.astype(np.float64) + 0.5) * dp
    pos += rng.uniform(-1e-4 * dp, 1e-4 * dp, size=pos.shape)
    ptype = np.empty(n, np.uint8)
    ptype[: fluid_idx.shape[1]] = FLUID
    ptype[fluid_idx.shape[1]:] = wall_type

    h = h_factor * math.sqrt(dim) * dp
    rho0, gamma = 1000.0, 7.0
    c0 = 10.0 * math.sqrt(GRAVITY * fluid_height)
    b_tait = c0 * c0 * rho0 / gamma
    depth = np.maximum(fluid_height - pos[dim - 1], 0.0)
    rho = rho0 * np.power(1.0 + rho0 * GRAVITY * depth / b_tait, 1.0 / gamma)
    mass = rho0 * dp ** dim

    cs = 2.0 * h / cell_div
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    nc = np.ceil((hi - lo) / cs).astype(np.int64)
    nc[0] *= x_sub  # key cells of cs/x_sub along x
    origin = [float(v) for v in lo] + [0.0] * (3 - dim)
    ncell = [int(v) for v in nc] + [1] * (3 - dim)
    grav = [0.0, 0.0, 0.0]
    grav[dim - 1] = -GRAVITY

    params = CaseParams(
        name=name, dim=dim, dp=dp, h=h, rho0=rho0, gamma=gamma, c0=c0,
        alpha=0.01, delta=0.1, eta2=0.001 * h * h, cfl=0.2,
        mass_fluid=mass, mass_bound=mass, gravity=tuple(grav), ddt=1,
        cell_div=cell_div, x_sub=x_sub, origin=tuple(origin), cell_size=cs,
        inv_cell_size=1.0 / cs, ncell=tuple(ncell), motion_amp=motion_amp,
        motion_omega=motion_omega, fluid_height=fluid_height)
    normal = np.zeros((dim, n), np.float32)
    if tank is not None and wall_idx.shape[1]:
        normal[:, fluid_idx.shape[1]:] = _ghost_vectors(wall_idx, tank, dp)
    return Case(params=params, pos=np.ascontiguousarray(pos), normal=normal,
                vel=np.zeros((dim, n), np.float32),
                rho=rho.astype(np.float32), type=ptype, meta=dict(meta or {}))


# ----------------------------------------------------------------------------
# the workloads
# ----------------------------------------------------------------------------
def dam_break_2d(dp=0.01, tank=(1.6, 1.0), column=(0.4, 0.8), seed=0,
                 cell_div=1, x_sub=1) -> Case:
    """2-D dam break: a column at x_min in an open-top tank."""
    nxt, nzt = int(round(tank[0] / dp)), int(round(tank[1] / dp))
    nxf, nzf = int(round(column[0] / dp)), int(round(column[1] / dp))
    fluid = _grid((0, nxf), (0, nzf))
    walls = _walls(2, nxt, 1, nzt, closed_top=False)
    lo = (-2.0 * dp - 1e-3 * dp, -2.0 * dp - 1e-3 * dp)
    hi = (nxt * dp + 2.0 * dp, max(nzt * dp, 2.5 * nzf * dp) + 2.0 * dp)
    return _finish("dam_break_2d", 2, dp, fluid, walls, nzf * dp, lo, hi, seed,
                   cell_div=cell_div, x_sub=x_sub, meta=dict(tank=tank, column=column),
                   tank=(nxt, nzt))


def dam_break_3d(dp=0.6 / 126, tank=(1.6, 0.6, 0.6), block=(0.6, 0.6, 0.3),
                 seed=0, cell_div=1, x_sub=1) -> Case:
    """3-D dam break: a water block at x_min filling the tank width."""
    nxt, nyt, nzt = (int(round(v / dp)) for v in tank)
    nxf, nyf, nzf = (int(round(v / dp)) for v in block)
    fluid = _grid((0, nxf), (0, nyf), (0, nzf))
    walls = _walls(3, nxt, nyt, nzt, closed_top=False)
    m = 2.0 * dp + 1e-3 * dp
    lo = (-m, -m, -m)
    hi = (nxt * dp + m, nyt * dp + m, max(nzt * dp, 2.5 * nzf * dp) + m)
    return _finish("dam_break_3d", 3, dp, fluid, walls, nzf * dp, lo, hi, seed,
                   cell_div=cell_div, x_sub=x_sub, meta=dict(tank=tank, block=block),
                   tank=(nxt, nyt, nzt))


def sloshing_3d(dp=0.0025, tank=(2.0, 1.0, 1.0), fill=0.5, seed=0,
                cell_div=1, accel=0.05 * GRAVITY, freq_hz=0.5, x_sub=1) -> Case:
    """Closed tank, half full, whose walls follow the imposed sinusoidal
    motion x_B(t) = x_B0 + (A/w^2)(1 - cos wt) (peak acceleration A)."""
    nxt, nyt, nzt = (int(round(v / dp)) for v in tank)
    nzf = int(round(fill * tank[2] / dp))
    fluid = _grid((0, nxt), (0, nyt), (0, nzf))
    walls = _walls(3, nxt, nyt, nzt, closed_top=True)
    omega = 2.0 * math.pi * freq_hz
    travel = 2.0 * accel / omega ** 2
    m = 2.0 * dp + 1e-3 * dp
    lo = (-m, -m, -m)
    hi = (nxt * dp + m + travel, nyt * dp + m, nzt * dp + m)
    return _finish("sloshing_3d", 3, dp, fluid, walls, nzf * dp, lo, hi, seed,
                   cell_div=cell_div, x_sub=x_sub, wall_type=BOUND_MOVING,
                   motion_amp=accel, motion_omega=omega,
                   meta=dict(tank=tank, fill=fill), tank=(nxt, nyt, nzt))


def block_case(dim, shape, dp=0.01, seed=0, walls=False, cell_div=1,
               vel_scale=0.0, rho_jitter=0.0, margin_cells=2, x_sub=1) -> Case:
    """A fluid block of ``shape`` lattice cells (optionally in a closed box
    of walls), with optional random velocities and densities.  Used for
    invariance and parity tests."""
    fluid = _grid(*[(0, s) for s in shape])
    if walls:
        if dim == 3:
            wall = _walls(3, shape[0], shape[1], shape[2], closed_top=True)
        else:
            wall = _walls(2, shape[0], 1, shape[1], closed_top=True)
    else:
        wall = np.zeros((dim, 0), np.int64)
    height = shape[-1] * dp
    h = math.sqrt(dim) * dp
    cs = 2.0 * h / cell_div
    m = 2.0 * dp + margin_cells * cs
    lo = tuple(-m for _ in range(dim))
    hi = tuple(s * dp + m for s in shape)
    case = _finish(f"block{dim}d", dim, dp, fluid, wall, height, lo, hi, seed,
                   cell_div=cell_div, x_sub=x_sub, meta=dict(shape=shape, walls=walls),
                   tank=tuple(shape))
    rng = np.random.default_rng(seed + 7919)
    if vel_scale:
        case.vel[:] = rng.uniform(-vel_scale, vel_scale, case.vel.shape).astype(np.float32)
    if rho_jitter:
        case.rho[:] = (case.rho * (1.0 + rng.uniform(-rho_jitter, rho_jitter,
                                                     case.rho.shape))).astype(np.float32)
    return case


def random_serving_case(rng: np.random.Generator, n_min=2000, n_max=500_000,
                        seed=None, cell_div=2, x_sub=4) -> Case:
    """One request of the serving stream: a 2-D or 3-D dam break or sloshing
    case with a log-uniform fluid particle count, column aspect ratio
    uniform in [0.5, 2] and fill ratio uniform in [0.3, 0.7]."""
    dim = int(rng.integers(2, 4))
    kind = "dam_break" if rng.random() < 0.5 else "sloshing"
    n_target = math.exp(rng.uniform(math.log(n_min), math.log(n_max)))
    aspect = rng.uniform(0.5, 2.0)
    fill = rng.uniform(0.3, 0.7)
    steps = int(rng.integers(1000, 5001))
    sub_seed = int(rng.integers(0, 2**31 - 1)) if seed is None else seed
    if kind == "dam_break":
        length = 1.6
        width = fill * length / 2.0
        height = aspect * width
        tank_h = max(1.0, 1.25 * height)
        if dim == 2:
            dp = math.sqrt(width * height / n_target)
            case = dam_break_2d(dp=dp, tank=(length, tank_h), column=(width, height),
                                seed=sub_seed, cell_div=cell_div, x_sub=x_sub)
        else:
            depth_y = 0.6
            dp = (width * depth_y * height / n_target) ** (1.0 / 3.0)
            case = dam_break_3d(dp=dp, tank=(length, depth_y, tank_h),
                                block=(width, depth_y, height), seed=sub_seed,
                                cell_div=cell_div, x_sub=x_sub)
    else:
        if dim == 2:
            dp = math.sqrt(2.0 * fill * 1.0 / n_target)
            case = _sloshing_2d(dp, fill, sub_seed, cell_div=cell_div, x_sub=x_sub)
        else:
            dp = (2.0 * 1.0 * fill * 1.0 / n_target) ** (1.0 / 3.0)
            case = sloshing_3d(dp=dp, fill=fill, seed=sub_seed, cell_div=cell_div, x_sub=x_sub)
    case.meta.update(kind=kind, steps=steps, aspect=aspect, fill=fill,
                     n_target=n_target)
    return case


def _sloshing_2d(dp, fill, seed, tank=(2.0, 1.0), accel=0.05 * GRAVITY,
                 freq_hz=0.5, cell_div=1, x_sub=1) -> Case:
    nxt, nzt = int(round(tank[0] / dp)), int(round(tank[1] / dp))
    nzf = max(1, int(round(fill * tank[1] / dp)))
    fluid = _grid((0, nxt), (0, nzf))
    walls = _walls(2, nxt, 1, nzt, closed_top=True)
    omega = 2.0 * math.pi * freq_hz
    travel = 2.0 * accel / omega ** 2
    m = 2.0 * dp + 1e-3 * dp
    lo = (-m, -m)
    hi = (nxt * dp + m + travel, nzt * dp + m)
    return _finish("sloshing_2d", 2, dp, fluid, walls, nzf * dp, lo, hi, seed,
                   wall_type=BOUND_MOVING, motion_amp=accel, motion_omega=omega,
                   cell_div=cell_div, x_sub=x_sub, meta=dict(tank=tank, fill=fill),
                   tank=(nxt, nzt))


def floating_box(dim=2, dp=0.02, tank=None, column=None, layer=0.15, box=None,
                 box_x=0.9, box_density=500.0, seed=0, cell_div=1, x_sub=1) -> Case:
    """A dam-break column released into a tank that holds a still water
    layer, with a rigid box floating on the layer (Section 3.2: a
    fluid-driven object).

    The box is a solid block of lattice cells (its particles are FLOATING,
    ids right after the fluid) of density ``box_density``, centred at
    x = box_x (and mid-width in 3-D) with its bottom at its equilibrium draft
    box_density / rho0 times its height below the layer surface; fluid cells
    it covers are removed.  Fluid and box particles start at the hydrostatic
    density below their own free surface (column or layer); the speed of
    sound is set by the column height.  The box stays clear of the walls
    for the first second or so; contact with walls is not modelled."""
    if tank is None:
        tank = (1.6, 0.8) if dim == 2 else (1.6, 0.6, 0.6)
    if column is None:
        column = (0.4, 0.5) if dim == 2 else (0.4, 0.6, 0.4)
    if box is None:
        box = (0.16, 0.10) if dim == 2 else (0.16, 0.16, 0.12)
    nt = [int(round(v / dp)) for v in tank]
    nc = [int(round(v / dp)) for v in column]
    nb = [int(round(v / dp)) for v in box]
    nzl = int(round(layer / dp))
    # lattice ranges: x, (y), z
    if dim == 2:
        col = _grid((0, nc[0]), (0, nc[1]))
        lay = _grid((nc[0], nt[0]), (0, nzl))
    else:
        col = _grid((0, nc[0]), (0, nt[1]), (0, nc[2]))
        lay = _grid((nc[0], nt[0]), (0, nt[1]), (0, nzl))
    draft = int(round(box_density / 1000.0 * nb[-1]))
    bx0 = int(round(box_x / dp)) - nb[0] // 2
    bz0 = nzl - draft
    if dim == 2:
        bidx = _grid((bx0, bx0 + nb[0]), (bz0, bz0 + nb[1]))
    else:
        by0 = nt[1] // 2 - nb[1] // 2
        bidx = _grid((bx0, bx0 + nb[0]), (by0, by0 + nb[1]), (bz0, bz0 + nb[2]))
    lo_b = bidx.min(axis=1)
    hi_b = bidx.max(axis=1)
    inside = np.all((lay >= lo_b[:, None]) & (lay <= hi_b[:, None]), axis=0)
    lay = lay[:, ~inside]
    fluid = np.concatenate([col, lay], axis=1)
    walls = _walls(dim, nt[0], nt[1] if dim == 3 else 1, nt[-1], closed_top=False)
    m = 2.0 * dp + 1e-3 * dp
    lo = tuple(-m for _ in range(dim))
    top = max(nt[-1] * dp, 2.5 * nc[-1] * dp) + m
    hi = tuple([nt[k] * dp + m for k in range(dim - 1)] + [top])
    tank_cells = tuple(nt)
    case = _finish(f"floating_box_{dim}d", dim, dp, fluid, np.concatenate([bidx, walls], axis=1),
                   nc[-1] * dp, lo, hi, seed, cell_div=cell_div, x_sub=x_sub,
                   meta=dict(tank=tank, column=column, layer=layer, box=box,
                             box_density=box_density), tank=tank_cells)
    nf = fluid.shape[1]
    nbox = bidx.shape[1]
    case.type[nf: nf + nbox] = FLOATING
    case.normal[:, nf: nf + nbox] = 0.0
    # hydrostatic density below each particle's own free surface: the layer
    # surface for the layer and the box, the column top for the column
    rho0 = case.params.rho0
    b_tait = case.params.c0 ** 2 * rho0 / case.params.gamma
    z = case.pos[dim - 1]
    in_layer = np.zeros(case.n, bool)
    in_layer[col.shape[1]: nf + nbox] = True
    depth = np.maximum(nzl * dp - z, 0.0)
    rho_layer = rho0 * np.power(1.0 + rho0 * GRAVITY * depth / b_tait, 1.0 / case.params.gamma)
    case.rho[in_layer] = rho_layer[in_layer].astype(np.float32)
    center = case.pos[:, nf: nf + nbox].mean(axis=1)
    c3 = [float(v) for v in center] + [0.0] * (3 - dim)
    case.bodies = [dict(id_first=nf, count=nbox, mass=box_density * nbox * dp ** dim,
                        center=tuple(c3), vel=(0.0, 0.0, 0.0), omega=(0.0, 0.0, 0.0))]
    case.params.floating = 1
    return case


def periodic_box(dim=2, shape=None, dp=0.01, periodic=(0,), walls=True, gravity=None,
                 seed=0, cell_div=1, x_sub=1, vel_scale=0.0, rho_jitter=0.0) -> Case:
    """A block of fluid of ``shape`` lattice cells that repeats along the
    components listed in ``periodic`` (Section 2.7), e.g. a channel periodic
    along x between a bottom and a top wall (``walls``: two layers on each
    open side of every non-periodic component; none if False).

    Along a periodic component the grid starts at the periodic boundary
    (x = 0) and spans the period exactly, so the cell size is a whole number
    of lattice spacings (the smallest one >= 2h / cell_div) and the period a
    whole number of cells (``shape`` is rounded up to one).  ``gravity``
    defaults to -g along the last component; the initial density is
    hydrostatic below the top of the fluid when gravity has a vertical part.
    Optional seeded random velocities and density jitter as in block_case."""
    if shape is None:
        shape = (40, 12) if dim == 2 else (16, 12, 10)
    periodic = tuple(sorted(set(int(k) for k in periodic)))
    h = math.sqrt(dim) * dp
    k_cs = int(math.ceil(2.0 * h / (cell_div * dp) - 1e-9))
    cs = k_cs * dp
    shape = [int(math.ceil(s / k_cs) * k_cs) if k in periodic else int(s)
             for k, s in enumerate(shape)]
    fluid = _grid(*[(0, s) for s in shape])
    parts = []
    if walls:
        for k in range(dim):
            if k in periodic:
                continue
            for side in (0, 1):
                rng_k = [(0, s) for s in shape]
                # the wall layers span the other non-periodic components'
                # wall thickness too (corners), the periodic ones as they are
                for j in range(dim):
                    if j != k and j not in periodic:
                        rng_k[j] = (-2, shape[j] + 2)
                rng_k[k] = (-2, 0) if side == 0 else (shape[k], shape[k] + 2)
                parts.append(_grid(*rng_k))
        # corners counted once: keep unique lattice points
        if parts:
            wall = np.unique(np.concatenate(parts, axis=1), axis=1)
        else:
            wall = np.zeros((dim, 0), np.int64)
    else:
        wall = np.zeros((dim, 0), np.int64)
    idx = np.concatenate([fluid, wall], axis=1)
    n = idx.shape[1]
    rng = np.random.default_rng(seed)
    pos = (idx.astype(np.float64) + 0.5) * dp
    pos += rng.uniform(-1e-4 * dp, 1e-4 * dp, size=pos.shape)
    ptype = np.full(n, FLUID, np.uint8)
    ptype[fluid.shape[1]:] = BOUND_FIXED
    g = [0.0, 0.0, 0.0]
    if gravity is None:
        g[dim - 1] = -GRAVITY
    else:
        g = [float(v) for v in gravity] + [0.0] * (3 - len(gravity))
    height = shape[dim - 1] * dp
    rho0, gamma = 1000.0, 7.0
    c0 = 10.0 * math.sqrt(GRAVITY * height)
    b_tait = c0 * c0 * rho0 / gamma
    gz = abs(g[dim - 1])
    depth = np.maximum(height - pos[dim - 1], 0.0)
    rho = rho0 * np.power(1.0 + rho0 * gz * depth / b_tait, 1.0 / gamma)
    origin, ncell, period = [0.0] * 3, [1, 1, 1], [0.0] * 3
    for k in range(dim):
        if k in periodic:
            origin[k] = 0.0
            ncell[k] = shape[k] // k_cs
            period[k] = shape[k] * dp
        else:
            m = 2.0 * dp + 1e-3 * dp + 2 * cs
            origin[k] = -m
            ncell[k] = int(math.ceil((shape[k] * dp + 2 * m) / cs))
    ncell[0] *= x_sub
    mass = rho0 * dp ** dim
    params = CaseParams(
        name=f"periodic_box_{dim}d", dim=dim, dp=dp, h=h, rho0=rho0, gamma=gamma, c0=c0,
        alpha=0.01, delta=0.1, eta2=0.001 * h * h, cfl=0.2, mass_fluid=mass, mass_bound=mass,
        gravity=tuple(g), ddt=1, cell_div=cell_div, x_sub=x_sub, origin=tuple(origin),
        cell_size=cs, inv_cell_size=1.0 / cs, ncell=tuple(ncell), fluid_height=height,
        period=tuple(period))
    normal = np.zeros((dim, n), np.float32)
    if wall.shape[1]:
        # walls lie outside the fluid only along non-periodic components
        normal[:, fluid.shape[1]:] = _ghost_vectors(wall, tuple(shape), dp)
    case = Case(params=params, pos=np.ascontiguousarray(pos),
                vel=np.zeros((dim, n), np.float32), rho=rho.astype(np.float32), type=ptype,
                meta=dict(shape=tuple(shape), periodic=periodic, walls=walls), normal=normal)
    rng2 = np.random.default_rng(seed + 7919)
    if vel_scale:
        case.vel[:] = rng2.uniform(-vel_scale, vel_scale, case.vel.shape).astype(np.float32)
    if rho_jitter:
        case.rho[:] = (case.rho * (1.0 + rng2.uniform(-rho_jitter, rho_jitter,
                                                      case.n))).astype(np.float32)
    return case
