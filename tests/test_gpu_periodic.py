"""Periodic boundaries (Section 2.7) on the GPU through the C ABI, against
the CPU oracle and a closed form.

Bars: wrapped positions and keys bit-exact (both sides wrap with the same
FP64 operations); FP64 neighbour counts bit-exact; rates within 1e-4 of the
oracle's maximum (the interaction's FP32 bar); a uniformly moving periodic
lattice at its start plus v t after whole steps, to 1e-8 m (the forces of an
exact lattice cancel to FP32 rounding); a periodic channel after whole steps
within 1e-5 of the period of the oracle's positions.
"""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
from paper_2104_00537_amd import cases

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
if torch.cuda.is_available():
    from paper_2104_00537_amd import sph as S
    from paper_2104_00537_amd.runner import Simulation
    from test_gpu_parity import _perturbed, _rel_errors, _say, _u32


CASES = {
    "2d_channel_cd1": dict(dim=2, shape=(60, 14), periodic=(0,), walls=True, cell_div=1, x_sub=1),
    "2d_channel_cd2_xs4": dict(dim=2, shape=(60, 14), periodic=(0,), walls=True, cell_div=2,
                               x_sub=4),
    "2d_full": dict(dim=2, shape=(36, 24), periodic=(0, 1), walls=False, cell_div=2, x_sub=4,
                    gravity=(0.0, 0.0, 0.0)),
    "3d_channel": dict(dim=3, shape=(24, 16, 10), periodic=(0, 1), walls=True, cell_div=2,
                       x_sub=4),
    "3d_channel_cd1": dict(dim=3, shape=(24, 16, 10), periodic=(0,), walls=True, cell_div=1,
                           x_sub=2),
    "3d_full": dict(dim=3, shape=(16, 16, 16), periodic=(0, 1, 2), walls=False, cell_div=2,
                    x_sub=4, gravity=(0.0, 0.0, 0.0)),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_periodic_binning_and_interaction_match_oracle(name):
    kw = dict(CASES[name])
    c = cases.periodic_box(**kw, seed=3, vel_scale=0.4, rho_jitter=0.003)
    cp, n = c.params, c.n
    # move everything by 0.4 of the period along x (and y) so that the
    # periodic boundary cuts through the fluid and positions must be wrapped
    pos = c.pos.copy()
    for k in kw["periodic"]:
        pos[k] += 0.4 * cp.period[k]
    c = cases.Case(cp, pos, c.vel, c.rho, c.type, dict(c.meta), c.normal)
    P = S.make_params(cp)
    src = S.DeviceState.from_case(c, DEV)
    dst = S.DeviceState.empty(cp.dim, n, DEV)
    key = torch.empty(n, dtype=torch.int32, device=DEV)
    perm = torch.empty_like(key)
    start = torch.empty(cp.ncell_total() + 1, dtype=torch.int32, device=DEV)
    ws = torch.zeros(S.sph_workspace_bytes(P, n), dtype=torch.uint8, device=DEV)
    S.sph_bin_cells(P, n, src, dst, key, perm, start, ws)
    torch.cuda.synchronize()
    assert S.sph_read_error(ws) == 0
    pm = _u32(perm)[:n].astype(np.int64)
    want_pos = oracle.wrap(cp, pos)
    got_pos = dst.pos.cpu().numpy()
    assert np.array_equal(got_pos, want_pos[:, pm])
    keys_o = oracle.cell_keys(cp, want_pos)
    assert np.array_equal(_u32(key)[:n], keys_o[pm])
    assert np.array_equal(pm, oracle.sort_perm(keys_o))
    vel = dst.vel.cpu().numpy().astype(np.float64)
    rho = dst.rho.cpu().numpy().astype(np.float64)
    typ = dst.type.cpu().numpy()
    res = {}
    for flags in (S.SPH_DIAG_COUNT_F64, 0):
        ace = torch.full((cp.dim, n), float("nan"), dtype=torch.float32, device=DEV)
        arho = torch.full((n,), float("nan"), dtype=torch.float32, device=DEV)
        visc = torch.full((n,), float("nan"), dtype=torch.float32, device=DEV)
        nbr = torch.full((n,), -1, dtype=torch.int32, device=DEV)
        S.sph_interact(P, n, dst, key, start, ace, arho, ws, visc=visc, nbr=nbr, flags=flags)
        torch.cuda.synchronize()
        res[flags] = (ace.cpu().numpy().astype(np.float64), arho.cpu().numpy().astype(np.float64),
                      visc.cpu().numpy().astype(np.float64), _u32(nbr)[:n])
    ace_o, arho_o, visc_o, nbr_o = oracle.interact(cp, got_pos, vel, rho, typ)
    fl = typ == cases.FLUID
    assert np.array_equal(res[S.SPH_DIAG_COUNT_F64][3], nbr_o)
    open_nbr = oracle.interact(dataclasses.replace(cp, period=(0.0, 0.0, 0.0)), got_pos, vel, rho,
                               typ)[3]
    assert nbr_o.sum() > open_nbr.sum()  # pairs across the boundary exist
    for flags, (ace, arho, visc, _) in res.items():
        ea, er, ev = _rel_errors((ace, arho, visc), (ace_o, arho_o, visc_o), fl)
        _say(f"  {name} flags {flags}: n {n}, rel err ace {ea:.2e} arho {er:.2e} visc {ev:.2e}; "
             f"pairs {nbr_o.sum()} (open {open_nbr.sum()})")
        assert ea < 1e-4 and er < 1e-4 and ev < 1e-4


@pytest.mark.parametrize("dim", [2, 3])
def test_moving_periodic_lattice_translates_on_gpu(dim):
    """An exact lattice at uniform density filling a fully periodic box and
    moving uniformly: after whole steps every particle is at its start plus
    v t brought back into the box; many cross the boundary."""
    c = cases.periodic_box(dim, shape=(36, 24) if dim == 2 else (16, 16, 16),
                           periodic=tuple(range(dim)), walls=False, gravity=(0.0, 0.0, 0.0),
                           cell_div=2, x_sub=4)
    cp = c.params
    idx = np.round(c.pos / cp.dp - 0.5)
    pos = (idx + 0.5) * cp.dp
    v = np.array([3.7, -2.1, 1.3][:dim], np.float32)
    vel = np.tile(v[:, None], (1, c.n)).astype(np.float32)
    c = cases.Case(cp, pos, vel, np.full(c.n, 1005.0, np.float32), c.type, dict(c.meta),
                   c.normal)
    sim = Simulation(c, DEV)
    sim.run(60)
    torch.cuda.synchronize()
    assert sim.error() == 0
    st = sim.host_state()
    t = st["t"]
    L = np.array(cp.period[:dim])[:, None]
    shift = v.astype(np.float64)[:, None] * t
    want = np.mod(pos + shift, L)
    d = np.abs(st["pos"] - want)
    d = np.minimum(d, L - d)
    crossed = np.any((pos + shift >= L) | (pos + shift < 0), axis=0).sum()
    _say(f"  {dim}d lattice: t {t:.4f}, max position error {d.max():.2e} m, crossed {crossed}")
    assert d.max() < 1e-8
    assert crossed > c.n // 20
    assert np.all(st["pos"] >= 0) and np.all(st["pos"] < L)


@pytest.mark.parametrize("dim,steps", [(2, 100), (3, 15)])
def test_periodic_channel_steps_match_oracle(dim, steps):
    """A channel periodic along x (and y), driven along x by a body force,
    whole symplectic steps on the GPU and in the oracle: positions (nearest
    image) within 1e-5 of the period, no particle lost."""
    kw = dict(dim=dim, shape=(60, 14) if dim == 2 else (24, 16, 10),
              periodic=(0,) if dim == 2 else (0, 1), walls=True, cell_div=2, x_sub=4)
    g = [2.0, 0.0, 0.0]
    g[dim - 1] = -cases.GRAVITY
    c = cases.periodic_box(**kw, gravity=tuple(g[:dim]) + (0.0,) * (3 - dim), seed=1,
                           vel_scale=0.3)
    fl = c.type == cases.FLUID
    c.vel[0, fl] += 1.5  # a mean flow along x, so particles cross the boundary
    sim = Simulation(c, DEV)
    sim.run(steps)
    torch.cuda.synchronize()
    assert sim.error() == 0
    st = sim.host_state()
    out = oracle.run(c.params, c.pos, c.vel, c.rho, c.type, steps)
    assert out["status"] == 0 and not np.any(out["type"] & cases.EXCLUDED)
    d = np.abs(st["pos"] - out["pos"])
    for k in kw["periodic"]:
        d[k] = np.minimum(d[k], c.params.period[k] - d[k])
    Lx = c.params.period[0]
    crossed = np.sum(np.abs(st["pos"][0] - c.pos[0]) > 0.5 * Lx)
    _say(f"  {dim}d channel after {steps} steps: t {st['t']:.4f} (oracle {out['t']:.4f}), "
         f"max position diff {d.max():.2e} m, wrapped particles {crossed}")
    assert st["t"] == pytest.approx(out["t"], rel=1e-5)
    assert d.max() < 1e-5 * Lx
    assert crossed > 0
