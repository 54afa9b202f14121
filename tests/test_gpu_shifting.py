"""Particle shifting (Section 2.8, Eq. 40-41, 53, 54) on the GPU through the
C ABI, against the CPU oracle.

Bars: the concentration C within 1e-5 of the oracle's (a sum of positive
FP32 terms); the shift within 1e-4 of the largest oracle shift (the
interaction's FP32 bar), on particles whose surface decision (C below the
threshold) is the oracle's; the positions move by exactly the reported
shift; a 2-D dam break with shifting after 150 steps within 1e-3 of the
tank length of the oracle's front.
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
    from test_gpu_parity import _perturbed, _say, _u32


def _cases():
    return {
        "2d_dam": _perturbed(cases.dam_break_2d(cell_div=2, x_sub=4), 71, vel=0.5),
        "2d_dam_cd1_cubic": _with(_perturbed(cases.dam_break_2d(), 72, vel=0.5), kernel=1),
        "3d_block": _perturbed(cases.block_case(3, (14, 12, 10), walls=True, seed=3, cell_div=2,
                                                x_sub=4), 73, vel=0.4),
        "3d_channel_periodic": _perturbed(cases.periodic_box(3, shape=(24, 16, 10),
                                                             periodic=(0, 1), cell_div=2,
                                                             x_sub=4), 74, vel=0.4),
        "2d_periodic_cd1": _perturbed(cases.periodic_box(2, shape=(60, 14), periodic=(0,),
                                                         cell_div=1), 75, vel=0.4),
    }


def _with(c, **kw):
    return cases.Case(dataclasses.replace(c.params, **kw), c.pos, c.vel, c.rho, c.type,
                      dict(c.meta), c.normal)


@pytest.mark.parametrize("name", ["2d_dam", "2d_dam_cd1_cubic", "3d_block",
                                  "3d_channel_periodic", "2d_periodic_cd1"])
@pytest.mark.parametrize("fs", [0.0, 0.9])
def test_shifting_matches_oracle(name, fs):
    c = _cases()[name]
    c = _with(c, shift_coef=2.0, shift_fs=fs)
    cp, n = c.params, c.n
    P = S.make_params(cp)
    src = S.DeviceState.from_case(c, DEV)
    dst = S.DeviceState.empty(cp.dim, n, DEV)
    key = torch.empty(n, dtype=torch.int32, device=DEV)
    perm = torch.empty_like(key)
    start = torch.empty(cp.ncell_total() + 1, dtype=torch.int32, device=DEV)
    ws = torch.zeros(S.sph_workspace_bytes(P, n), dtype=torch.uint8, device=DEV)
    S.sph_bin_cells(P, n, src, dst, key, perm, start, ws)
    torch.cuda.synchronize()
    pos = dst.pos.cpu().numpy()
    vel = dst.vel.cpu().numpy().astype(np.float64)
    rho = dst.rho.cpu().numpy().astype(np.float64)
    typ = dst.type.cpu().numpy()
    dt_v = 2e-4
    dt = torch.full((1,), dt_v, dtype=torch.float64, device=DEV)
    conc = torch.full((n,), float("nan"), dtype=torch.float32, device=DEV)
    shift = torch.full((cp.dim, n), float("nan"), dtype=torch.float32, device=DEV)
    S.sph_shifting(P, n, dst, key, start, dt, ws, conc=conc, shift=shift)
    torch.cuda.synchronize()
    assert S.sph_read_error(ws) == 0
    cg = conc.cpu().numpy().astype(np.float64)
    dg = shift.cpu().numpy().astype(np.float64)
    pos1 = dst.pos.cpu().numpy()
    co, _, do = oracle.shift(cp, pos, vel, rho, typ, dt_v)
    ec = np.abs(cg - co).max()
    fl = typ == cases.FLUID
    same = np.ones(n, bool)
    if fs > 0:
        same = (cg < fs) == (co < fs)
    scale = np.abs(do[:, fl]).max()
    ed = np.abs(dg - do)[:, fl & same].max() / scale
    _say(f"  {name} fs {fs}: n {n}, C err {ec:.2e} (range {co[fl].min():.3f}..{co.max():.3f}), "
         f"shift rel err {ed:.2e} (max {scale:.2e} m), surface decisions differing "
         f"{(~same & fl).sum()}")
    assert ec < 1e-5
    assert ed < 1e-4
    assert (~same & fl).sum() <= max(2, fl.sum() // 1000)
    assert np.all(dg[:, ~fl] == 0)
    assert np.array_equal(pos1, pos + dg)


def test_dam_break_with_shifting_matches_oracle():
    """The small 2-D dam break with shifting (A_s = 2, surface threshold
    0.9), 150 symplectic steps: the front within 1e-3 of the tank length of
    the oracle's, and different from the run without shifting."""
    c = cases.dam_break_2d(cell_div=2, x_sub=4)
    cs = _with(c, shift_coef=2.0, shift_fs=0.9)
    sim = Simulation(cs, DEV)
    sim.run(150)
    torch.cuda.synchronize()
    assert sim.error() == 0
    st = sim.host_state()
    fg = st["pos"][0][st["type"] == 0].max()
    out = oracle.run(cs.params, c.pos, c.vel, c.rho, c.type, 150)
    assert out["status"] == 0
    fo = out["pos"][0][out["type"] == 0].max()
    d = np.abs(st["pos"] - out["pos"]).max()
    _say(f"  shifting front after 150 steps: gpu {fg:.6f} oracle {fo:.6f}; max position diff "
         f"{d:.2e} m")
    assert abs(fg - fo) < 1e-3 * 1.6
    assert st["t"] == pytest.approx(out["t"], rel=1e-4)
    plain = oracle.run(c.params, c.pos, c.vel, c.rho, c.type, 150)
    assert np.abs(plain["pos"] - out["pos"]).max() > 1e-6


@pytest.mark.parametrize("name", ["3d_block", "3d_periodic"])
@pytest.mark.parametrize("move", [0.05, 0.3])
def test_shifting_on_reused_cells_matches_oracle(name, move):
    """Shifting after the corrector in a step that bins once: the view of
    the moved state is refreshed on the cells of state n and both passes
    search them with SPH_INTERACT_REUSE_CELLS (one more cell of reach, the
    cut widened by the recorded displacement).  C and the shifts against the
    oracle's shifting of the moved positions, particles moved by 0.05 and 0.3
    of a cell; half a cell raises SPH_ERR_MARGIN."""
    from test_gpu_reuse import HalfStep, _case
    c = _with(_case(name), shift_coef=2.0, shift_fs=0.9)
    hs = HalfStep(c, move)
    cp, n = hs.cp, hs.n
    S.sph_refresh_view(hs.P, n, hs.st, hs.key, hs.ws)
    torch.cuda.synchronize()
    pos = hs.st.pos.cpu().numpy()
    vel = hs.st.vel.cpu().numpy().astype(np.float64)
    rho = hs.st.rho.cpu().numpy().astype(np.float64)
    typ = hs.st.type.cpu().numpy()
    moved = np.sqrt(((pos - hs.saved.pos.cpu().numpy()) ** 2).sum(axis=0)).max()
    dt_v = 2e-4
    dt = torch.full((1,), dt_v, dtype=torch.float64, device=DEV)
    conc = torch.full((n,), float("nan"), dtype=torch.float32, device=DEV)
    shift = torch.full((cp.dim, n), float("nan"), dtype=torch.float32, device=DEV)
    S.sph_shifting(hs.P, n, hs.st, hs.key, hs.start, dt, hs.ws, conc=conc, shift=shift,
                   flags=S.SPH_INTERACT_REUSE_CELLS)
    torch.cuda.synchronize()
    assert S.sph_read_error(hs.ws) == 0
    cg = conc.cpu().numpy().astype(np.float64)
    dg = shift.cpu().numpy().astype(np.float64)
    co, _, do = oracle.shift(cp, pos, vel, rho, typ, dt_v)
    fl = typ == cases.FLUID
    same = (cg < cp.shift_fs) == (co < cp.shift_fs)
    scale = np.abs(do[:, fl]).max()
    ec = np.abs(cg - co).max()
    ed = np.abs(dg - do)[:, fl & same].max() / scale
    _say(f"  {name} move {move} cell (max {moved / cp.cell_size:.3f}): C err {ec:.2e}, shift "
         f"rel err {ed:.2e}, surface decisions differing {(~same & fl).sum()}")
    assert ec < 1e-5
    assert ed < 1e-4
    assert (~same & fl).sum() <= max(2, fl.sum() // 1000)
    assert np.array_equal(hs.st.pos.cpu().numpy(), pos + dg)


def test_shifting_on_reused_cells_beyond_the_margin_raises_the_error():
    from test_gpu_reuse import HalfStep, _case
    c = _with(_case("3d_block"), shift_coef=2.0, shift_fs=0.9)
    hs = HalfStep(c, 0.6)
    S.sph_refresh_view(hs.P, hs.n, hs.st, hs.key, hs.ws)
    dt = torch.full((1,), 2e-4, dtype=torch.float64, device=DEV)
    S.sph_shifting(hs.P, hs.n, hs.st, hs.key, hs.start, dt, hs.ws,
                   flags=S.SPH_INTERACT_REUSE_CELLS)
    torch.cuda.synchronize()
    err = S.sph_read_error(hs.ws)
    _say(f"  shifting after a 0.6-cell move: error word {err}")
    assert err & S.SPH_ERR_MARGIN
