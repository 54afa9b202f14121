"""The second interaction of a symplectic step on the cells of the first
(sph_refresh_view + SPH_INTERACT_REUSE_CELLS) on the GPU: the same pairs as
a new binning would give, against the CPU oracle, with the displacement
margin at work.

Bars: FP64 neighbour counts bit-exact with the oracle's on the half-step
state; rates within 1e-4 of the oracle's maximum (the interaction's FP32
bar) and within 1e-5 of those of a new binning of the same state (only the
summation order differs); particles moved by up to 0.3 cell; a move of half
a cell or more raises SPH_ERR_MARGIN; whole runs with and without reused
cells agree to 1e-6 of the tank length.
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


def _case(name):
    if name == "3d_block":
        return _perturbed(cases.block_case(3, (16, 12, 10), walls=True, seed=5, cell_div=2,
                                           x_sub=4), 91, vel=0.6)
    if name == "2d_dam_cd1":
        return _perturbed(cases.dam_break_2d(), 92, vel=0.6)
    if name == "3d_periodic":
        return _perturbed(cases.periodic_box(3, shape=(24, 16, 10), periodic=(0, 1), cell_div=2,
                                             x_sub=4), 93, vel=0.6)
    if name == "2d_floating":
        c = cases.floating_box(2, dp=0.02, cell_div=2, x_sub=4)
        p = _perturbed(c, 94, vel=0.3)
        p.bodies = [dict(b, vel=(0.4, -0.2, 0.0), omega=(3.0, 0.0, 0.0)) for b in c.bodies]
        p.vel[:, c.type == cases.FLOATING] = 0.0
        return p
    raise KeyError(name)


class HalfStep:
    """Bin and interact at state n, then the predictor with a chosen dt and
    zero rates (the particles move dt/2 v, up to a given fraction of a cell;
    floating bodies move rigidly), leaving the half state."""

    def __init__(self, c, move_cells):
        cp = self.cp = c.params
        n = self.n = c.n
        self.P = S.make_params(cp)
        self.src = S.DeviceState.from_case(c, DEV)
        self.st = S.DeviceState.empty(cp.dim, n, DEV)
        self.saved = S.DeviceState.empty(cp.dim, n, DEV, with_type=False, with_id=False)
        self.key = torch.empty(n, dtype=torch.int32, device=DEV)
        self.perm = torch.empty_like(self.key)
        self.start = torch.empty(cp.ncell_total() + 1, dtype=torch.int32, device=DEV)
        self.ws = torch.zeros(S.sph_workspace_bytes(self.P, n), dtype=torch.uint8, device=DEV)
        self.ace = torch.empty((cp.dim, n), dtype=torch.float32, device=DEV)
        self.arho = torch.empty(n, dtype=torch.float32, device=DEV)
        S.sph_bin_cells(self.P, n, self.src, self.st, self.key, self.perm, self.start, self.ws)
        S.sph_interact(self.P, n, self.st, self.key, self.start, self.ace, self.arho, self.ws)
        vmax = float(np.sqrt((c.vel.astype(np.float64) ** 2).sum(axis=0)).max())
        if c.bodies:  # a bound on the body's particle speeds (box half-diagonal < 0.1 m)
            b = c.bodies[0]
            vmax = max(vmax, float(np.linalg.norm(b["vel"])) + abs(b["omega"][0]) * 0.1)
        dt_v = 2.0 * move_cells * cp.cell_size / vmax  # the predictor moves dt/2 v
        self.dt = torch.full((1,), dt_v, dtype=torch.float64, device=DEV)
        # a pure move: with this long a step the rates would change the
        # velocities and densities far more than a real step does
        self.ace.zero_()
        self.arho.zero_()
        self.t = torch.zeros(1, dtype=torch.float64, device=DEV)
        S.sph_symplectic_step(self.P, n, 0, self.dt, self.t, self.saved, self.st, self.ace,
                              self.arho, self.ws)
        if c.bodies:
            self.bodies = S.bodies_to_device(c.bodies, DEV)
            S.sph_floating_step(self.P, n, 0, self.dt, self.bodies, self.saved, self.st, self.ace,
                                self.ws)
        torch.cuda.synchronize()

    def interact(self, flags):
        n, cp = self.n, self.cp
        ace = torch.full((cp.dim, n), float("nan"), dtype=torch.float32, device=DEV)
        arho = torch.full((n,), float("nan"), dtype=torch.float32, device=DEV)
        visc = torch.full((n,), float("nan"), dtype=torch.float32, device=DEV)
        nbr = torch.full((n,), -1, dtype=torch.int32, device=DEV)
        S.sph_interact(self.P, n, self.st, self.key, self.start, ace, arho, self.ws, visc=visc,
                       nbr=nbr, flags=flags)
        torch.cuda.synchronize()
        return (ace.cpu().numpy().astype(np.float64), arho.cpu().numpy().astype(np.float64),
                visc.cpu().numpy().astype(np.float64), _u32(nbr)[:n])


@pytest.mark.parametrize("name", ["3d_block", "2d_dam_cd1", "3d_periodic", "2d_floating"])
@pytest.mark.parametrize("move", [0.05, 0.3])
def test_reused_cells_find_the_oracles_pairs(name, move):
    c = _case(name)
    hs = HalfStep(c, move)
    S.sph_refresh_view(hs.P, hs.n, hs.st, hs.key, hs.ws)
    torch.cuda.synchronize()
    # the default lane count (four lanes per target for the small cases here)
    # and one lane per target, the kernel that runs the n+1/2 pass of large
    # cases
    one = S.SPH_INTERACT_ONE_LANE
    res = {f: hs.interact(f | S.SPH_INTERACT_REUSE_CELLS)
           for f in (S.SPH_DIAG_COUNT_F64, 0, S.SPH_DIAG_COUNT_F64 | one, one)}
    err = S.sph_read_error(hs.ws)
    assert err == 0, err
    pos = hs.st.pos.cpu().numpy()
    vel = hs.st.vel.cpu().numpy().astype(np.float64)
    rho = hs.st.rho.cpu().numpy().astype(np.float64)
    typ = hs.st.type.cpu().numpy()
    moved = np.sqrt(((pos - hs.saved.pos.cpu().numpy()) ** 2).sum(axis=0)).max()
    ace_o, arho_o, visc_o, nbr_o = oracle.interact(hs.cp, pos, vel, rho, typ)
    assert np.array_equal(res[S.SPH_DIAG_COUNT_F64][3], nbr_o)
    assert np.array_equal(res[S.SPH_DIAG_COUNT_F64 | one][3], nbr_o)
    fl = typ == cases.FLUID
    for f, (ace, arho, visc, _) in res.items():
        ea, er, ev = _rel_errors((ace, arho, visc), (ace_o, arho_o, visc_o), fl)
        _say(f"  {name} move {move} cell (max {moved / hs.cp.cell_size:.3f}) flags {f}: ace "
             f"{ea:.2e} arho {er:.2e} visc {ev:.2e}")
        assert ea < 1e-4 and er < 1e-4 and ev < 1e-4
    # a new binning of the same half state gives the same rates
    half = cases.Case(hs.cp, pos, hs.st.vel.cpu().numpy(), hs.st.rho.cpu().numpy(), typ, {},
                      np.zeros_like(hs.st.vel.cpu().numpy()))
    src = S.DeviceState.from_case(half, DEV)
    dst = S.DeviceState.empty(hs.cp.dim, hs.n, DEV)
    ws = torch.zeros_like(hs.ws)
    key = torch.empty_like(hs.key)
    perm = torch.empty_like(hs.perm)
    start = torch.empty_like(hs.start)
    S.sph_bin_cells(hs.P, hs.n, src, dst, key, perm, start, ws)
    ace = torch.empty_like(hs.ace)
    arho = torch.empty_like(hs.arho)
    S.sph_interact(hs.P, hs.n, dst, key, start, ace, arho, ws)
    torch.cuda.synchronize()
    pm = _u32(perm)[:hs.n].astype(np.int64)  # dst slot j holds half-state index pm[j]
    ace_b = np.empty_like(ace_o)
    arho_b = np.empty_like(arho_o)
    ace_b[:, pm] = ace.cpu().numpy()
    arho_b[pm] = arho.cpu().numpy()
    ace_r, arho_r = res[0][0], res[0][1]
    assert np.abs(ace_r - ace_b)[:, fl].max() <= 1e-5 * np.abs(ace_o[:, fl]).max()
    assert np.abs(arho_r - arho_b).max() <= 1e-5 * np.abs(arho_o).max()


def test_cells_of_a_moved_state_without_reuse_raise_the_error():
    """After a predictor moved the particles, an interaction that keeps the
    cells' own reach (no SPH_INTERACT_REUSE_CELLS) may miss pairs: it sets
    SPH_ERR_MARGIN; a new binning clears the record."""
    hs = HalfStep(_case("3d_block"), 0.05)
    S.sph_refresh_view(hs.P, hs.n, hs.st, hs.key, hs.ws)
    hs.interact(S.SPH_INTERACT_REUSE_CELLS)
    assert S.sph_read_error(hs.ws) == 0
    for flags in (0, S.SPH_INTERACT_ONE_LANE):
        S.sph_clear_error(hs.ws)
        hs.interact(flags)
        err = S.sph_read_error(hs.ws)
        _say(f"  error word, interaction without reuse after a move (flags {flags}): {err}")
        assert err == S.SPH_ERR_MARGIN
    S.sph_clear_error(hs.ws)
    dst = S.DeviceState.empty(hs.cp.dim, hs.n, DEV)
    S.sph_bin_cells(hs.P, hs.n, hs.st, dst, hs.key, hs.perm, hs.start, hs.ws)
    ace = torch.empty_like(hs.ace)
    arho = torch.empty_like(hs.arho)
    S.sph_interact(hs.P, hs.n, dst, hs.key, hs.start, ace, arho, hs.ws)
    torch.cuda.synchronize()
    assert S.sph_read_error(hs.ws) == 0


def test_moves_beyond_the_margin_raise_the_error():
    hs = HalfStep(_case("3d_block"), 0.6)
    S.sph_refresh_view(hs.P, hs.n, hs.st, hs.key, hs.ws)
    hs.interact(S.SPH_INTERACT_REUSE_CELLS)
    err = S.sph_read_error(hs.ws)
    _say(f"  error word after a 0.6-cell move: {err}")
    assert err & S.SPH_ERR_MARGIN


@pytest.mark.parametrize("name", ["dam2d", "floating2d", "periodic3d", "shifting2d"])
def test_runs_with_and_without_reused_cells_agree(name):
    if name == "dam2d":
        c = cases.dam_break_2d(cell_div=2, x_sub=4)
    elif name == "shifting2d":
        # shifting after the corrector on the reused cells, surface correction on
        d = cases.dam_break_2d(cell_div=2, x_sub=4)
        c = cases.Case(dataclasses.replace(d.params, shift_coef=2.0, shift_fs=0.9), d.pos, d.vel,
                       d.rho, d.type, dict(d.meta), d.normal)
    elif name == "floating2d":
        c = cases.floating_box(2, dp=0.02, cell_div=2, x_sub=4)
    else:
        c = cases.periodic_box(3, shape=(24, 16, 10), periodic=(0, 1), cell_div=2, x_sub=4,
                               vel_scale=0.3, seed=4)
    out = []
    for reuse in (True, False):
        sim = Simulation(c, DEV, reuse_cells=reuse)
        sim.run(100)
        torch.cuda.synchronize()
        assert sim.error() == 0
        out.append(sim.host_state())
    d = np.abs(out[0]["pos"] - out[1]["pos"])
    for k in range(c.params.dim):
        L = c.params.period[k]
        if L > 0:
            d[k] = np.minimum(d[k], L - d[k])
    _say(f"  {name}: 100 steps with/without reused cells, max position diff {d.max():.2e} m")
    assert d.max() < 1e-6 * 1.6
    assert out[0]["t"] == pytest.approx(out[1]["t"], rel=1e-5)
