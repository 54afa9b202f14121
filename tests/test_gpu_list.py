"""Neighbour lists (sph_build_list / sph_interact_list) against the cell walk
(sph_interact) on the same views, through the C ABI.

The replay runs every listed candidate through the walk's FP32 test and pair
terms in the walk's order, so the bar is equality: rates, visc and counts
(FP32 and FP64) identical to the walk's, on the binning's view (state n) and
on the view refreshed after a predictor (n+1/2, reused cells), including
the fallbacks: a displacement beyond the skin (the pass walks every target),
targets whose chunks do not fit a small buffer (they walk), and a list built
on an earlier binning (walks, and SPH_ERR_LIST).  The walk itself is pinned
against the oracle by the other parity tests.
"""
import numpy as np
import pytest
import torch

from paper_2104_00537_amd import cases

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2104_00537_amd import sph as S
    from paper_2104_00537_amd.runner import Simulation

DEV = "cuda:0"
ONE = 16  # SPH_INTERACT_ONE_LANE: the walk of one lane per target (the replay's order)


def _say(*a):
    print(*a, flush=True)


def _perturbed(case, seed, vel=0.5):
    rng = np.random.default_rng(seed)
    c = cases.Case(case.params, case.pos.copy(), case.vel.copy(), case.rho.copy(),
                   case.type.copy(), dict(case.meta), case.normal)
    c.vel[:] = rng.uniform(-vel, vel, c.vel.shape).astype(np.float32)
    c.rho[:] = (c.rho * (1 + rng.uniform(-0.003, 0.003, c.n))).astype(np.float32)
    return c


class Setup:
    def __init__(self, case, list_bytes=None):
        self.case = case
        cp = case.params
        self.P = S.make_params(cp)
        self.n = n = case.n
        self.dim = cp.dim
        self.src = S.DeviceState.from_case(case, DEV)
        self.dst = S.DeviceState.empty(cp.dim, n, DEV)
        self.saved = S.DeviceState.empty(cp.dim, n, DEV, with_type=False, with_id=False)
        self.key = torch.empty(n, dtype=torch.int32, device=DEV)
        self.perm = torch.empty(n, dtype=torch.int32, device=DEV)
        self.start = torch.empty(cp.ncell_total() + 1, dtype=torch.int32, device=DEV)
        self.ws = torch.zeros(S.sph_workspace_bytes(self.P, n), dtype=torch.uint8, device=DEV)
        nb = S.sph_list_bytes(self.P, n) if list_bytes is None else list_bytes
        self.lst = torch.zeros(nb, dtype=torch.uint8, device=DEV)
        self.dt = torch.zeros(1, dtype=torch.float64, device=DEV)
        self.t = torch.zeros(1, dtype=torch.float64, device=DEV)

    def bin(self):
        S.sph_bin_cells(self.P, self.n, self.src, self.dst, self.key, self.perm, self.start,
                        self.ws)

    def build(self, skin):
        S.sph_build_list(self.P, self.n, self.dst, self.key, self.start, skin, self.lst, self.ws)

    def out(self):
        n = self.n
        return (torch.full((self.dim, n), float("nan"), dtype=torch.float32, device=DEV),
                torch.full((n,), float("nan"), dtype=torch.float32, device=DEV),
                torch.full((n,), float("nan"), dtype=torch.float32, device=DEV),
                torch.full((n,), -1, dtype=torch.int32, device=DEV))

    def walk_marked(self):
        """Targets whose list did not fit (count = 0xffffffff after the
        256-byte header): they walk their cells."""
        cnt = self.lst[256: 256 + 4 * self.n].view(torch.int32)
        return int((cnt == -1).sum().item())

    def walk(self, flags):
        o = self.out()
        S.sph_interact(self.P, self.n, self.dst, self.key, self.start, o[0], o[1], self.ws,
                       visc=o[2], nbr=o[3], flags=flags | ONE)
        return o

    def replay(self, flags):
        o = self.out()
        S.sph_interact_list(self.P, self.n, self.dst, self.key, self.start, self.lst, o[0], o[1],
                            self.ws, visc=o[2], nbr=o[3], flags=flags)
        return o

    def predictor_and_refresh(self, scale=1.0):
        """dt from the last pass, the predictor (its displacement recorded),
        then the view of the half state on the binning's cells; scale > 1
        moves the particles further (dt times scale)."""
        S.sph_reduce_dt(self.P, self.n, self.dt, self.ws)
        self.dt *= scale
        S.sph_symplectic_step(self.P, self.n, 0, self.dt, self.t, self.saved, self.dst,
                              torch.zeros((self.dim, self.n), dtype=torch.float32, device=DEV),
                              torch.zeros(self.n, dtype=torch.float32, device=DEV), self.ws)
        S.sph_refresh_view(self.P, self.n, self.dst, self.key, self.ws)


def _equal(a, b, what):
    names = ("ace", "arho", "visc", "nbr")
    for x, y, nm in zip(a, b, names):
        torch.cuda.synchronize()
        assert torch.isfinite(x.float()).all() if nm != "nbr" else True, (what, nm)
        assert torch.equal(x, y), (what, nm, (x.double() - y.double()).abs().max().item())


CASES = {
    "3d_block": lambda: _perturbed(cases.block_case(3, (19, 15, 13), walls=True, seed=3,
                                                    cell_div=2, x_sub=4), 7),
    "2d_dam": lambda: _perturbed(cases.dam_break_2d(dp=0.01, cell_div=2, x_sub=4), 8),
    "3d_cd1": lambda: _perturbed(cases.block_case(3, (15, 13, 11), walls=True, seed=4,
                                                  cell_div=1), 9),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("diag", [False, True])
def test_replay_equals_walk_at_state_n(name, diag):
    c = CASES[name]()
    s = Setup(c)
    s.bin()
    s.build(0.02 * c.params.h)
    assert s.walk_marked() == 0  # every target replays (cells of 2h too)
    fl = S.SPH_DIAG_COUNT_F64 if diag else 0
    _equal(s.replay(fl), s.walk(fl), f"{name} state n")
    assert S.sph_read_error(s.ws) == 0


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("scale,expect_walk", [(1.0, False), (40.0, True)])
def test_replay_equals_walk_on_reused_cells(name, scale, expect_walk):
    """After a predictor: the replay with SPH_INTERACT_REUSE_CELLS equals the
    reused-cells walk; with the step scaled so that twice the displacement
    exceeds the skin, the pass walks (counted), with the same results."""
    c = CASES[name]()
    s = Setup(c)
    s.bin()
    s.build(0.02 * c.params.h)
    s.walk(0)  # the pass at n sets the block maxima for dt
    s.predictor_and_refresh(scale)
    w0 = S.sph_list_walks(s.ws)
    fl = S.SPH_INTERACT_REUSE_CELLS | S.SPH_DIAG_COUNT_F64
    _equal(s.replay(fl), s.walk(fl), f"{name} n+1/2 x{scale}")
    walked = S.sph_list_walks(s.ws) - w0
    _say(f"  {name} scale {scale}: list walks {walked}")
    assert walked == (1 if expect_walk else 0)
    assert S.sph_read_error(s.ws) & ~S.SPH_ERR_EXCLUDED == 0


@pytest.mark.parametrize("n", [0, 1])
def test_empty_and_single(n):
    """No particle, and one fluid particle (its list is empty: a target is
    not its own candidate): build and replay succeed and equal the walk."""
    base = cases.dam_break_2d(dp=0.02)
    c = cases.Case(base.params, base.pos[:, :n].copy(), base.vel[:, :n].copy(),
                   base.rho[:n].copy(), base.type[:n].copy())
    s = Setup(c)
    s.bin()
    s.build(0.02 * c.params.h)
    r, w = s.replay(0), s.walk(0)
    _equal(r, w, f"n={n}")
    if n == 1:
        assert torch.allclose(r[0][:, 0].cpu(), torch.tensor(base.params.gravity[:2],
                                                              dtype=torch.float32))
        assert r[1][0].item() == 0 and r[3][0].item() == 0
    assert S.sph_read_error(s.ws) == 0


def test_small_buffer_targets_walk():
    """A list buffer with room for 2 chunks per target: most targets do not
    fit and walk their cells, any others replay; the results equal the walk's."""
    c = CASES["3d_block"]()
    P = S.make_params(c.params)
    n = c.n
    full = S.sph_list_bytes(P, n)
    header_and_counts = 256 + (4 * n + 255) // 256 * 256
    assert full == header_and_counts + 8 * n * 40
    s = Setup(c, list_bytes=header_and_counts + 8 * n * 2)
    s.bin()
    s.build(0.02 * c.params.h)
    marked = s.walk_marked()
    _say(f"  cap 2: {marked} of {n} targets walk")
    assert marked > 0
    _equal(s.replay(0), s.walk(0), "cap 2")


def test_stale_list_walks_and_reports():
    c = CASES["3d_block"]()
    s = Setup(c)
    s.bin()
    s.build(0.02 * c.params.h)
    s.bin()  # a new binning: the list belongs to the previous one
    _equal(s.replay(0), s.walk(0), "stale list")
    assert S.sph_read_error(s.ws) & S.SPH_ERR_LIST


def test_other_list_bytes_walks_and_reports():
    """A replay given another list_bytes than the build (another capacity)
    does not use the list: it walks, with the walk's results, and reports."""
    c = CASES["3d_block"]()
    s = Setup(c)
    s.bin()
    s.build(0.02 * c.params.h)
    full = s.lst
    s.lst = full[: full.numel() - 8 * c.n]  # one chunk per target less
    _equal(s.replay(0), s.walk(0), "other list_bytes")
    assert S.sph_read_error(s.ws) & S.SPH_ERR_LIST


@pytest.mark.parametrize("skin_h,expect_walk", [(0.05, False), (0.01, True)])
def test_1m_both_passes_equal_walk(skin_h, expect_walk):
    """The 3-D dam break at 1.32M particles in the benchmark's configuration,
    with the velocities of a developed flow (predictor displacement about
    0.012 h): both passes of a step equal the walk's, replayed from the list
    with a skin of 0.05 h, and walked (counted) with a skin of 0.01 h."""
    c = _perturbed(cases.dam_break_3d(cell_div=2, x_sub=4), 11, vel=2.0)
    s = Setup(c)
    s.bin()
    s.build(skin_h * c.params.h)
    assert s.walk_marked() == 0
    _equal(s.replay(0), s.walk(0), "1m state n")
    s.predictor_and_refresh(1.0)
    w0 = S.sph_list_walks(s.ws)
    fl = S.SPH_INTERACT_REUSE_CELLS
    _equal(s.replay(fl), s.walk(fl), "1m n+1/2")
    walked = S.sph_list_walks(s.ws) - w0
    _say(f"  1M, skin {skin_h} h: list walks {walked}")
    assert walked == (1 if expect_walk else 0)


def test_runner_trajectory_with_lists_equals_walk():
    """Ten symplectic steps with neighbour lists (adaptive skin) give the same
    trajectory bit for bit as the reused-cells walk (one lane per target)."""
    c = _perturbed(cases.dam_break_3d(dp=0.6 / 60, cell_div=2, x_sub=4), 12, vel=1.0)
    assert c.n > 131072
    a = Simulation(c, DEV, neighbour_list=True)
    b = Simulation(c, DEV, neighbour_list=False, flags=ONE)
    for _ in range(10):
        a.step()
        b.step()
    torch.cuda.synchronize()
    assert a.error() == 0 and b.error() == 0
    sa, sb = a.host_state(), b.host_state()
    for k in ("pos", "vel", "rho"):
        assert np.array_equal(sa[k], sb[k]), k
    assert a.interaction_count() == b.interaction_count()
    _say(f"  runner: list walks {S.sph_list_walks(a.ws)} of 10 steps")


def test_list_step_graph_replay_equals_eager():
    """Steps with lists captured in a HIP graph (two steps, the buffers
    alternate) and replayed three times with eager work between: the same
    state bit for bit as the eager run."""
    c = _perturbed(cases.dam_break_2d(dp=0.015, cell_div=2, x_sub=4), 21, vel=0.3)
    a = Simulation(c, DEV, neighbour_list=True)
    b = Simulation(c, DEV, neighbour_list=True)
    a.run(2 + 3 * 2)
    b.run(2)
    b.capture(2)
    for _ in range(3):
        b.replay(1)
        torch.cuda.synchronize()
        _ = b.state.rho.sum().item()  # eager work between replays
    torch.cuda.synchronize()
    assert a.error() == 0 and b.error() == 0
    sa, sb = a.host_state(), b.host_state()
    for k in ("pos", "vel", "rho", "type"):
        assert np.array_equal(sa[k], sb[k]), k
    assert sa["t"] == sb["t"]
