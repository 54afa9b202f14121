"""The batched path (continuous batching) on the GPU: per-case results are
bit-identical alone and in a mix, agree with the single-case path and with
the oracle, and a small request stream is served end to end.  Steps bin once
(the n+1/2 interaction reuses each slot's cells, widened by the slot's own
recorded displacement) or twice; a slot that moved half a cell or more gets
SPH_ERR_MARGIN in its own error word only."""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
from paper_2104_00537_amd import cases

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2104_00537_amd import serve as V
    from paper_2104_00537_amd import sph as S
    from paper_2104_00537_amd.runner import Simulation

DEV = "cuda:0"


def _say(*a):
    print(*a, flush=True)


def _mix_cases():
    rng = np.random.default_rng(5)
    out = [cases.dam_break_2d(dp=0.02, seed=1),
           cases.block_case(3, (12, 10, 9), walls=True, seed=2),
           cases.sloshing_3d(dp=0.06, seed=3),
           cases.dam_break_3d(dp=0.03, seed=4)]
    for c in out:
        c.vel[:] = rng.uniform(-0.2, 0.2, c.vel.shape).astype(np.float32)
    return out


def _options_mix():
    """The mix with formulation options per slot: cubic spline kernel,
    laminar viscosity, Fourtakas DDT, and one slot of the default
    formulation."""
    rng = np.random.default_rng(6)
    base = [cases.dam_break_2d(dp=0.02, seed=1),
            cases.block_case(3, (12, 10, 9), walls=True, seed=2),
            cases.dam_break_3d(dp=0.03, seed=4),
            cases.sloshing_3d(dp=0.06, seed=3)]
    opts = [dict(kernel=1), dict(viscosity=1, visc_nu=1e-2), dict(ddt=2), {}]
    out = []
    for c, kw in zip(base, opts):
        c.vel[:] = rng.uniform(-0.2, 0.2, c.vel.shape).astype(np.float32)
        out.append(cases.Case(dataclasses.replace(c.params, **kw), c.pos, c.vel, c.rho, c.type,
                              dict(c.meta), c.normal))
    return out


def _periodic_mix(shift=False):
    """Slots with periodic components (a 2-D channel periodic along x, a
    2-D column periodic along its vertical, a 3-D box periodic along x and
    y) beside a slot without any; shift: with particle shifting."""
    rng = np.random.default_rng(9)
    base = [cases.periodic_box(2, shape=(60, 14), periodic=(0,), seed=1),
            cases.periodic_box(2, shape=(14, 30), periodic=(1,), seed=2),
            cases.periodic_box(3, shape=(24, 20, 10), periodic=(0, 1), seed=3),
            cases.dam_break_2d(dp=0.02, seed=4)]
    out = []
    for c in base:
        c.vel[:] = rng.uniform(-0.3, 0.3, c.vel.shape).astype(np.float32)
        kw = dict(shift_coef=2.0) if shift else {}
        out.append(cases.Case(dataclasses.replace(c.params, **kw), c.pos, c.vel, c.rho, c.type,
                              dict(c.meta), c.normal))
    return out


MIXES = {"default": _mix_cases, "options": _options_mix, "periodic": _periodic_mix}


def _engine(cs, graph=False, reuse=True, pad=True, four=False):
    return V.BatchEngine(cap_particles=sum(V.padded(c.n) for c in cs) + 16,
                         cap_cells=sum(c.params.ncell_total() + 1 for c in cs) + 16,
                         max_slots=8, device=DEV, use_graph=graph, reuse_cells=reuse,
                         pad_slots=pad, four_lanes=four)


def _run_engine(cs, steps, graph, reuse=True, pad=True, four=False):
    eng = _engine(cs, graph, reuse, pad, four)
    reqs = [V.Request(rid=k, case=c, steps=steps, arrival=0.0) for k, c in enumerate(cs)]
    eng.repack([], reqs)
    eng.run(steps)
    torch.cuda.synchronize()
    errs = S.sph_batch_read_errors(eng.batch, eng.ws)
    return [eng.slot_result(k) for k in range(len(cs))], errs, eng


@pytest.mark.parametrize("reuse,pad,four,mixname", [
    (True, True, False, "default"), (False, True, False, "default"),
    (True, False, False, "default"), (True, True, True, "default"),
    (True, True, False, "options"), (True, False, False, "options"),
    (True, True, False, "periodic"), (False, True, False, "periodic"),
    (True, True, True, "periodic")])
def test_batch_alone_vs_mix_bit_identical(reuse, pad, four, mixname):
    """pad: slots padded to whole wavefronts (the aligned kernel) or not (the
    unaligned kernel, wavefronts straddling slots); four: four lanes per
    target for the small slots (all of these).  In the options mix every
    slot runs the general pair terms, and alone the default slot runs the
    default kernel: the same bits either way."""
    cs = MIXES[mixname]()
    _say("mix of", [c.n for c in cs])
    mix, errs, eng = _run_engine(cs, 7, graph=True, reuse=reuse, pad=pad, four=four)
    assert not errs.any()
    assert bool(eng.batch.flags & S.SPH_BATCH_WAVE_ALIGNED) == pad
    assert bool(eng.batch.flags & S.SPH_BATCH_FOUR_LANES) == four
    assert bool(eng.batch.flags & S.SPH_BATCH_GENERAL) == (mixname == "options")
    assert bool(eng.batch.flags & S.SPH_BATCH_PERIODIC) == (mixname == "periodic")
    for k, c in enumerate(cs):
        alone, e1, _ = _run_engine([c], 7, graph=False, reuse=reuse, pad=pad, four=four)
        assert not e1.any()
        for f in ("pos", "vel", "rho", "type"):
            assert np.array_equal(mix[k][f], alone[0][f]), (k, f)
        assert mix[k]["t"] == alone[0]["t"]


@pytest.mark.parametrize("reuse", [True, False])
def test_batch_matches_single_case_path(reuse):
    cs = _mix_cases()
    mix, errs, eng = _run_engine(cs, 4, graph=False, reuse=reuse)
    assert not errs.any()
    inter = eng.inter[: len(cs)].cpu().numpy()
    for k, c in enumerate(cs):
        sim = Simulation(c, DEV, reuse_cells=reuse)
        sim.run(4)
        g = sim.host_state()
        assert sim.error() == 0
        # pair counts of both passes of every step (FP32 tests: near-ties only)
        pairs = sim.interactions.cpu().numpy()
        assert abs(int(inter[k, 0]) - int(pairs[0])) <= 1e-4 * pairs[0] + 2, (inter[k], pairs)
        b = mix[k]
        assert b["t"] == pytest.approx(g["t"], rel=1e-6)
        scale = max(np.abs(g["vel"]).max(), 1e-3)
        dv = np.abs(b["vel"] - g["vel"]).max()
        dx = np.abs(b["pos"] - g["pos"]).max()
        dr = np.abs(b["rho"].astype(np.float64) - g["rho"]).max()
        _say(f"  slot {k} (dim {c.params.dim}): |dv| {dv:.2e} |dx| {dx:.2e} |drho| {dr:.2e}")
        assert dv <= 1e-4 * scale + 1e-6 and dx <= 1e-7 and dr <= 1e-2
        assert np.array_equal(b["type"], g["type"])


@pytest.mark.parametrize("pad,four,mixname", [(True, False, "default"), (False, False, "default"),
                                              (True, True, "default"), (True, False, "options"),
                                              (False, False, "options"), (True, True, "options"),
                                              (True, False, "periodic"),
                                              (False, False, "periodic")])
def test_batch_interaction_matches_oracle(pad, four, mixname):
    cs = MIXES[mixname]()
    eng = _engine(cs, pad=pad, four=four)
    reqs = [V.Request(rid=k, case=c, steps=1, arrival=0.0) for k, c in enumerate(cs)]
    eng.repack([], reqs)
    b = eng.batch
    n = b.n_total
    a, bb = eng._dev_state(eng.cur, n), eng._dev_state(1 - eng.cur, n)
    key, perm = eng._key.view(n), eng._perm.view(n)
    ace, arho = eng._ace.view(n), eng._arho.view(n)
    nbr = torch.zeros(n, dtype=torch.int32, device=DEV)
    S.sph_batch_bin_cells(b, a, bb, key, perm, eng.cell_start, eng.ws)
    S.sph_batch_interact(b, bb, key, eng.cell_start, ace, arho, eng.ws, nbr=nbr)
    torch.cuda.synchronize()
    pos_all = bb.pos.cpu().numpy()
    vel_all = bb.vel.cpu().numpy().astype(np.float64)
    rho_all = bb.rho.cpu().numpy().astype(np.float64)
    typ_all = bb.type.cpu().numpy()
    ace_all = ace.cpu().numpy().astype(np.float64)
    arho_all = arho.cpu().numpy().astype(np.float64)
    nbr_all = nbr.cpu().numpy().astype(np.int64)
    for k, c in enumerate(cs):
        o0, o1 = eng.offsets[k], eng.offsets[k + 1]
        pos, vel = V.from_3d(c.params.dim, pos_all[:, o0:o1], vel_all[:, o0:o1])
        typ = typ_all[o0:o1]
        ace_o, arho_o, _, nbr_o = oracle.interact(c.params, pos, vel, rho_all[o0:o1], typ)
        ace_g = ace_all[:, o0:o1] if c.params.dim == 3 else ace_all[[0, 2], o0:o1]
        fl = typ == cases.FLUID
        ea = np.abs(ace_g - ace_o)[:, fl].max() / np.abs(ace_o[:, fl]).max()
        er = np.abs(arho_all[o0:o1] - arho_o).max() / np.abs(arho_o).max()
        flips = np.abs(nbr_all[o0:o1] - nbr_o.astype(np.int64)).sum()
        _say(f"  slot {k}: rel err ace {ea:.2e} arho {er:.2e} count flips {flips}")
        assert ea < 1e-4 and er < 1e-4 and flips <= 5e-4 * nbr_o.sum() + 2


class BatchHalfStep:
    """Bin and interact the mix at state n, then the batched predictor with a
    per-slot dt that moves each slot's particles by up to the given fraction
    of its cell (zero rates: a pure move), leaving the half state in `st`."""

    def __init__(self, cs, move_cells):
        eng = self.eng = _engine(cs)
        eng.repack([], [V.Request(rid=k, case=c, steps=1, arrival=0.0)
                        for k, c in enumerate(cs)])
        b = self.b = eng.batch
        n = self.n = b.n_total
        a, self.st = eng._dev_state(eng.cur, n), eng._dev_state(1 - eng.cur, n)
        self.saved = eng._dev_saved(0, n)
        self.key, perm = eng._key.view(n), eng._perm.view(n)
        ace, arho = eng._ace.view(n), eng._arho.view(n)
        S.sph_batch_bin_cells(b, a, self.st, self.key, perm, eng.cell_start, eng.ws)
        S.sph_batch_interact(b, self.st, self.key, eng.cell_start, ace, arho, eng.ws)
        dts = []
        for c, m in zip(cs, move_cells):
            fl = c.type == cases.FLUID  # walls are not moved by their stored velocity
            vmax = float(np.sqrt((c.vel[:, fl].astype(np.float64) ** 2).sum(axis=0)).max())
            dts.append(2.0 * m * c.params.cell_size / vmax)  # the predictor moves dt/2 v
        dt = torch.tensor(dts, dtype=torch.float64, device=DEV)
        t = torch.zeros(len(cs), dtype=torch.float64, device=DEV)
        ace.zero_()
        arho.zero_()
        S.sph_batch_symplectic_step(b, 0, dt, t, self.saved, self.st, ace, arho, eng.ws)
        torch.cuda.synchronize()


@pytest.mark.parametrize("mixname", ["default", "periodic"])
@pytest.mark.parametrize("move", [0.05, 0.3])
def test_batch_reused_cells_find_the_oracles_pairs(move, mixname):
    """The n+1/2 interaction on the cells of state n, per slot against the
    oracle on the half state: rates to the interaction's bar, FP32 neighbour
    counts with flips only at near-ties (periodic slots: pairs across their
    periodic boundaries, particles moved past them not yet wrapped)."""
    cs = MIXES[mixname]()
    hs = BatchHalfStep(cs, [move] * len(cs))
    eng, b, n = hs.eng, hs.b, hs.n
    S.sph_batch_refresh_view(b, hs.st, hs.key, eng.ws)
    ace = torch.full((3, n), float("nan"), dtype=torch.float32, device=DEV)
    arho = torch.full((n,), float("nan"), dtype=torch.float32, device=DEV)
    nbr = torch.full((n,), -1, dtype=torch.int32, device=DEV)
    S.sph_batch_interact(b, hs.st, hs.key, eng.cell_start, ace, arho, eng.ws, nbr=nbr,
                         flags=S.SPH_INTERACT_REUSE_CELLS)
    inter = torch.zeros((len(cs), 2), dtype=torch.int64, device=DEV)
    dth = torch.zeros(len(cs), dtype=torch.float64, device=DEV)
    S.sph_batch_reduce_dt(b, dth, eng.ws, interactions=inter)
    torch.cuda.synchronize()
    errs = S.sph_batch_read_errors(b, eng.ws)
    assert not errs.any(), errs
    inter = inter.cpu().numpy()
    pos_all = hs.st.pos.cpu().numpy()
    vel_all = hs.st.vel.cpu().numpy().astype(np.float64)
    rho_all = hs.st.rho.cpu().numpy().astype(np.float64)
    typ_all = hs.st.type.cpu().numpy()
    moved_all = np.sqrt(((pos_all - hs.saved.pos.cpu().numpy()) ** 2).sum(axis=0))
    ace_all = ace.cpu().numpy().astype(np.float64)
    arho_all = arho.cpu().numpy().astype(np.float64)
    nbr_all = nbr.cpu().numpy().astype(np.int64)
    for k, c in enumerate(cs):
        o0, o1 = eng.offsets[k], eng.offsets[k + 1]
        pos, vel = V.from_3d(c.params.dim, pos_all[:, o0:o1], vel_all[:, o0:o1])
        typ = typ_all[o0:o1]
        ace_o, arho_o, _, nbr_o = oracle.interact(c.params, pos, vel, rho_all[o0:o1], typ)
        ace_g = ace_all[:, o0:o1] if c.params.dim == 3 else ace_all[[0, 2], o0:o1]
        fl = typ == cases.FLUID
        ea = np.abs(ace_g - ace_o)[:, fl].max() / np.abs(ace_o[:, fl]).max()
        er = np.abs(arho_all[o0:o1] - arho_o).max() / np.abs(arho_o).max()
        flips = np.abs(nbr_all[o0:o1] - nbr_o.astype(np.int64)).sum()
        mv = moved_all[o0:o1].max() / c.params.cell_size
        _say(f"  slot {k} moved {mv:.3f} cell: rel err ace {ea:.2e} arho {er:.2e} "
             f"count flips {flips}")
        assert mv > 0.99 * move
        # the slot's pair count is this pass's alone (the refresh restarts it)
        assert inter[k, 0] == nbr_all[o0:o1].sum()
        assert ea < 1e-4 and er < 1e-4 and flips <= 5e-4 * nbr_o.sum() + 2


def test_batch_margin_error_is_per_slot():
    """Slot 1 moves 0.6 of a cell before the n+1/2 interaction on reused
    cells: its error word gets SPH_ERR_MARGIN, the other slots' words stay
    clear (their own records are below the margin)."""
    cs = _mix_cases()
    hs = BatchHalfStep(cs, [0.1, 0.6, 0.1, 0.1])
    eng, b, n = hs.eng, hs.b, hs.n
    S.sph_batch_refresh_view(b, hs.st, hs.key, eng.ws)
    S.sph_batch_interact(b, hs.st, hs.key, eng.cell_start, eng._ace.view(n),
                         eng._arho.view(n), eng.ws, flags=S.SPH_INTERACT_REUSE_CELLS)
    errs = S.sph_batch_read_errors(b, eng.ws)
    _say(f"  per-slot error words: {list(errs)}")
    assert errs[1] & S.SPH_ERR_MARGIN
    for k in (0, 2, 3):
        assert not (errs[k] & S.SPH_ERR_MARGIN)
    assert S.sph_read_error(eng.ws) & S.SPH_ERR_MARGIN


def test_engine_capacity_counts_the_padding():
    """Slots are padded to whole wavefronts: a case that fits the particle
    capacity only unpadded is refused with a clear error (before any copy),
    and admission (fits) counts the padded size."""
    c = cases.dam_break_2d(dp=0.02, seed=1)
    assert c.n % V.WAVE != 0
    eng = V.BatchEngine(cap_particles=c.n, cap_cells=c.params.ncell_total() + 16, max_slots=2,
                        device=DEV)
    req = V.Request(rid=0, case=c, steps=1, arrival=0.0)
    assert not eng.fits([], req)
    with pytest.raises(S.SphError, match="capacity"):
        eng.repack([], [req])
    eng2 = V.BatchEngine(cap_particles=V.padded(c.n), cap_cells=c.params.ncell_total() + 16,
                         max_slots=2, device=DEV)
    assert eng2.fits([], req)
    eng2.repack([], [req])
    eng2.run(2)
    torch.cuda.synchronize()
    assert not S.sph_batch_read_errors(eng2.batch, eng2.ws).any()
    r = eng2.slot_result(0)
    assert r["pos"].shape == c.pos.shape and np.all(r["type"] == c.type)


def test_served_stream_small():
    """A short stream through the batched and the plain path: every request
    completes without error and gets the same answer either way."""
    reqs = V.make_stream(6, rate=50.0, seed=3, n_min=800, n_max=6000, steps_min=5,
                         steps_max=20)
    eng = V.BatchEngine(cap_particles=200_000, cap_cells=2_000_000, max_slots=8, device=DEV)
    sb = V.serve_batched(reqs, eng, max_chunk=7, keep_results=True)
    res_b = {r.rid: r.result for r in reqs}
    assert sb["errors"] == 0 and all(r.finish is not None for r in reqs)
    reqs2 = V.make_stream(6, rate=50.0, seed=3, n_min=800, n_max=6000, steps_min=5,
                          steps_max=20)
    sp = V.serve_plain(reqs2, device=DEV, keep_results=True)
    assert sp["errors"] == 0
    for r in reqs2:
        a, b = res_b[r.rid], r.result
        assert a["t"] == pytest.approx(b["t"], rel=1e-6)
        assert np.abs(a["pos"] - b["pos"]).max() < 1e-6
    _say("  batched", {k: round(v, 4) for k, v in sb.items() if isinstance(v, float)})
    _say("  plain  ", {k: round(v, 4) for k, v in sp.items() if isinstance(v, float)})


def _shifting_mix():
    """Slots with particle shifting (A_s = 2; with and without the surface
    correction) beside a slot without it."""
    rng = np.random.default_rng(8)
    base = [(cases.dam_break_2d(dp=0.02, seed=1), dict(shift_coef=2.0, shift_fs=0.9)),
            (cases.block_case(3, (12, 10, 9), walls=True, seed=2), dict(shift_coef=2.0)),
            (cases.sloshing_3d(dp=0.06, seed=3), {}),
            (cases.dam_break_3d(dp=0.03, seed=4), dict(shift_coef=1.0, shift_fs=0.9,
                                                      kernel=1))]
    out = []
    for c, kw in base:
        c.vel[:] = rng.uniform(-0.3, 0.3, c.vel.shape).astype(np.float32)
        out.append(cases.Case(dataclasses.replace(c.params, **kw), c.pos, c.vel, c.rho, c.type,
                              dict(c.meta), c.normal))
    return out


@pytest.mark.parametrize("pad,mixname", [(True, "shift"), (False, "shift"),
                                         (True, "periodic")])
def test_batch_shifting_matches_oracle(pad, mixname):
    """sph_batch_shifting on a freshly binned batch against the oracle's
    shifting per slot (the single-case bars: C within 1e-5, the shift within
    1e-4 of the slot's largest on matching surface decisions); a slot
    without shifting is left as it is.  periodic: every slot shifted, three
    of them with periodic components."""
    cs = _shifting_mix() if mixname == "shift" else _periodic_mix(shift=True)
    eng = _engine(cs, pad=pad)
    eng.repack([], [V.Request(rid=k, case=c, steps=1, arrival=0.0) for k, c in enumerate(cs)])
    assert eng.shifting
    b = eng.batch
    n = b.n_total
    a, bb = eng._dev_state(eng.cur, n), eng._dev_state(1 - eng.cur, n)
    key, perm = eng._key.view(n), eng._perm.view(n)
    S.sph_batch_bin_cells(b, a, bb, key, perm, eng.cell_start, eng.ws)
    torch.cuda.synchronize()
    pos0 = bb.pos.cpu().numpy()
    vel_all = bb.vel.cpu().numpy().astype(np.float64)
    rho_all = bb.rho.cpu().numpy().astype(np.float64)
    typ_all = bb.type.cpu().numpy()
    dts = [2e-4, 1.5e-4, 1e-4, 2.5e-4][: len(cs)]
    dt = torch.tensor(dts, dtype=torch.float64, device=DEV)
    conc = torch.full((n,), float("nan"), dtype=torch.float32, device=DEV)
    shift = torch.full((3, n), float("nan"), dtype=torch.float32, device=DEV)
    S.sph_batch_shifting(b, bb, key, eng.cell_start, dt, eng.ws, conc=conc, shift=shift)
    torch.cuda.synchronize()
    assert not S.sph_batch_read_errors(b, eng.ws).any()
    pos1 = bb.pos.cpu().numpy()
    cg_all = conc.cpu().numpy().astype(np.float64)
    dg_all = shift.cpu().numpy().astype(np.float64)
    assert np.array_equal(pos1, pos0 + dg_all)
    for k, c in enumerate(cs):
        o0, o1 = eng.offsets[k], eng.offsets[k + 1]
        cp, dim = c.params, c.params.dim
        typ = typ_all[o0:o1]
        cg, dg = cg_all[o0:o1], dg_all[:, o0:o1]
        if not cp.shift_coef > 0:
            assert np.all(cg == 0) and np.all(dg == 0), k
            continue
        pos, vel = V.from_3d(dim, pos0[:, o0:o1], vel_all[:, o0:o1])
        co, _, do = oracle.shift(cp, pos, vel, rho_all[o0:o1], typ, dts[k])
        d3 = dg if dim == 3 else dg[[0, 2]]
        if dim == 2:
            assert np.all(dg[1] == 0)
        fl = typ == cases.FLUID
        same = (cg < cp.shift_fs) == (co < cp.shift_fs) if cp.shift_fs > 0 else np.ones_like(fl)
        ec = np.abs(cg - co).max()
        ed = np.abs(d3 - do)[:, fl & same].max() / np.abs(do[:, fl]).max()
        _say(f"  slot {k} (dim {dim}): C err {ec:.2e}, shift rel err {ed:.2e}, surface "
             f"decisions differing {(~same & fl).sum()}")
        assert ec < 1e-5 and ed < 1e-4
        assert (~same & fl).sum() <= max(2, fl.sum() // 1000)
        assert np.all(dg[:, ~fl] == 0)


@pytest.mark.parametrize("reuse", [True, False])
def test_batch_shifting_alone_vs_mix_bit_identical(reuse):
    """Steps with shifting in some slots: every case gives the same bits
    alone and in the mix."""
    cs = _shifting_mix()
    mix, errs, eng = _run_engine(cs, 6, graph=True, reuse=reuse)
    assert not errs.any() and eng.shifting
    for k, c in enumerate(cs):
        alone, e1, _ = _run_engine([c], 6, graph=False, reuse=reuse)
        assert not e1.any()
        for f in ("pos", "vel", "rho", "type"):
            assert np.array_equal(mix[k][f], alone[0][f]), (k, f)
        assert mix[k]["t"] == alone[0]["t"]


def test_batch_shifting_matches_single_case_path():
    """A case with shifting in the batch follows the single-case runner's
    trajectory (reused cells, shifting after each corrector) to FP32
    summation order."""
    cs = _shifting_mix()
    mix, errs, eng = _run_engine(cs, 4, graph=False)
    assert not errs.any()
    for k in (0, 1):
        c = cs[k]
        sim = Simulation(c, DEV)
        assert sim.shifting
        sim.run(4)
        g = sim.host_state()
        assert sim.error() == 0
        b = mix[k]
        scale = max(np.abs(g["vel"]).max(), 1e-3)
        dv = np.abs(b["vel"] - g["vel"]).max()
        dx = np.abs(b["pos"] - g["pos"]).max()
        _say(f"  slot {k}: |dv| {dv:.2e} |dx| {dx:.2e}")
        assert dv <= 1e-4 * scale + 1e-6 and dx <= 1e-7


@pytest.mark.parametrize("reuse", [True, False])
@pytest.mark.parametrize("mixname", ["default", "options", "periodic", "shift"])
def test_batch_equals_single_case_path_bit_for_bit(reuse, mixname):
    """With one lane per target on both sides, a case stepped in the batch
    (one slot of a mix, 2-D cases in the packed (x, 0, z) layout) and the
    same case stepped alone by the single-case runner
    (SPH_INTERACT_ONE_LANE) have the same state bit for bit: the same keys,
    stable order, view, pair terms in the same order, Δt, update and
    shifting."""
    cs = MIXES[mixname]() if mixname != "shift" else _shifting_mix()
    mix, errs, eng = _run_engine(cs, 5, graph=False, reuse=reuse)
    assert not errs.any()
    for k, c in enumerate(cs):
        sim = Simulation(c, DEV, reuse_cells=reuse, flags=S.SPH_INTERACT_ONE_LANE)
        sim.run(5)
        g = sim.host_state()
        assert sim.error() == 0
        b = mix[k]
        for f in ("pos", "vel", "rho", "type"):
            assert np.array_equal(b[f], g[f]), (k, f, np.abs(b[f].astype(np.float64)
                                                             - g[f]).max())
        assert b["t"] == g["t"], k
