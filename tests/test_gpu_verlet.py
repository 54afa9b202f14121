"""The Verlet integrator (Section 2.5.1, Eq. 30-31) on the GPU against the
CPU oracle, through the C ABI.

Bars (as for the symplectic step): one step within the 1e-4 rate tolerance
times dt (times 2 for the doubled step of Eq. 30) plus FP32 storage of v and
rho; a 2-D dam-break run's front within 1e-3 of the tank length of the
oracle's; graph replay bit-identical to eager steps."""
import numpy as np
import pytest
import torch

import oracle
from paper_2104_00537_amd import cases

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
if torch.cuda.is_available():
    from paper_2104_00537_amd.runner import Simulation
    from test_gpu_parity import _perturbed, _say


def _host(sim):
    """Current state and the carried previous (v, rho), in input order."""
    st, pv = sim.state, sim.saved[0]
    ids = st.id.cpu().numpy().view(np.uint32).astype(np.int64)
    inv = np.empty_like(ids)
    inv[ids] = np.arange(ids.shape[0])
    return (st.pos.cpu().numpy()[:, inv], st.vel.cpu().numpy()[:, inv],
            st.rho.cpu().numpy()[inv], st.type.cpu().numpy()[inv],
            pv.vel.cpu().numpy()[:, inv], pv.rho.cpu().numpy()[inv])


@pytest.mark.parametrize("maker", ["dam2d", "slosh3d"])
def test_verlet_steps_match_oracle(maker):
    """Step 1 (Eq. 31) and step 2 (Eq. 30) each against the oracle's update
    from the GPU's state before the step, with the GPU's dt."""
    if maker == "dam2d":
        c = _perturbed(cases.dam_break_2d(cell_div=2, x_sub=4), 13, vel=0.5)
    else:
        c = _perturbed(cases.sloshing_3d(dp=0.04, seed=1, cell_div=2, x_sub=4), 14, vel=0.2)
    cp = c.params
    sim = Simulation(c, DEV, integrator="verlet", verlet_ns=40)
    sim.t.fill_(0.3)
    before = (c.pos, c.vel.astype(np.float64), c.rho.astype(np.float64), c.type,
              np.zeros_like(c.vel, dtype=np.float64), np.zeros_like(c.rho, dtype=np.float64))
    for k, mode in enumerate((1, 0)):
        t0 = sim.time()
        sim.step()
        torch.cuda.synchronize()
        assert sim.error() == 0
        dt = sim.dt.item()
        pos, vel, rho, typ, vp, rp = before
        ace, arho, _, _ = oracle.interact(cp, pos, vel, rho, typ)
        (pos_o, vel_o, rho_o), (vp_o, rp_o) = oracle.verlet(cp, dt, t0, mode, pos, vel, rho, vp,
                                                            rp, typ, ace, arho)
        g = _host(sim)
        f = 2.0 if mode == 0 else 1.0
        amax, rmax = np.abs(ace).max(), np.abs(arho).max()
        tol_v = 2e-4 * amax * dt * f + 2 * 6e-8 * np.abs(vel_o).max()
        tol_r = 2e-4 * rmax * dt * f + 2.5e-4
        tol_x = 0.5 * dt * dt * 2e-4 * amax + 1e-12
        ev = np.abs(g[1] - vel_o).max()
        er = np.abs(g[2] - rho_o).max()
        ex = np.abs(g[0] - pos_o).max()
        _say(f"  {maker} step {k + 1} mode {mode}: dv {ev:.2e} ({tol_v:.2e}) "
             f"drho {er:.2e} ({tol_r:.2e}) dx {ex:.2e} ({tol_x:.2e})")
        assert ev <= tol_v and er <= tol_r and ex <= tol_x
        # the carried previous state is exactly the state before the step
        assert np.array_equal(g[4], before[1].astype(np.float32))
        assert np.array_equal(g[5], before[2].astype(np.float32))
        before = (g[0], g[1].astype(np.float64), g[2].astype(np.float64), g[3],
                  g[4].astype(np.float64), g[5].astype(np.float64))


def test_verlet_2d_front_against_oracle():
    """The small 2-D dam break, 400 Verlet steps (Eq. 31 every 40): the
    front stays within 1e-3 of the tank length of the oracle's."""
    c = cases.dam_break_2d(cell_div=2, x_sub=4)
    sim = Simulation(c, DEV, integrator="verlet", verlet_ns=40)
    out = dict(pos=c.pos, vel=c.vel, rho=c.rho, type=c.type, t=0.0)
    fg, fo = [], []
    for k in range(4):
        sim.run(100)
        st = sim.host_state()
        fg.append(st["pos"][0][st["type"] == 0].max())
    assert sim.error() == 0
    out = oracle.run_verlet(c.params, c.pos, c.vel, c.rho, c.type, 400, ns=40)
    assert out["status"] == 0
    fo = out["pos"][0][out["type"] == 0].max()
    _say(f"  fronts gpu {np.round(fg, 5)}; oracle after 400 steps {fo:.5f}")
    assert abs(fg[-1] - fo) < 1e-3 * 1.6
    assert st["t"] == pytest.approx(out["t"], rel=1e-4)


def test_verlet_graph_replay_is_bit_identical():
    c = _perturbed(cases.dam_break_2d(dp=0.015, cell_div=2, x_sub=4), 22, vel=0.3)
    a = Simulation(c, DEV, integrator="verlet", verlet_ns=4)
    b = Simulation(c, DEV, integrator="verlet", verlet_ns=4)
    a.run(24)
    b.run(8)
    b.capture(8)
    for _ in range(2):
        b.replay(1)
        torch.cuda.synchronize()
        _ = b.state.rho.sum().item()   # eager work between replays
    torch.cuda.synchronize()
    sa, sb = a.host_state(), b.host_state()
    for k in ("pos", "vel", "rho", "type"):
        assert np.array_equal(sa[k], sb[k]), k
    assert sa["t"] == sb["t"]
