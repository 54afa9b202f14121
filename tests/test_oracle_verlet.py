"""Pins of the oracle's Verlet integrator (Section 2.5.1, Eq. 30-31), on the
CPU, against what the scheme fixes exactly or physically."""
import numpy as np
import pytest

import oracle
from paper_2104_00537_amd import cases

G = 9.81


@pytest.mark.parametrize("ns", [1, 7, 40])
def test_verlet_free_fall_is_exact(ns):
    """A lone fluid particle under gravity: both update forms are exact for a
    constant acceleration (Eq. 30 steps over two intervals from the exact
    v^{n-1}; Eq. 31 and the position update are Taylor-exact), so any mix of
    them gives r = r0 + v0 t + g t^2/2 and v = v0 + g t."""
    cp = cases.dam_break_2d().params
    pos = np.array([[0.2], [0.3]])
    vel = np.array([[0.7], [1.1]])
    rho = np.array([1000.0])
    out = oracle.run_verlet(cp, pos, vel, rho, np.zeros(1, np.uint8), 150, ns=ns)
    t = out["t"]
    g = np.array(cp.gravity[:2])[:, None]
    assert out["status"] == 0 and np.all(out["dt"] == out["dt"][0])
    assert np.allclose(out["pos"], pos + vel * t + 0.5 * g * t * t, rtol=0, atol=1e-12)
    assert np.allclose(out["vel"], vel + g * t, rtol=0, atol=1e-12)


def test_verlet_density_follows_a_constant_rate_linearly():
    """With R held fixed, Eq. 30 (rho^{n-1} + 2 dt R) and Eq. 31
    (rho^n + dt R) both continue the exact line rho0 + R t, for fluid and
    wall particles alike."""
    cp = cases.block_case(2, (1, 1)).params
    n = 4
    rho0 = np.linspace(995.0, 1005.0, n)
    typ = np.array([0, 0, 1, 2], np.uint8)
    R = np.array([3.0, -2.0, 1.5, -0.5])
    dt = 1e-3
    pos, vel = np.zeros((2, n)), np.zeros((2, n))
    rho, vp, rp = rho0.copy(), vel.copy(), rho0.copy()
    for k in range(25):
        mode = 1 if k % 6 == 0 else 0
        (pos, vel, rho), (vp, rp) = oracle.verlet(cp, dt, k * dt, mode, pos, vel, rho, vp, rp,
                                                  typ, np.zeros((2, n)), R)
        assert np.allclose(rho, rho0 + R * (k + 1) * dt, rtol=0, atol=1e-11)


def test_verlet_walls_hold_still_and_moving_walls_follow_the_law():
    """Fixed walls keep position and (zero) velocity; moving walls take the
    imposed x_B(t + dt) and v_B(t + dt) of the motion law."""
    c = cases.sloshing_3d(dp=0.1, seed=0)
    cp = c.params
    n = c.n
    typ = c.type
    ace = np.ones((3, n))
    out, _ = oracle.verlet(cp, 0.01, 0.3, 1, c.pos, c.vel, c.rho, c.vel, c.rho, typ, ace,
                           np.zeros(n))
    w, A = cp.motion_omega, cp.motion_amp
    disp = lambda t: A / w ** 2 * (1 - np.cos(w * t))  # noqa: E731
    mv = typ == cases.BOUND_MOVING
    assert mv.any()
    assert np.allclose(out[0][0, mv], c.pos[0, mv] + disp(0.31) - disp(0.3), rtol=0, atol=1e-14)
    assert np.allclose(out[1][0, mv], A / w * np.sin(w * 0.31), rtol=0, atol=1e-14)
    assert np.array_equal(out[0][1:, mv], c.pos[1:, mv])


def test_verlet_hydrostatic_column_at_rest():
    """The 2-D column of the symplectic pin, advanced with Verlet (Eq. 31 every
    40 steps): after 0.5 s, pressure follows rho0 g (H - z) to within 5 % of
    rho0 g H away from the free surface and the walls."""
    width = 0.4
    c = cases.dam_break_2d(dp=0.02, tank=(width, 0.5), column=(width, 0.4), seed=1)
    cp = c.params
    steps = int(1.05 * 0.5 / (0.2 * cp.h / cp.c0)) + 1
    out = oracle.run_verlet(cp, c.pos, c.vel, c.rho, c.type, steps, ns=40)
    assert out["status"] == 0 and out["t"] > 0.5
    fl = out["type"] == cases.FLUID
    x, z = out["pos"]
    H = cp.fluid_height
    sel = fl & (z < H - 3 * cp.h) & (z > 2 * cp.h) & (x > 2 * cp.h) & (x < width - 2 * cp.h)
    assert sel.sum() > 100
    P = np.array([oracle.pressure(cp, r) for r in out["rho"][sel]])
    err = np.abs(P - cp.rho0 * G * (H - z[sel]))
    assert err.max() < 0.05 * cp.rho0 * G * H
    assert not np.any(out["type"] & cases.EXCLUDED)
    assert np.abs(out["vel"][:, fl]).max() < 0.05
