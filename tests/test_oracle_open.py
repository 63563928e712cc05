"""Pins of the oracle's open top boundary (the outflow condition of the paper's open-top problems,
Sections 4.2 and 4.3, read as the convective outflow condition of Lou et al.):

  * a uniform liquid at rest under an open top stays exactly at rest (the entering populations
    keep their equilibrium values when U = 0);
  * mass bookkeeping, every step: the change of total mass equals what enters the top row from
    outside minus the post-collision populations that leave it, to rounding (nothing else leaks,
    the bottom wall and the periodic sides stay closed);
  * a pressure pulse leaves through the open top: the wave that comes back is a small fraction of
    the one a wall sends back;
  * the thermal Dirichlet top (T_top) still holds: steady conduction between the heated bottom
    wall and the open top is exactly linear.
"""
import numpy as np
import pytest

from workloads import FREEZE_FLOW, Params, heated_droplet


def test_open_top_keeps_a_fluid_at_rest(orc, sat):
    Tc, T0, rl, rg, _ = sat
    nx, ny = 12, 20
    p = Params(nx=nx, ny=ny, y_walls=1, open_top=1, T_bot=T0, T_top=T0)
    rho = np.full((ny, nx), rl)
    o = orc.Oracle(p).init(rho, 0 * rho, 0 * rho, np.full((ny, nx), T0))
    o.step(300)
    r, ux, uy, T = o.fields()
    assert np.abs(r - rl).max() <= 1e-12 * rl
    assert max(np.abs(ux).max(), np.abs(uy).max()) <= 1e-14
    assert np.abs(T - T0).max() <= 1e-13


def test_open_top_mass_bookkeeping(orc, sat):
    Tc, T0, rl, rg, _ = sat
    w = heated_droplet(Tc, rl, rg, nx=80, ny=48, R=14.0, T_h_rel=0.95)
    o = orc.Oracle(w.params).init(w.rho, w.ux, w.uy, w.T)
    o.step(40)
    ny = w.params.ny
    down = [4, 7, 8]  # c_y = -1
    up = [2, 5, 6]    # c_y = +1
    moved = 0.0
    for _ in range(6):
        m0 = o.state()[0].sum()
        o.step(1)
        fn = o.state()[0]
        fs = o.post_collision()
        inflow = fn[down, ny - 1, :].sum()
        outflow = fs[up, ny - 1, :].sum()
        assert fn.sum() - m0 == pytest.approx(inflow - outflow, abs=1e-12 * m0)
        moved += abs(inflow - outflow)
    assert moved > 1e-10  # the boundary really exchanges mass in this case


def _pulse_reflection(orc, T0, rl, open_top, nx=4, ny=400, y0=300, probe=340, width=5.0):
    """Liquid column, periodic in x, wall at the bottom, Gaussian density bump at y0 near the top.
    Its upward half passes the probe (about step 50), meets the top at ny - 1/2 and what comes back
    passes the probe again (about step 200 with a wall on top); the downward half cannot return
    from the bottom wall before step y0 + probe = 640, since nothing moves faster than one node
    per step.  Returns the peak density deviation at the probe over steps [120, 500) divided by
    the one over steps [0, 100)."""
    p = Params(nx=nx, ny=ny, y_walls=1, open_top=open_top, T_bot=T0, T_top=T0)
    y = np.arange(ny)[:, None] * np.ones((1, nx))
    rho = rl * (1 + 1e-4 * np.exp(-((y - y0) ** 2) / (2 * width ** 2)))
    o = orc.Oracle(p).init(rho, 0 * rho, 0 * rho, np.full((ny, nx), T0))
    sig = []
    for _ in range(500):
        o.step(1)
        sig.append(abs(o.fields()[0][probe, 0] - rl))
    sig = np.array(sig)
    return sig[120:].max() / sig[:100].max()


def test_open_top_lets_a_pressure_pulse_out(orc, sat):
    Tc, T0, rl, rg, _ = sat
    wall = _pulse_reflection(orc, T0, rl, 0)
    open_ = _pulse_reflection(orc, T0, rl, 1)
    print(f"reflected / incident at the probe: wall {wall:.3f}, open top {open_:.3f}")
    assert wall > 0.5  # a wall sends the pulse back (viscous damping aside)
    assert open_ < 0.2 * wall


def test_open_top_dirichlet_temperature_conduction(orc, sat):
    T0 = sat[1]
    nx, ny = 4, 12
    Tb, Tt = 1.03 * T0, 0.98 * T0
    p = Params(nx=nx, ny=ny, y_walls=1, open_top=1, T_bot=Tb, T_top=Tt, flags=FREEZE_FLOW)
    rho = np.full((ny, nx), 0.2)
    o = orc.Oracle(p).init(rho, 0 * rho, 0 * rho, np.full((ny, nx), T0))
    o.step(6000)
    T = o.fields()[3]
    y = np.arange(ny)[:, None]
    assert np.allclose(T, Tb + (Tt - Tb) * (y + 0.5) / ny, rtol=0, atol=1e-12)


def test_open_top_buoyancy_follows_the_current_mean_density(orc, sat):
    """Section 4.3 takes rho_ave of F_b = (rho - rho_ave) g as the mean density of the whole
    domain.  Under an open top mass leaves, so that mean moves: at every step the oracle's rho_ave
    must equal the mean of the density field it reads out at that step, and the buoyancy then adds
    no net force to the domain (sum of (rho - rho_ave) g = 0 to rounding), although the mass has
    changed by far more than rounding (so a rho_ave frozen at its initial value would leave a net
    force of (M(t) - M(0)) g, checked below to be large)."""
    from workloads import boiling
    Tc, T0, rl, rg, _ = sat
    w = boiling(Tc, rl, rg, nx=64, ny=48, hot_width=6.0, dT_rel=0.2, gravity=1e-4, seed=4, fill=0.6, open_top=1)
    o = orc.Oracle(w.params).init(w.rho, w.ux, w.uy, w.T)
    g = abs(w.params.gy)
    m0 = float(w.rho.sum())
    worst = 0.0
    for _ in range(40):
        o.step(10)
        rho = o.fields()[0]
        mean = float(rho.sum()) / rho.size
        assert o.rho_ave == pytest.approx(mean, rel=1e-14)
        worst = max(worst, abs(float((rho - o.rho_ave).sum())) * g)
    drained = abs(float(rho.sum()) - m0)
    print(f"mass change {drained / m0:.2e} (relative); net buoyancy with the current mean {worst:.2e}, "
          f"with the initial mean {drained * g:.2e}")
    assert drained > 1e-4 * m0
    assert worst <= 1e-13 * m0 * g
    assert drained * g > 1e6 * worst
