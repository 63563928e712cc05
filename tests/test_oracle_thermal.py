"""Pins of the oracle's thermal step (D2Q5 MRT with the rho c_v modified collision, Eqs. 20-26, 39-53).

All cases freeze the flow (populations f fixed, u = j/rho), so the temperature equation
rho c_v dT/dt = div(lambda grad T) - rho c_v u.grad T - T (dp/dT) div u (Eq. 20) can be
compared with closed forms:
  * Gaussian pulse diffusion with D = lambda/(rho c_v), for rho c_v = 1 and 5;
  * a sine mode advected by a uniform u: phase speed u, decay rate D_eff k^2, where a
    Chapman-Enskog expansion carried one order further than the paper's gives
    D_eff = D - rho c_v (tau_g - 1) u^2 with the correction S_i of Eq. (24) on and an extra
    -u^2/2 with it off (tau_g = 1/varsigma_1).  At tau_g = 1 the S term must cancel exactly u^2/2;
  * one step of compression heating by a frozen sinusoidal velocity (closed form);
  * steady conduction between two Dirichlet walls (exact linear profile);
  * relaxation of a box with Dirichlet edges to the edge temperature;
  * the discrete energy identity sum rho c_v (T^{t+1} - T^t) = sum (Q + S).
"""
import numpy as np
import pytest

from workloads import FREEZE_FLOW, NO_S, Params


def _frozen(orc, p, rho, ux, uy, T):
    return orc.Oracle(p.replace(flags=p.flags | FREEZE_FLOW)).init(rho, ux, uy, T)


@pytest.mark.parametrize("rho0", [0.2, 1.0])  # rho c_v = 1 and 5 with c_v = 5
def test_gaussian_pulse_diffusion(orc, sat, rho0):
    Tc, T0 = sat[0], sat[1]
    n, s0, A, steps = 128, 8.0, 0.005, 400
    p = Params(nx=n, ny=n)
    y, x = np.mgrid[0:n, 0:n].astype(float)
    r2 = (x - n / 2) ** 2 + (y - n / 2) ** 2
    T = T0 + A * np.exp(-r2 / (2 * s0 ** 2))
    o = _frozen(orc, p, np.full((n, n), rho0), 0 * T, 0 * T, T)
    o.step(steps)
    Tn = o.fields()[3]
    D = p.lambda_ / (rho0 * p.cv)
    s2 = s0 ** 2 + 2 * D * steps
    Ta = T0 + A * s0 ** 2 / s2 * np.exp(-r2 / (2 * s2))
    assert np.abs(Tn - Ta).max() <= 0.005 * A
    # the heat capacity matters: the same pulse with D = lambda (no rho c_v) is far off
    s2w = s0 ** 2 + 2 * p.lambda_ * steps
    Tw = T0 + A * s0 ** 2 / s2w * np.exp(-r2 / (2 * s2w))
    if rho0 * p.cv != 1.0:
        assert np.abs(Tn - Tw).max() > 0.1 * A


def _sine_mode(orc, T0, u, flags, rho0=1.0, lam=1 / 3, nx=64, steps=1000, A=1e-3):
    p = Params(nx=nx, ny=3, lambda_=lam, flags=flags | FREEZE_FLOW)
    x = np.arange(nx)[None, :] * np.ones((3, 1))
    k = 2 * np.pi / nx
    T = T0 + A * np.sin(k * x)
    rho = np.full((3, nx), rho0)
    o = orc.Oracle(p).init(rho, np.full((3, nx), u), 0 * rho, T)
    amps, ph = [], []
    for _ in range(steps // 100):
        o.step(100)
        c = np.fft.fft(o.fields()[3][0] - T0)[1]
        amps.append(abs(c) * 2 / nx)
        ph.append(np.angle(c))
    t = np.arange(100, steps + 1, 100)
    rate = -np.polyfit(t, np.log(amps), 1)[0]
    speed = -np.polyfit(t, np.unwrap(ph), 1)[0] / k
    return rate / k ** 2, speed, lam / (rho0 * p.cv)


@pytest.mark.parametrize("u", [0.05, 0.1])
@pytest.mark.parametrize("rho0", [0.2, 1.0])
def test_advection_tau1_S_cancels_half_u2(orc, sat, u, rho0):
    """tau_g = 1 (lambda = chat_s^2 / 2): the S term of Eq. (24) removes exactly the -u^2/2 error."""
    T0 = sat[1]
    lam = (2 / 3) / 2 / 2  # chat_s^2 (1 - 1/2) with tau_g = 1
    Don, c_on, D = _sine_mode(orc, T0, u, 0, rho0, lam)
    Doff, c_off, _ = _sine_mode(orc, T0, u, NO_S, rho0, lam)
    assert c_on == pytest.approx(u, rel=3e-3) and c_off == pytest.approx(u, rel=3e-3)
    assert abs(Don - D) <= 0.06 * u * u
    assert (D - Doff) == pytest.approx(0.5 * u * u, rel=0.03)


@pytest.mark.parametrize("rho0", [0.2, 0.4, 1.0])
def test_advection_gradient_lag_term(orc, sat, rho0):
    """tau_g = 1.5 (lambda = 1/3): D_eff = D - rho c_v (tau_g - 1) u^2 (S on), one u^2/2 lower (S off)."""
    T0, u = sat[1], 0.1
    Don, c_on, D = _sine_mode(orc, T0, u, 0, rho0)
    Doff, _, _ = _sine_mode(orc, T0, u, NO_S, rho0)
    rcv = rho0 * 5.0
    assert c_on == pytest.approx(u, rel=3e-3)
    assert (D - Don) == pytest.approx(rcv * 0.5 * u * u, rel=0.1, abs=0.1 * u * u)
    assert (Don - Doff) == pytest.approx(0.5 * u * u, rel=0.15)


def test_diffusion_rate_without_flow(orc, sat):
    for rho0 in (0.2, 1.0):
        Dm, c, D = _sine_mode(orc, sat[1], 0.0, 0, rho0)
        assert Dm == pytest.approx(D, rel=2e-3)
        assert abs(c) < 1e-10


def test_compression_heating_one_step(orc, base_params, sat):
    """Uniform rho, T and a frozen u_x = U sin(kx): after one step T changes by
    -T dpdT div(u) / (rho c_v) smoothed by the D2Q5 weights; div u of the isotropic stencil is
    U sin(k) cos(kx).  dp/dT is taken here by a finite difference of the EOS."""
    T0 = sat[1]
    nx, U, rho0 = 32, 0.02, 2.0
    p = Params(nx=nx, ny=3)
    k = 2 * np.pi / nx
    x = np.arange(nx)[None, :] * np.ones((3, 1))
    ux = U * np.sin(k * x)
    o = _frozen(orc, p, np.full((3, nx), rho0), ux, 0 * ux, np.full((3, nx), T0))
    o.step(1)
    T1 = o.fields()[3][0]
    h = 1e-7 * T0
    dpdT = (orc.eos_p(p, rho0, T0 + h) - orc.eos_p(p, rho0, T0 - h)) / (2 * h)
    w0, w1 = 1 - p.wdot, p.wdot / 4
    smooth = w0 + 2 * w1 * np.cos(k) + 2 * w1
    expect = T0 - T0 * dpdT * U * np.sin(k) * np.cos(k * x[0]) * smooth / (rho0 * p.cv)
    assert np.allclose(T1, expect, rtol=0, atol=1e-9 * abs(expect - T0).max())


def test_steady_conduction_between_dirichlet_walls(orc, sat):
    """Halfway anti-bounce-back walls: steady T is exactly linear, T_bot at y=-1/2, T_top at ny-1/2."""
    T0 = sat[1]
    nx, ny = 4, 12
    Tb, Tt = 1.02 * T0, 0.97 * T0
    p = Params(nx=nx, ny=ny, y_walls=1, T_bot=Tb, T_top=Tt)
    rho = np.full((ny, nx), 0.2)
    o = _frozen(orc, p, rho, 0 * rho, 0 * rho, np.full((ny, nx), T0))
    o.step(6000)
    T = o.fields()[3][:, 0]
    y = np.arange(ny)
    assert np.allclose(T, Tb + (Tt - Tb) * (y + 0.5) / ny, rtol=0, atol=1e-12)


def test_dirichlet_box_relaxes_to_edge_temperature(orc, sat):
    T0 = sat[1]
    n = 10
    p = Params(nx=n, ny=n, thermal_box=1, T_box=1.05 * T0)
    rho = np.full((n, n), 0.2)
    o = _frozen(orc, p, rho, 0 * rho, 0 * rho, np.full((n, n), T0))
    o.step(4000)
    assert np.allclose(o.fields()[3], 1.05 * T0, rtol=0, atol=1e-12)


@pytest.mark.parametrize("flags", [0, NO_S])
def test_discrete_energy_identity(orc, sat, flags):
    """Reading of the modified collision (rho c_v at the destination node, time t): on a periodic
    grid sum_y rho(y,t) c_v [T(y,t+1) - T(y,t)] equals sum_x [Q + S](x,t) for every step."""
    Tc, T0, rl, rg, _ = sat
    from workloads import droplet
    w = droplet(Tc, rl, rg, nx=32, ny=32, R=8.0, flags=flags)
    o = orc.Oracle(w.params).init(w.rho, w.ux, w.uy, w.T)
    o.step(30)
    for _ in range(5):
        f, g, _ = o.state()
        rho_t, T_t = f.sum(0), g.sum(0)
        o.step(1)
        T_n = o.state()[1].sum(0)
        _, _, sQ, sS = o.diagnostics()
        lhs = (rho_t * w.params.cv * (T_n - T_t)).sum()
        assert lhs == pytest.approx(sQ + sS, rel=1e-10, abs=1e-14 * (rho_t * T_t).sum())
        if flags & NO_S:
            assert sS == 0.0
