"""Pins of the oracle's collision and streaming against textbook special cases, written here in
velocity space (no moment matrices):

  * Flow: with every non-conserved rate of the MRT (Eq. 5) equal to one value s and sigma = 0 in
    Li's forcing (Eq. 8), the flow step is the single-relaxation-time (BGK) collision with Guo's
    forcing term, f* = f - s (f - f_eq) + (1 - s/2) w_i [3 (c_i - u) + 9 (c_i . u) c_i] . F, with
    u = (j + F/2)/rho and F the Shan-Chen interaction force plus buoyancy.  From a random
    non-equilibrium state the oracle's post-collision populations must equal it to rounding, and
    the streamed populations must be those values moved by c_i (periodic box).
  * Temperature: with every non-conserved rate of the D2Q5 MRT (Eq. 39) equal, the fluid at rest
    (Q = 0), the history flat (S = 0) and rho c_v = 1 (the modified streaming of Eq. 21 is then
    plain streaming), one step is the textbook D2Q5 BGK diffusion step g_i(x + c_i) =
    g_i - s_g (g_i - w_i T).

  * Three dimensions: every D3Q19 rate 1 and sigma = 0 gives f* = f_eq + G/2 with Guo's term and
    the interaction force of weights 1/6 and 1/12; D3Q7 at equal rates, at rest, with S off and
    rho c_v = 1 gives the textbook D3Q7 BGK diffusion step.

A transposed or mistyped transformation matrix, a wrong sign or weight in the forcing, a rate on
the wrong row, or streaming in the wrong direction fails these.
"""
import numpy as np

from workloads import FREEZE_FLOW, Params

C9 = np.array([(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)])
W9 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
C5 = C9[:5]


def _shift(a, c):
    """a moved by the lattice vector c (periodic): out(x + c) = a(x)."""
    return np.roll(a, shift=(c[1], c[0]), axis=(0, 1))


def _at(a, c):
    """a(x + c) at every node x (periodic)."""
    return np.roll(a, shift=(-c[1], -c[0]), axis=(0, 1))


def test_flow_step_at_equal_rates_is_bgk_with_guo_forcing(orc, sat):
    Tc, T0, rl, rg, _ = sat
    nx, ny, nu, gy = 14, 11, 0.1, -3e-3
    s = 1.0 / (3.0 * nu + 0.5)
    p = Params(nx=nx, ny=ny, nu=nu, s_e=s, s_eps=s, s_q=s, sigma=0.0, gy=gy)
    rng = np.random.default_rng(7)
    rho = rng.uniform(0.5, 6.0, (ny, nx))
    u = 0.02 * rng.standard_normal((2, ny, nx))
    T = T0 * (1.0 + 0.05 * rng.uniform(-1, 1, (ny, nx)))
    o = orc.Oracle(p).init(rho, u[0], u[1], T)
    S, _ = o.relaxation()
    assert np.all(S[[1, 2, 4, 6, 7, 8]] == s)  # every non-conserved row relaxes at s

    # a random state away from equilibrium
    f0, g0, _ = o.state()
    f = f0 * (1.0 + 0.05 * rng.uniform(-1, 1, f0.shape))
    g = g0 * (1.0 + 0.01 * rng.uniform(-1, 1, g0.shape))
    Tn = g.sum(axis=0)
    o.set_state(f, g, np.stack([Tn, Tn]))
    o.step(1)

    # the same collision in velocity space
    rho = f.sum(axis=0)
    j = np.einsum("iyx,ic->cyx", f, C9.astype(float))
    psi = np.vectorize(lambda r, t: orc.psi(p, r, t))(rho, Tn)
    assert np.all(psi > 0)
    Fm = np.zeros((2, ny, nx))
    for i in range(1, 9):
        wi = 1 / 3 if i < 5 else 1 / 12
        Fm += -p.G * psi * wi * _at(psi, C9[i])[None] * C9[i][:, None, None]
    F = Fm + np.stack([np.zeros_like(rho), (rho - o.rho_ave) * gy])
    uu = (j + 0.5 * F) / rho
    fs = np.empty_like(f)
    for i in range(9):
        cu = C9[i, 0] * uu[0] + C9[i, 1] * uu[1]
        feq = W9[i] * rho * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * (uu[0] ** 2 + uu[1] ** 2))
        guo = W9[i] * ((3 * (C9[i, 0] - uu[0]) + 9 * cu * C9[i, 0]) * F[0] +
                       (3 * (C9[i, 1] - uu[1]) + 9 * cu * C9[i, 1]) * F[1])
        fs[i] = f[i] - s * (f[i] - feq) + (1 - s / 2) * guo
    post = o.post_collision()
    assert np.abs(post - fs).max() <= 1e-13 * np.abs(fs).max()
    # the forcing matters at this size: without it the populations differ far above rounding
    assert np.abs(F).max() > 1e-3

    # push streaming in a periodic box
    fn = o.state()[0]
    for i in range(9):
        assert np.array_equal(fn[i], _shift(post[i], C9[i]))


def test_thermal_step_at_equal_rates_and_unit_heat_capacity_is_bgk_diffusion(orc, sat):
    T0 = sat[1]
    nx, ny, lam = 13, 9, 1.0 / 3.0
    wdot = 2.0 / 3.0
    sg = 1.0 / (lam / (wdot / 2.0) + 0.5)
    cv = 5.0
    p = Params(nx=nx, ny=ny, lambda_=lam, wdot=wdot, vs3=sg, vs4=sg, cv=cv, flags=FREEZE_FLOW)
    rng = np.random.default_rng(8)
    rho = np.full((ny, nx), 0.2)  # rho c_v = 1
    assert np.all(rho * cv == 1.0)
    T = T0 * (1.0 + 0.05 * rng.uniform(-1, 1, (ny, nx)))
    o = orc.Oracle(p).init(rho, 0 * T, 0 * T, T)
    _, L = o.relaxation()
    assert np.all(L[1:] == sg)
    f0, g0, _ = o.state()
    g = g0 * (1.0 + 0.05 * rng.uniform(-1, 1, g0.shape))  # away from equilibrium
    Tn = g.sum(axis=0)
    o.set_state(f0, g, np.stack([Tn, Tn]))  # flat history: S = 0; fluid at rest: Q = 0
    o.step(1)

    w5 = np.array([1 - wdot] + [wdot / 4] * 4)
    gn = o.state()[1]
    for i in range(5):
        gs = g[i] - sg * (g[i] - w5[i] * Tn)
        expect = _shift(gs, C5[i])
        assert np.abs(gn[i] - expect).max() <= 1e-15 * np.abs(expect).max() * 10


# ---- three dimensions (D3Q19 flow, D3Q7 temperature; the oracle's velocity order)
C19 = np.array([(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
                (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1), (1, 0, -1),
                (-1, 0, 1), (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)])
W19 = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)


def _shift3(a, c):
    return np.roll(a, shift=(c[2], c[1], c[0]), axis=(0, 1, 2))


def _at3(a, c):
    return np.roll(a, shift=(-c[2], -c[1], -c[0]), axis=(0, 1, 2))


def test_3d_flow_step_at_unit_rates_is_bgk_with_guo_forcing(orc, sat):
    """Every D3Q19 rate 1 (nu = 1/6, s_e = s_eps = 1) and sigma = 0: f* = f_eq(rho, u) + G/2 with
    Guo's term G and u = (j + F/2)/rho, F the interaction force with the weights 1/6 and 1/12."""
    from oracle import o3d
    from workloads import Params3D
    T0 = sat[1]
    n = (7, 6, 5)  # nz, ny, nx
    p = Params3D(nx=n[2], ny=n[1], nz=n[0], nu=1.0 / 6.0, sigma=0.0)
    assert 3.0 * p.nu + 0.5 == 1.0
    rng = np.random.default_rng(9)
    rho = rng.uniform(0.5, 6.0, n)
    u = 0.02 * rng.standard_normal((3,) + n)
    T = T0 * (1.0 + 0.05 * rng.uniform(-1, 1, n))
    o = o3d.Oracle3D(p).init(rho, u[0], u[1], u[2], T)
    f, g, _ = o.state()
    o.step(1)

    rho = f.sum(axis=0)
    j = np.einsum("izyx,ic->czyx", f, C19.astype(float))
    Tn = g.sum(axis=0)
    pe = np.vectorize(lambda r, t: o3d.eos_p(p, r, t))(rho, Tn)
    psi = np.sqrt(2.0 * (rho / 3.0 - pe) / -p.G)
    F = np.zeros((3,) + n)
    for i in range(1, 19):
        wi = 1 / 6 if np.abs(C19[i]).sum() == 1 else 1 / 12
        F += -p.G * psi * wi * _at3(psi, C19[i])[None] * C19[i][:, None, None, None]
    uu = (j + 0.5 * F) / rho
    u2 = (uu ** 2).sum(axis=0)
    fn = o.state()[0]
    for i in range(19):
        c = C19[i]
        cu = sum(c[a] * uu[a] for a in range(3))
        feq = W19[i] * rho * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * u2)
        guo = W19[i] * sum((3 * (c[a] - uu[a]) + 9 * cu * c[a]) * F[a] for a in range(3))
        fs = feq + 0.5 * guo
        assert np.abs(fn[i] - _shift3(fs, c)).max() <= 1e-13 * rho.max()
    assert np.abs(F).max() > 1e-3


def test_3d_thermal_step_at_equal_rates_and_unit_heat_capacity_is_bgk_diffusion(orc, sat):
    """D3Q7 with every non-conserved rate equal (vs3 = varsigma), the fluid frozen at rest (Q = 0),
    the S term off and rho c_v = 1: the second step, from the streamed (non-equilibrium) state of
    the first, is g_i(x + c_i) = g_i - s (g_i - w_i T) with w = (1 - wdot, wdot/6 x 6)."""
    from oracle import o3d
    from workloads import NO_S, Params3D
    T0 = sat[1]
    n = (5, 7, 6)
    lam, wdot, cv = 0.25, 2.0 / 3.0, 5.0
    sg = 1.0 / (lam / (wdot / 3.0) + 0.5)
    p = Params3D(nx=n[2], ny=n[1], nz=n[0], lambda_=lam, wdot=wdot, vs3=sg, cv=cv, flags=FREEZE_FLOW | NO_S)
    rng = np.random.default_rng(10)
    T = T0 * (1.0 + 0.05 * rng.uniform(-1, 1, n))
    z = np.zeros(n)
    o = o3d.Oracle3D(p).init(np.full(n, 0.2), z, z, z, T)
    o.step(1)
    g = o.state()[1]
    Tn = g.sum(axis=0)
    w7 = np.array([1 - wdot] + [wdot / 6] * 6)
    assert np.abs(g - w7[:, None, None, None] * Tn).max() > 1e-6  # away from equilibrium
    o.step(1)
    gn = o.state()[1]
    for i in range(7):
        gs = g[i] - sg * (g[i] - w7[i] * Tn)
        expect = _shift3(gs, C19[i])  # the D3Q7 velocities are the first seven of D3Q19
        assert np.abs(gn[i] - expect).max() <= 1e-14 * np.abs(expect).max()
