"""Pins of the oracle's flow step (D2Q9 MRT pseudopotential model, Eqs. 1-11, 54; buoyancy).

  * mass is conserved exactly on periodic and walled domains;
  * total momentum is conserved on a periodic domain with gravity: the interaction force of
    Eq. (9) cancels pairwise and (rho - rho_ave) g sums to zero;
  * body-force-driven Poiseuille flow between halfway bounce-back walls is exact (to rounding)
    with the MRT magic combination (1/s_p - 1/2)(1/s_q - 1/2) = 3/16;
  * a flat interface relaxes to the Maxwell coexistence densities with the tuned sigma (Eq. 8);
  * droplets obey the Laplace law (pressure jump linear in 1/R, one surface tension for two radius
    ranges, a small finite-size offset that shrinks with the radius);
  * a droplet in vapour at the paper's T_g = 1.0 Tc evaporates following the D^2 law (Eq. 55).
"""
import numpy as np
import pytest

from workloads import FREEZE_THERMAL, Params, boiling, droplet, tanh_disk


def test_mass_conserved_periodic(orc, sat):
    Tc, T0, rl, rg, _ = sat
    w = droplet(Tc, rl, rg, nx=48, ny=40, R=10.0)
    o = orc.Oracle(w.params).init(w.rho, w.ux, w.uy, w.T)
    m0 = o.diagnostics()[0]
    o.step(300)
    assert o.diagnostics()[0] == pytest.approx(m0, rel=1e-13)


def test_mass_conserved_with_walls_gravity_hot_spot(orc, sat):
    Tc, T0, rl, rg, _ = sat
    w = boiling(Tc, rl, rg, nx=40, ny=48, hot_width=4.0, gravity=3e-4, seed=7)
    o = orc.Oracle(w.params).init(w.rho, w.ux, w.uy, w.T)
    m0 = o.diagnostics()[0]
    o.step(300)
    assert o.diagnostics()[0] == pytest.approx(m0, rel=1e-13)


def test_momentum_conserved_periodic_with_gravity(orc, sat):
    Tc, T0, rl, rg, _ = sat
    n = 40
    rng = np.random.default_rng(5)
    rho = tanh_disk(n, n, 17.3, 21.1, 9.0, rl, rg)
    ux = 0.01 * rng.standard_normal((n, n))
    uy = 0.01 * rng.standard_normal((n, n))
    p = Params(nx=n, ny=n, gy=-1e-3, gx=4e-4)
    o = orc.Oracle(p).init(rho, ux, uy, np.full((n, n), T0))
    cx = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])[:, None, None]
    cy = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])[:, None, None]
    f = o.state()[0]
    j0 = np.array([(cx * f).sum(), (cy * f).sum()])
    for _ in range(4):
        o.step(50)
        f = o.state()[0]
        j = np.array([(cx * f).sum(), (cy * f).sum()])
        assert np.abs(j - j0).max() <= 1e-13 * rho.sum()


def test_poiseuille_exact(orc, sat):
    """Uniform liquid (no interaction force), walls at y = -1/2 and ny - 1/2, force rho g_x with
    rho_ave = 0: u_x(y) = g/(2 nu) (y + 1/2)(ny - 1/2 - y) at steady state."""
    T0, rl = sat[1], sat[2]
    nx, ny, g = 4, 16, 1e-6
    p = Params(nx=nx, ny=ny, y_walls=1, T_bot=T0, T_top=T0, gx=g, rho_ave=0.0, s_q=8.0 / 9.0)
    rho = np.full((ny, nx), rl)
    o = orc.Oracle(p).init(rho, 0 * rho, 0 * rho, np.full((ny, nx), T0))
    o.step(12000)
    _, ux, uy, T = o.fields()
    y = np.arange(ny)
    exact = g / (2 * p.nu) * (y + 0.5) * (ny - 0.5 - y)
    assert np.allclose(ux[:, 0], exact, rtol=0, atol=1e-9 * exact.max())
    assert np.abs(uy).max() < 1e-9 * exact.max()
    assert np.allclose(T, T0, rtol=0, atol=1e-11 * T0)


def test_flat_interface_reaches_maxwell_densities(orc, sat):
    Tc, T0, rl, rg, _ = sat
    nx, ny = 4, 256
    p = Params(nx=nx, ny=ny, flags=FREEZE_THERMAL)
    y = np.arange(ny, dtype=float)[:, None] * np.ones((1, nx))
    rho = 0.5 * (rl + rg) - 0.5 * (rl - rg) * np.tanh((np.abs(y - (ny - 1) / 2) - ny / 4) / 2.5)
    o = orc.Oracle(p).init(rho, 0 * rho, 0 * rho, np.full((ny, nx), T0))
    o.step(25000)
    liq, vap = [], []
    for _ in range(20):
        o.step(100)
        r = o.fields()[0][:, 0]
        liq.append(r[ny // 2 - 16: ny // 2 + 16].mean())
        vap.append(np.concatenate([r[:16], r[-16:]]).mean())
    assert np.mean(liq) == pytest.approx(rl, rel=1e-3)
    assert np.mean(vap) == pytest.approx(rg, rel=1e-2)


def _equivalent_radius(rho, rl, rg):
    return np.sqrt(np.clip((rho - rg) / (rl - rg), 0, 1).sum() / np.pi)


def _laplace_fit(orc, T0, rl, rg, Tc, n, radii, steps):
    """Isothermal droplets of the given radii on an n x n periodic box: fitted (gamma, intercept, R^2)
    of p_in - p_out against 1/R, and the pressure jumps."""
    inv_r, dp = [], []
    for R in radii:
        w = droplet(Tc, rl, rg, nx=n, ny=n, R=R, flags=FREEZE_THERMAL)
        o = orc.Oracle(w.params).init(w.rho, w.ux, w.uy, w.T)
        o.step(steps)  # the slowest acoustic mode of the largest droplet has decayed by then
        rho = o.fields()[0]
        c = n // 2
        p_in = orc.eos_p(w.params, rho[c - 2:c + 3, c - 2:c + 3].mean(), T0)
        p_out = orc.eos_p(w.params, rho[:4, :4].mean(), T0)
        inv_r.append(1.0 / _equivalent_radius(rho, rl, rg))
        dp.append(p_in - p_out)
    inv_r, dp = np.array(inv_r), np.array(dp)
    slope, icpt = np.polyfit(inv_r, dp, 1)
    fit = slope * inv_r + icpt
    r2 = 1 - ((dp - fit) ** 2).sum() / ((dp - dp.mean()) ** 2).sum()
    return slope, icpt, r2, dp


@pytest.mark.slow
def test_laplace_law(orc, sat):
    """Isothermal droplets: p_in - p_out = gamma / R.  Two independent sets, R = 12..21 on an 80^2
    box and R = 16..28 on a 112^2 box: each is linear in 1/R (R^2 >= 0.999), both give the same
    surface tension within 0.5 % (measured 0.05 %), and the small offset of the line (a finite-size
    effect of the diffuse interface, measured -4.2 % and -3.7 % of the jump at the smallest radius
    of each set) shrinks as the droplets grow.  A wrong force, ghost-free stencil or collision
    term would change gamma with the radius range or bend the line."""
    Tc, T0, rl, rg, _ = sat
    g1, b1, r2a, dp1 = _laplace_fit(orc, T0, rl, rg, Tc, 80, (12.0, 15.0, 18.0, 21.0), 8000)
    g2, b2, r2b, dp2 = _laplace_fit(orc, T0, rl, rg, Tc, 112, (16.0, 20.0, 24.0, 28.0), 8000)
    print(f"gamma {g1:.5e} / {g2:.5e}; offsets {b1 / dp1[0]:.4f} / {b2 / dp2[0]:.4f} of the first jump; "
          f"R^2 {r2a:.6f} / {r2b:.6f}")
    assert g1 > 0 and g2 > 0
    assert r2a >= 0.999 and r2b >= 0.999
    assert g1 == pytest.approx(g2, rel=5e-3)
    assert abs(b1) <= 0.07 * dp1[0] and abs(b2) <= 0.05 * dp2[0]
    assert abs(b2) < abs(b1)


@pytest.mark.slow
def test_d2_law_evaporation(orc, sat):
    """The D^2-law test of Section 4.1 with the paper's values (saturated droplet at 0.86 Tc in
    vapour and box edges at T_g = 1.0 Tc, lambda = 1/3, nu = 0.1, c_v = 5), scaled from D_0 = 60 on
    200^2 to D_0 = 20 on 64^2 (same box-to-droplet ratio; the evaporation time scales with D_0^2):
    the droplet area, measured as the liquid excess over the far-field vapour
    sum clip((rho - rho_v)/(rho_l - rho_v), 0, 1) with rho_v the median density, falls linearly in
    time (Eq. 55, (D/D_0)^2 = 1 - K t / D_0^2) while it goes from 0.9 to 0.2 of its start: R^2 >= 0.995
    (measured 0.9971)."""
    Tc, T0, rl, rg, _ = sat
    from workloads import evaporation
    w = evaporation(Tc, rl, rg, nx=64, ny=64, R=10.0, superheat=1.0 / 0.86, hot_vapour=True)
    o = orc.Oracle(w.params).init(w.rho, w.ux, w.uy, w.T)
    A0 = np.clip((w.rho - rg) / (rl - rg), 0, 1).sum()
    t, a = [], []
    while o.steps < 80000:
        o.step(250)
        rho = o.fields()[0]
        rv = float(np.median(rho))
        t.append(o.steps)
        a.append(np.clip((rho - rv) / (rl - rv), 0, 1).sum() / A0)
        if a[-1] < 0.15:
            break
    t, a = np.array(t), np.array(a)
    sel = (a <= 0.9) & (a >= 0.2)
    assert sel.sum() >= 100, a
    slope, icpt = np.polyfit(t[sel], a[sel], 1)
    fit = slope * t[sel] + icpt
    r2 = 1 - ((a[sel] - fit) ** 2).sum() / ((a[sel] - a[sel].mean()) ** 2).sum()
    print(f"D^2 law: slope {slope:.4e} per step, R^2 {r2:.5f} over {sel.sum()} points")
    assert slope < 0
    assert r2 >= 0.995


@pytest.mark.parametrize("theta", [60.0, 90.0, 120.0])
def test_contact_angle_of_sessile_droplet(orc, sat, theta):
    """Geometric wetting condition (Eq. 54): a droplet on the bottom wall relaxes to a circular
    cap whose angle 2 atan(2h/b) (height h above the wall plane, base width b at the first
    fluid row, both at rho_mid) is the prescribed angle."""
    Tc, T0, rl, rg, _ = sat
    nx, ny = 120, 60
    p = Params(nx=nx, ny=ny, y_walls=1, T_bot=T0, T_top=T0, theta_bot_deg=theta, flags=FREEZE_THERMAL)
    rho = tanh_disk(nx, ny, nx / 2, 0.0, 22.0, rl, rg)
    o = orc.Oracle(p).init(rho, 0 * rho, 0 * rho, np.full((ny, nx), T0))
    o.step(3000)
    r = o.fields()[0]
    rmid = 0.5 * (rl + rg)
    row, col = r[0], r[:, nx // 2]
    liq = np.where(row > rmid)[0]
    L, R = liq.min(), liq.max()
    b = (R + (row[R] - rmid) / (row[R] - row[R + 1])) - (L - (row[L] - rmid) / (row[L] - row[L - 1]))
    top = np.where(col > rmid)[0].max()
    h = top + (col[top] - rmid) / (col[top] - col[top + 1]) + 0.5  # wall plane at y = -1/2
    assert np.degrees(2 * np.arctan(2 * h / b)) == pytest.approx(theta, abs=5.0)
