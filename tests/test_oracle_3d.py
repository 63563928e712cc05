"""Pins of the three-dimensional oracle (D3Q19 pseudopotential flow with the paper's temperature
model on D3Q7; the readings are listed in oracle/lbm3d_oracle.c):

  * matrices: the D3Q19 moment basis is orthogonal; M f_eq gives the equilibrium moments rho,
    j = rho u, e = -11 rho + 19 rho u^2, eps = 3 rho - (11/2) rho u^2; the D3Q7 matrix maps
    what T to [T, 0, 0, 0, wdot T, 0, 0];
  * mass (exact) and total momentum (zero net interaction force on a periodic domain) of a
    droplet; the discrete energy identity sum rho c_v (T^{t+1} - T^t) = sum (Q + S);
  * a uniform state stays uniform;
  * Gaussian temperature pulse in three dimensions (frozen flow) against the exact diffusion
    solution with D = lambda/(rho c_v), lambda = (wdot/3)(tau_g - 1/2);
  * a flat interface across a thin periodic box settles at the Maxwell densities with the sigma
    of the two-dimensional model (the per-component reading of the sigma term);
  * two spherical droplets give the same surface tension from the Laplace law dp = 2 gamma / R;
  * a shear wave decays at nu k^2 with nu = (1/s_nu - 1/2)/3, in each of the three orientations
    that put it on one of the off-diagonal stress moments (xz, xy, yz), at two viscosities.
"""
import numpy as np
import pytest

from workloads import Params, Params3D, droplet3d


@pytest.fixture(scope="module")
def o3(orc):
    from oracle import o3d
    return o3d


def test_matrices(o3, sat):
    T0, rl = sat[1], sat[2]
    o = o3.Oracle3D(Params3D(nx=4, ny=4, nz=4))
    M, M7 = o.matrices()
    G = M @ M.T
    assert np.abs(G - np.diag(np.diag(G))).max() < 1e-12
    rho, u = 1.7, np.array([0.03, -0.02, 0.05])
    m = M @ o3.feq(rho, *u)
    uu = float(u @ u)
    assert m[0] == pytest.approx(rho, rel=1e-14)
    assert np.allclose(m[[3, 5, 7]], rho * u, rtol=0, atol=1e-15)
    assert m[1] == pytest.approx(-11 * rho + 19 * rho * uu, rel=1e-13)
    assert m[2] == pytest.approx(3 * rho - 5.5 * rho * uu, rel=1e-13)
    wd = Params3D().wdot
    w = np.array([1 - wd] + [wd / 6] * 6)
    assert np.allclose(M7 @ (w * T0), [T0, 0, 0, 0, wd * T0, 0, 0], rtol=0, atol=1e-15)


def test_mass_momentum_and_energy_identity(o3, sat):
    Tc, T0, rl, rg, _ = sat
    w = droplet3d(Tc, rl, rg, n=16, R=5.0)
    w.uz[:] = 0.01 * np.sin(2 * np.pi * np.arange(16) / 16)[:, None, None]
    o = o3.Oracle3D(w.params).init(w.rho, w.ux, w.uy, w.uz, w.T)
    m0 = float(w.rho.sum())
    o.step(20)
    for _ in range(4):
        f, g, _ = o.state()
        rho_t, T_t = f.sum(0), g.sum(0)
        o.step(1)
        fn, gn, _ = o.state()
        mass, _, sQ, sS = o.diagnostics()
        assert mass == pytest.approx(m0, rel=1e-13)
        lhs = (rho_t * w.params.cv * (gn.sum(0) - T_t)).sum()
        assert lhs == pytest.approx(sQ + sS, rel=1e-10, abs=1e-14 * (rho_t * T_t).sum())
    # total momentum: the initial sine flow has zero mean, the interaction force sums to zero
    C = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1], [1, 1, 0],
                  [-1, -1, 0], [1, -1, 0], [-1, 1, 0], [1, 0, 1], [-1, 0, -1], [1, 0, -1], [-1, 0, 1], [0, 1, 1],
                  [0, -1, -1], [0, 1, -1], [0, -1, 1]])
    j = np.tensordot(C.T, fn, axes=(1, 0)).reshape(3, -1).sum(1)
    assert np.abs(j).max() <= 1e-11 * m0


def test_uniform_state_is_steady(o3, sat):
    T0, rl = sat[1], sat[2]
    p = Params3D(nx=6, ny=5, nz=4)
    rho = np.full((4, 5, 6), rl)
    z = 0 * rho
    o = o3.Oracle3D(p).init(rho, z, z, z, np.full_like(rho, T0))
    o.step(30)
    r, ux, uy, uz, T = o.fields()
    assert np.allclose(r, rl, rtol=1e-13) and np.allclose(T, T0, rtol=1e-13)
    assert max(np.abs(ux).max(), np.abs(uy).max(), np.abs(uz).max()) < 1e-14


def _pulse_error(o3, T0, rho0, n, s0, steps, A=0.005):
    """Max |T - T_exact| / A of a frozen-flow Gaussian pulse in a periodic n^3 box (the exact
    solution summed with its 26 nearest images), and the D used."""
    p = Params3D(nx=n, ny=n, nz=n, flags=o3.FREEZE_FLOW)
    z, y, x = np.mgrid[0:n, 0:n, 0:n].astype(float)

    def gauss(s2):
        out = 0.0
        for dz in (-n, 0, n):
            for dy in (-n, 0, n):
                for dx in (-n, 0, n):
                    r2 = (x - n / 2 + dx) ** 2 + (y - n / 2 + dy) ** 2 + (z - n / 2 + dz) ** 2
                    out = out + (s0 ** 2 / s2) ** 1.5 * np.exp(-r2 / (2 * s2))
        return out

    T = T0 + A * gauss(s0 ** 2)
    o = o3.Oracle3D(p).init(np.full_like(T, rho0), 0 * T, 0 * T, 0 * T, T)
    o.step(steps)
    Tn = o.fields()[4]
    D = p.lambda_ / (rho0 * p.cv)
    err = float(np.abs(Tn - (T0 + A * gauss(s0 ** 2 + 2 * D * steps))).max() / A)
    err_wrong_D = float(np.abs(Tn - (T0 + A * gauss(s0 ** 2 + 2 * p.lambda_ * steps))).max() / A)
    return err, err_wrong_D


@pytest.mark.parametrize("rho0", [0.2, 1.0])
def test_gaussian_pulse_diffusion_3d(o3, sat, rho0):
    """D3Q7 with chat_s^2 = 2/9 runs at tau_g = 2 for lambda = 1/3, where the scheme's higher-order
    error is larger than in two dimensions: at rho c_v = 5 the narrow pulse (s0 = 4) is off by
    2.7 % of its amplitude, a wider one (s0 = 6) by 1.4 %.  Pins: within 2 % at s0 = 6, the error
    falls by at least 0.6 x from s0 = 4 to 6 (it converges), and using lambda instead of
    lambda/(rho c_v) as the diffusivity would be far off."""
    T0 = sat[1]
    e4, _ = _pulse_error(o3, T0, rho0, 40, 4.0, 60)
    e6, wrong = _pulse_error(o3, T0, rho0, 48, 6.0, 100)
    assert e6 <= 0.02
    assert e6 <= 0.6 * e4 or e4 <= 2e-3
    if rho0 * 5.0 != 1.0:
        assert wrong > 0.1


def test_flat_interface_at_maxwell_densities(o3, sat):
    """sigma = 1.25 (the two-dimensional value) with the per-component reading of the sigma term:
    a flat slab across a 4 x 4 x 128 periodic box, temperature frozen, 12000 steps, densities
    averaged over the last 2000 steps: within 5e-5 (liquid) and 3e-3 (vapour) of Maxwell's."""
    Tc, T0, rl, rg, _ = sat
    nz = 128
    p = Params3D(nx=4, ny=4, nz=nz, flags=o3.FREEZE_THERMAL)
    zz = np.arange(nz, dtype=float)[:, None, None] * np.ones((1, 4, 4))
    rho = 0.5 * (rl + rg) - 0.5 * (rl - rg) * np.tanh((np.abs(zz - (nz - 1) / 2) - nz / 4) / 2.5)
    z = 0 * rho
    o = o3.Oracle3D(p).init(rho, z, z, z, np.full_like(rho, T0))
    o.step(10000)
    liq, vap = [], []
    for _ in range(20):
        o.step(100)
        r = o.fields()[0][:, 0, 0]
        liq.append(r[nz // 2 - 8: nz // 2 + 8].mean())
        vap.append(np.concatenate([r[:8], r[-8:]]).mean())
    assert abs(np.mean(liq) / rl - 1) <= 5e-5
    assert abs(np.mean(vap) / rg - 1) <= 3e-3


def test_laplace_law_two_droplets(o3, sat):
    """Isothermal spherical droplets of radius 6.5 and 8.5 in a 24^3 periodic box (steady by 1250
    steps): the pressure jump (EOS pressure at the centre minus the far field, 3^3-node means)
    times R_e / 2, R_e from the liquid volume, gives one surface tension to within 10 % (measured
    0.0780 and 0.0748).  Smaller droplets (R = 4.5 here) dissolve into the supersaturated vapour."""
    Tc, T0, rl, rg, _ = sat
    n, c, gam = 24, 12, []
    for R in (6.5, 8.5):
        w = droplet3d(Tc, rl, rg, n=n, R=R, flags=o3.FREEZE_THERMAL)
        o = o3.Oracle3D(w.params).init(w.rho, w.ux, w.uy, w.uz, w.T)
        o.step(1500)
        r = o.fields()[0]
        p_in = o3.eos_p(w.params, r[c - 1:c + 2, c - 1:c + 2, c - 1:c + 2].mean(), T0)
        p_out = o3.eos_p(w.params, r[:3, :3, :3].mean(), T0)
        Re = (3 * np.clip((r - rg) / (rl - rg), 0, 1).sum() / (4 * np.pi)) ** (1 / 3)
        gam.append((p_in - p_out) * Re / 2)
    assert gam[0] > 0 and gam[1] > 0
    assert gam[0] == pytest.approx(gam[1], rel=0.10)


@pytest.mark.parametrize("nu", [0.1, 1.0 / 30.0])
@pytest.mark.parametrize("comp,axis", [("ux", "z"), ("uy", "x"), ("uz", "y")])
def test_shear_wave_decays_at_the_viscous_rate(o3, sat, nu, comp, axis):
    """u_comp = U sin(k axis) in a uniform liquid (psi uniform, so no interaction force; div u = 0,
    so the temperature stays uniform) decays as exp(-nu k^2 t), nu = (1/s_nu - 1/2)/3: the decay
    rate between steps 100 and 300 is within 0.5 % of nu k^2 (the finite-k correction is about
    k^2/12 of it).  A stress moment relaxed at another rate would be off by tens of percent."""
    T0, rl = sat[1], sat[2]
    n, U = 32, 1e-3
    k = 2 * np.pi / n
    p = Params3D(nx=n if axis == "x" else 4, ny=n if axis == "y" else 4, nz=n if axis == "z" else 4, nu=nu)
    shp = (p.nz, p.ny, p.nx)
    z, y, x = np.meshgrid(np.arange(p.nz), np.arange(p.ny), np.arange(p.nx), indexing="ij")
    mode = np.sin(k * {"x": x, "y": y, "z": z}[axis])
    u = {"ux": 0 * mode, "uy": 0 * mode, "uz": 0 * mode}
    u[comp] = U * mode
    o = o3.Oracle3D(p).init(np.full(shp, rl), u["ux"], u["uy"], u["uz"], np.full(shp, T0))
    amp = []
    for _ in range(3):
        o.step(100)
        f = o.fields()
        uc = {"ux": f[1], "uy": f[2], "uz": f[3]}[comp]
        amp.append(float((uc * mode).sum() / (mode * mode).sum()))
    rate = -np.log(amp[2] / amp[0]) / 200.0
    assert rate == pytest.approx(nu * k * k, rel=5e-3)
