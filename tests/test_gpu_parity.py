"""GPU parity: the HIP library (through the C ABI) against the FP64 CPU oracle on the same seeded
inputs, element by element, for every boundary kind, ragged grids spanning several tiles, the
smallest grids, and the full-size static-droplet configuration.

FP64 runs must agree to rounding level.  FP32 runs are held to bounds derived from the FP32 unit
roundoff: see the tolerances next to each case.
"""
import numpy as np
import pytest

from workloads import FREEZE_FLOW, NO_S, Params, boiling, droplet, evaporation

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_00686_amd as lbm
    return lbm


def _case(name, w, steps, precision, lbm, orc):
    print(f"\n[case] {name} {w.params.nx}x{w.params.ny} steps={steps} "
          f"{'fp64' if precision == lbm.LBM_FP64 else 'fp32'}", flush=True)
    ref = orc.Oracle(w.params).init(w.rho, w.ux, w.uy, w.T)
    ref.step(steps)
    s = lbm.Solver(w.params, precision=precision).init(w.rho, w.ux, w.uy, w.T)
    s.step(steps)
    got = s.fields()
    exp = ref.fields()
    names = ("rho", "ux", "uy", "T")
    err = {n: float(np.abs(g - e).max()) for n, g, e in zip(names, got, exp)}
    print("   max abs err " + " ".join(f"{n}={v:.3e}" for n, v in err.items()), flush=True)
    return s, ref, got, exp, err


def _fixtures(orc):
    base = Params()
    Tc = orc.Tc(base)
    rl, rg, _ = orc.maxwell(base, 0.86 * Tc)
    return Tc, rl, rg


def _cases(orc):
    Tc, rl, rg = _fixtures(orc)
    return {
        "droplet": droplet(Tc, rl, rg, nx=150, ny=70, R=18.0),
        "evaporation": evaporation(Tc, rl, rg, nx=130, ny=90, R=20.0, superheat=1.2, hot_vapour=True),
        "boiling": boiling(Tc, rl, rg, nx=140, ny=84, hot_width=8.0, dT_rel=0.2, gravity=1e-4, seed=11),
    }


@pytest.mark.parametrize("kind", ["droplet", "evaporation", "boiling"])
def test_fp64_matches_oracle(lbm, orc, kind):
    w = _cases(orc)[kind]
    s, ref, got, exp, err = _case(kind, w, 300, lbm.LBM_FP64, lbm, orc)
    assert err["rho"] <= 1e-11
    assert err["T"] <= 1e-13
    assert max(err["ux"], err["uy"]) <= 1e-13
    # raw populations too
    fg, gg, hg = s.state()
    fo, go, ho = ref.state()
    assert np.abs(fg - fo).max() <= 1e-11
    assert np.abs(gg - go).max() <= 1e-13
    assert np.abs(hg - ho).max() <= 1e-13


@pytest.mark.parametrize("kind", ["droplet", "evaporation", "boiling"])
def test_fp32_matches_oracle(lbm, orc, kind):
    """FP32 populations: after 300 steps rho within 2e-4 (relative to rho_l ~ 6.5, about 500 unit
    roundoffs accumulated over 300 collisions), T within 2e-6 relative, u within 1e-5."""
    w = _cases(orc)[kind]
    _, _, got, exp, err = _case(kind, w, 300, lbm.LBM_FP32, lbm, orc)
    Tmax = float(np.abs(exp[3]).max())
    assert err["rho"] <= 2e-4 * 6.5
    assert err["T"] <= 2e-6 * Tmax
    assert max(err["ux"], err["uy"]) <= 1e-5


@pytest.mark.parametrize("nx,ny,walls", [(3, 3, 0), (5, 3, 1), (64, 16, 0), (65, 17, 1), (200, 3, 0)])
def test_fp64_small_and_ragged_grids(lbm, orc, nx, ny, walls):
    Tc, rl, rg = _fixtures(orc)
    rng = np.random.default_rng(nx * 100 + ny)
    rho = rg + (rl - rg) * rng.uniform(0.0, 1.0, (ny, nx))
    T = 0.86 * Tc * (1 + 0.01 * rng.uniform(-1, 1, (ny, nx)))
    ux = 0.01 * rng.standard_normal((ny, nx))
    uy = 0.01 * rng.standard_normal((ny, nx))
    p = Params(nx=nx, ny=ny, y_walls=walls, T_bot=0.9 * Tc, T_top=0.85 * Tc, hot_dT=0.05 * Tc, hot_x0=nx / 3,
               hot_sigma=2.0, theta_bot_deg=70.0, theta_top_deg=100.0, gy=-1e-4 if walls else 0.0)
    from workloads import Workload
    w = Workload("random", p, rho, ux, uy, T, 20)
    _, _, got, exp, err = _case(f"random walls={walls}", w, 20, lbm.LBM_FP64, lbm, orc)
    assert err["rho"] <= 1e-11 and err["T"] <= 1e-13 and max(err["ux"], err["uy"]) <= 1e-12


@pytest.mark.parametrize("nx,ny,walls", [(3, 3, 0), (4, 5, 0), (65, 17, 0), (130, 23, 0), (5, 4, 1), (65, 17, 1)])
def test_fp64_thermal_box_small_and_ragged_grids(lbm, orc, nx, ny, walls):
    """Dirichlet temperature box (all four edges, anti-bounce-back), alone and with walls, on the
    smallest and ragged multi-tile grids from random fields: FP64 to rounding."""
    Tc, rl, rg = _fixtures(orc)
    rng = np.random.default_rng(nx * 100 + ny + 7)
    rho = rg + (rl - rg) * rng.uniform(0.0, 1.0, (ny, nx))
    T = 0.86 * Tc * (1 + 0.01 * rng.uniform(-1, 1, (ny, nx)))
    ux = 0.01 * rng.standard_normal((ny, nx))
    uy = 0.01 * rng.standard_normal((ny, nx))
    p = Params(nx=nx, ny=ny, thermal_box=1, T_box=0.9 * Tc, y_walls=walls, T_bot=0.9 * Tc, T_top=0.85 * Tc,
               theta_bot_deg=70.0, theta_top_deg=100.0, gy=-1e-4 if walls else 0.0)
    from workloads import Workload
    w = Workload("random box", p, rho, ux, uy, T, 20)
    _, _, got, exp, err = _case(f"random thermal box walls={walls}", w, 20, lbm.LBM_FP64, lbm, orc)
    assert err["rho"] <= 1e-11 and err["T"] <= 1e-13 and max(err["ux"], err["uy"]) <= 1e-12


@pytest.mark.parametrize("nx,ny,kind", [(3, 3, "periodic"), (5, 3, "walls"), (4, 5, "box"), (5, 4, "open"),
                                        (65, 17, "walls"), (130, 23, "box+walls"), (200, 3, "open")])
def test_fp32_small_and_ragged_grids(lbm, orc, nx, ny, kind):
    """Every boundary kind on the smallest and ragged grids in FP32, from random fields: within the
    FP32 bounds of the other parity tests (rho 2e-4 rho_l, T 2e-6 relative, u 1e-5)."""
    Tc, rl, rg = _fixtures(orc)
    rng = np.random.default_rng(nx * 100 + ny + 11)
    # densities up to 0.85 of the liquid's, so that the wetting ghost (Eq. 54) of a random field stays
    # below the density where the EOS leaves the pseudopotential undefined
    rho = rg + (rl - rg) * rng.uniform(0.0, 0.85, (ny, nx))
    T = 0.86 * Tc * (1 + 0.01 * rng.uniform(-1, 1, (ny, nx)))
    ux = 0.01 * rng.standard_normal((ny, nx))
    uy = 0.01 * rng.standard_normal((ny, nx))
    walls = int(kind in ("walls", "box+walls", "open"))
    p = Params(nx=nx, ny=ny, y_walls=walls, thermal_box=int("box" in kind), T_box=0.9 * Tc, open_top=int(kind == "open"),
               T_bot=0.9 * Tc, T_top=0.85 * Tc, hot_dT=0.05 * Tc if walls else 0.0, hot_x0=nx / 3, hot_sigma=2.0,
               theta_bot_deg=70.0, theta_top_deg=100.0, gy=-1e-4 if walls else 0.0)
    from workloads import Workload
    w = Workload("random", p, rho, ux, uy, T, 20)
    _, _, got, exp, err = _case(f"random fp32 {kind}", w, 20, lbm.LBM_FP32, lbm, orc)
    assert err["rho"] <= 2e-4 * rl and err["T"] <= 2e-6 * float(np.abs(exp[3]).max())
    assert max(err["ux"], err["uy"]) <= 1e-5


@pytest.mark.parametrize("flags", [FREEZE_FLOW, FREEZE_FLOW | NO_S, NO_S])
def test_fp64_test_flags(lbm, orc, flags):
    Tc, rl, rg = _fixtures(orc)
    w = droplet(Tc, rl, rg, nx=70, ny=40, R=10.0, flags=flags)
    w.ux[:] = 0.03
    _, _, got, exp, err = _case(f"flags={flags}", w, 100, lbm.LBM_FP64, lbm, orc)
    assert err["rho"] <= 1e-11 and err["T"] <= 1e-13


def test_static_droplet_full_config_fp64(lbm, orc):
    """Static droplet: periodic 64x64, R = 16, Maxwell densities at 0.86 Tc, FP64, 2000 steps.
    Bounds: max|drho| <= 1e-9 and max|dT| <= 1e-12.  Mass and energy against the initial mass and the
    oracle's energy at 1e-12 relative: the collision adds M^-1 dm, whose nine components sum to zero
    exactly, and each of the nine additions rounds by at most half an ulp of its population, so a
    node's mass moves by at most about 4.5 unit roundoffs (1.1e-16) per step; over 2000 steps the
    worst case is 4.5 * 1.1e-16 * 2000 = 1.0e-12 (measured 1.0e-13, so the roundings are partly
    systematic; the oracle's own 300-step pin at 1e-13 sits inside the same bound)."""
    Tc, rl, rg = _fixtures(orc)
    w = droplet(Tc, rl, rg, nx=64, ny=64, R=16.0, steps=2000)
    s, ref, got, exp, err = _case("static droplet (full)", w, 2000, lbm.LBM_FP64, lbm, orc)
    assert err["rho"] <= 1e-9
    assert err["T"] <= 1e-12
    m0 = float(w.rho.sum())
    m, e = s.diagnostics()
    assert m == pytest.approx(m0, rel=1e-12)
    mo, eo, _, _ = ref.diagnostics()
    assert e == pytest.approx(eo, rel=1e-12)
