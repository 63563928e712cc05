"""GPU parity of the thermal-lattice variants against the FP64 oracle, through the C ABI:
the D2Q9 thermal lattice with the BGK collision of Eq. (21), and the BGK variant of the D2Q5
model (the GPU runs it as the MRT step with every rate 1/tau_g; the oracle evaluates Eq. (21)
directly).  Same bounds as the D2Q5 MRT parity tests: FP64 to rounding, FP32 after 300 steps
rho within 2e-4 rho_l, T within 2e-6 relative, u within 1e-5.  Also: every one-step tile shape
gives the same bits for D2Q9, a batch of D2Q9 members equals their single runs, save/load
round-trips the 9 thermal planes, and the footprint is 160 B per node in FP32."""
import numpy as np
import pytest

from workloads import BGK, NO_S, Params, boiling, droplet, evaporation

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_00686_amd as lbm
    return lbm


def _sat(orc):
    base = Params()
    Tc = orc.Tc(base)
    rl, rg, _ = orc.maxwell(base, 0.86 * Tc)
    return Tc, rl, rg


def _cases(orc, **kw):
    Tc, rl, rg = _sat(orc)
    return {
        "droplet": droplet(Tc, rl, rg, nx=150, ny=70, R=18.0, **kw),
        "evaporation": evaporation(Tc, rl, rg, nx=130, ny=90, R=20.0, superheat=1.2, hot_vapour=True, **kw),
        "boiling": boiling(Tc, rl, rg, nx=140, ny=84, hot_width=8.0, dT_rel=0.2, gravity=1e-4, seed=11, **kw),
    }


def _run(lbm, orc, w, steps, precision, label):
    print(f"\n[case] {label} {w.params.nx}x{w.params.ny} steps={steps} "
          f"{'fp64' if precision == lbm.LBM_FP64 else 'fp32'}", flush=True)
    ref = orc.Oracle(w.params).init(w.rho, w.ux, w.uy, w.T)
    ref.step(steps)
    s = lbm.Solver(w.params, precision=precision).init(w.rho, w.ux, w.uy, w.T)
    s.step(steps)
    got, exp = s.fields(), ref.fields()
    err = {n: float(np.abs(g - e).max()) for n, g, e in zip(("rho", "ux", "uy", "T"), got, exp)}
    print("   max abs err " + " ".join(f"{n}={v:.3e}" for n, v in err.items()), flush=True)
    return s, ref, got, exp, err


@pytest.mark.parametrize("kind", ["droplet", "evaporation", "boiling"])
def test_q9_fp64_matches_oracle(lbm, orc, kind):
    w = _cases(orc, thermal_q=9)[kind]
    s, ref, got, exp, err = _run(lbm, orc, w, 300, lbm.LBM_FP64, f"D2Q9 {kind}")
    assert err["rho"] <= 1e-11 and err["T"] <= 1e-13 and max(err["ux"], err["uy"]) <= 1e-13
    fg, gg, hg = s.state()
    fo, go, ho = ref.state()
    assert gg.shape == go.shape == (9, w.params.ny, w.params.nx)
    assert np.abs(fg - fo).max() <= 1e-11 and np.abs(gg - go).max() <= 1e-13 and np.abs(hg - ho).max() <= 1e-13
    s.close()


@pytest.mark.parametrize("kind", ["droplet", "evaporation", "boiling"])
def test_q9_fp32_matches_oracle(lbm, orc, kind):
    w = _cases(orc, thermal_q=9)[kind]
    s, _, got, exp, err = _run(lbm, orc, w, 300, lbm.LBM_FP32, f"D2Q9 {kind}")
    Tmax = float(np.abs(exp[3]).max())
    assert err["rho"] <= 2e-4 * 6.5 and err["T"] <= 2e-6 * Tmax and max(err["ux"], err["uy"]) <= 1e-5
    s.close()


@pytest.mark.parametrize("kind", ["evaporation", "boiling"])
@pytest.mark.parametrize("precision", [0, 1])
def test_d2q5_bgk_matches_oracle(lbm, orc, kind, precision):
    """rho c_v >= 1.9 everywhere here (c_v = 5), where the D2Q5 BGK variant is stable."""
    w = _cases(orc, flags=BGK)[kind]
    s, _, got, exp, err = _run(lbm, orc, w, 300, precision, f"D2Q5-BGK {kind}")
    if precision == lbm.LBM_FP64:
        assert err["rho"] <= 1e-11 and err["T"] <= 1e-13 and max(err["ux"], err["uy"]) <= 1e-13
    else:
        Tmax = float(np.abs(exp[3]).max())
        assert err["rho"] <= 2e-4 * 6.5 and err["T"] <= 2e-6 * Tmax and max(err["ux"], err["uy"]) <= 1e-5
    s.close()


@pytest.mark.parametrize("nx,ny,walls", [(3, 3, 0), (5, 3, 1), (65, 17, 1), (200, 3, 0)])
def test_q9_fp64_small_and_ragged_grids(lbm, orc, nx, ny, walls):
    Tc, rl, rg = _sat(orc)
    rng = np.random.default_rng(nx * 100 + ny)
    rho = rg + (rl - rg) * rng.uniform(0.0, 1.0, (ny, nx))
    T = 0.86 * Tc * (1 + 0.01 * rng.uniform(-1, 1, (ny, nx)))
    ux = 0.01 * rng.standard_normal((ny, nx))
    uy = 0.01 * rng.standard_normal((ny, nx))
    p = Params(nx=nx, ny=ny, y_walls=walls, T_bot=0.9 * Tc, T_top=0.85 * Tc, hot_dT=0.05 * Tc, hot_x0=nx / 3,
               hot_sigma=2.0, theta_bot_deg=70.0, theta_top_deg=100.0, gy=-1e-4 if walls else 0.0, thermal_q=9)
    from workloads import Workload
    w = Workload("random", p, rho, ux, uy, T, 20)
    _, _, _, _, err = _run(lbm, orc, w, 20, lbm.LBM_FP64, f"D2Q9 random walls={walls}")
    assert err["rho"] <= 1e-11 and err["T"] <= 1e-13 and max(err["ux"], err["uy"]) <= 1e-12


def test_q9_thermal_box_corners_fp64(lbm, orc):
    """Temperature box with a hot corner region: diagonal populations leaving through a corner
    take the anti-bounce-back of Eq. (21)'s Dirichlet reading."""
    Tc, rl, rg = _sat(orc)
    w = evaporation(Tc, rl, rg, nx=67, ny=45, R=9.0, superheat=1.3, hot_vapour=True, thermal_q=9, flags=NO_S)
    _, _, _, _, err = _run(lbm, orc, w, 150, lbm.LBM_FP64, "D2Q9 box corners")
    assert err["rho"] <= 1e-11 and err["T"] <= 1e-13


def test_q9_every_shape_same_bits(lbm, orc):
    Tc, rl, rg = _sat(orc)
    w = boiling(Tc, rl, rg, nx=200, ny=120, hot_width=8.0, gravity=1e-4, seed=3, thermal_q=9)
    runs = []
    fits = [k for k in range(len(lbm.shapes(lbm.LBM_FP32))) if lbm.shape_fits(w.params, k)]
    assert fits and all(lbm.shapes(lbm.LBM_FP32)[k][3] == 1 for k in fits)
    for k in fits:
        print(f"[case] D2Q9 shape {k} {lbm.shapes(lbm.LBM_FP32)[k]}", flush=True)
        s = lbm.Solver(w.params).init(w.rho, w.ux, w.uy, w.T).set_shape(k)
        s.step(37)
        runs.append(s.state(absolute=False))
        s.close()
    for r in runs[1:]:
        for a, b in zip(r, runs[0]):
            assert np.array_equal(a, b)


def test_q9_batch_equals_alone_and_state_round_trip(lbm, orc):
    Tc, rl, rg = _sat(orc)
    ws = [droplet(Tc, rl, rg, nx=96, ny=80, R=16.0, thermal_q=9),
          evaporation(Tc, rl, rg, nx=130, ny=70, R=14.0, superheat=1.2, thermal_q=9),
          boiling(Tc, rl, rg, nx=128, ny=96, hot_width=8.0, seed=2, thermal_q=9)]
    steps = [40, 73, 55]
    alone = []
    for w, n in zip(ws, steps):
        s = lbm.Solver(w.params).init(w.rho, w.ux, w.uy, w.T)
        assert s.footprint >= 160 * w.params.nx * w.params.ny
        s.step(n)
        alone.append(s.fields())
        s.close()
    sols = [lbm.Solver(w.params).init(w.rho, w.ux, w.uy, w.T) for w in ws]
    b = lbm.Batch(sols)
    for i, n in enumerate(steps):
        b.set_budget(i, n)
    b.step(max(steps))
    assert b.sync() == [0, 0, 0]
    b.close()
    for s, exp in zip(sols, alone):
        for got, e in zip(s.fields(), exp):
            assert np.array_equal(got, e)
    # save / load of the 9 thermal planes resumes bit for bit
    s = sols[2]
    raw = s.save_state()
    s.step(20)
    after = s.fields()
    s.load_state(raw)
    s.step(20)
    for a, c in zip(s.fields(), after):
        assert np.array_equal(a, c)
    # a batch cannot mix thermal lattices
    w5 = droplet(Tc, rl, rg, nx=64, ny=64, R=12.0)
    s5 = lbm.Solver(w5.params).init(w5.rho, w5.ux, w5.uy, w5.T)
    with pytest.raises(lbm.LbmError):
        lbm.Batch([sols[0], s5])
    s5.close()
    for s in sols:
        s.close()
