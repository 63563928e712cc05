"""GPU parity of the open top boundary (outflow condition of the paper's open-top problems,
Sections 4.2-4.3) against the FP64 oracle through the C ABI: the heated-surface droplet and an
open-top boiling pool, FP64 to rounding and FP32 to the bounds of the other parity tests (rho
within 2e-4 rho_l after 300 steps, T within 2e-6 relative, u within 1e-5); the smallest and
ragged grids from random fields in FP64; every one-step tile shape gives the same bits; save/load
resumes bit for bit; a batch with open-top members equals their single runs."""
import numpy as np
import pytest

from workloads import Params, boiling, droplet, heated_droplet

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


def _cases(orc):
    Tc, rl, rg = _sat(orc)
    return {
        "heated_droplet": heated_droplet(Tc, rl, rg, nx=150, ny=70, R=22.0, T_h_rel=0.95),
        "open_boiling": boiling(Tc, rl, rg, nx=140, ny=84, hot_width=8.0, dT_rel=0.2, gravity=1e-4, seed=11,
                                fill=0.6, open_top=1),
        "heated_droplet_q9": heated_droplet(Tc, rl, rg, nx=96, ny=64, R=18.0, T_h_rel=0.95, thermal_q=9),
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


@pytest.mark.parametrize("kind", ["heated_droplet", "open_boiling", "heated_droplet_q9"])
def test_open_top_fp64_matches_oracle(lbm, orc, kind):
    w = _cases(orc)[kind]
    s, ref, got, exp, err = _run(lbm, orc, w, 300, lbm.LBM_FP64, kind)
    assert err["rho"] <= 1e-11 and err["T"] <= 1e-13 and max(err["ux"], err["uy"]) <= 1e-13
    fg, gg, hg = s.state()
    fo, go, ho = ref.state()
    assert np.abs(fg - fo).max() <= 1e-11 and np.abs(gg - go).max() <= 1e-13
    # mass really crosses the open top in these runs
    m, _ = s.diagnostics()
    assert abs(m - float(w.rho.sum())) > 1e-9 * float(w.rho.sum())
    s.close()


@pytest.mark.parametrize("kind", ["heated_droplet", "open_boiling"])
def test_open_top_fp32_matches_oracle(lbm, orc, kind):
    w = _cases(orc)[kind]
    s, _, got, exp, err = _run(lbm, orc, w, 300, lbm.LBM_FP32, kind)
    Tmax = float(np.abs(exp[3]).max())
    assert err["rho"] <= 2e-4 * 6.5 and err["T"] <= 2e-6 * Tmax and max(err["ux"], err["uy"]) <= 1e-5
    s.close()


def test_open_top_every_shape_same_bits_and_resume(lbm, orc):
    w = _cases(orc)["open_boiling"]
    fits = [k for k in range(len(lbm.shapes(lbm.LBM_FP32))) if lbm.shape_fits(w.params, k)]
    assert fits and all(lbm.shapes(lbm.LBM_FP32)[k][3] == 1 for k in fits)
    runs = []
    for k in fits:
        print(f"[case] open top shape {k} {lbm.shapes(lbm.LBM_FP32)[k]}", flush=True)
        s = lbm.Solver(w.params).init(w.rho, w.ux, w.uy, w.T).set_shape(k)
        s.step(100)  # more than one graph of steps
        runs.append(s.state(absolute=False))
        if k == fits[-1]:
            raw = s.save_state()
            s.step(21)
            after = s.fields()
            s.load_state(raw)
            s.step(21)
            for a, b in zip(s.fields(), after):
                assert np.array_equal(a, b)
        s.close()
    for r in runs[1:]:
        for a, b in zip(r, runs[0]):
            assert np.array_equal(a, b)


def test_batch_with_open_top_members_equals_alone(lbm, orc):
    """A batch mixing closed and open-top members (one-step launches, the boundary pass over
    every table entry that has an open top): each member's bits equal its single run."""
    Tc, rl, rg = _sat(orc)
    ws = [droplet(Tc, rl, rg, nx=64, ny=64, R=12.0),
          heated_droplet(Tc, rl, rg, nx=96, ny=48, R=14.0),
          boiling(Tc, rl, rg, nx=128, ny=96, hot_width=8.0, seed=2, fill=0.7, open_top=1)]
    steps = [50, 90, 71]
    alone = []
    for w, n in zip(ws, steps):
        s = lbm.Solver(w.params).init(w.rho, w.ux, w.uy, w.T)
        s.step(n)
        alone.append(s.fields())
        s.close()
    sols = [lbm.Solver(w.params).init(w.rho, w.ux, w.uy, w.T) for w in ws]
    b = lbm.Batch(sols)
    assert lbm.shapes(lbm.LBM_FP32)[b.shape][3] == 1
    for i, n in enumerate(steps):
        b.set_budget(i, n)
    b.step(max(steps))
    assert b.sync() == [0, 0, 0]
    b.close()
    for s, exp in zip(sols, alone):
        for got, e in zip(s.fields(), exp):
            assert np.array_equal(got, e)
        s.close()


@pytest.mark.parametrize("nx,ny", [(3, 3), (5, 4), (65, 17), (200, 3), (130, 23)])
def test_open_top_fp64_small_and_ragged_grids(lbm, orc, nx, ny):
    """Open top on the smallest grids (three rows: the wall row, one fluid row, the open row) and on
    ragged multi-tile grids, from random fields with gravity and a hot spot: FP64 to rounding."""
    Tc, rl, rg = _sat(orc)
    rng = np.random.default_rng(nx * 1000 + ny)
    rho = rg + (rl - rg) * rng.uniform(0.0, 1.0, (ny, nx))
    T = 0.86 * Tc * (1 + 0.01 * rng.uniform(-1, 1, (ny, nx)))
    ux = 0.01 * rng.standard_normal((ny, nx))
    uy = 0.01 * rng.standard_normal((ny, nx))
    p = Params(nx=nx, ny=ny, y_walls=1, open_top=1, T_bot=0.9 * Tc, T_top=0.85 * Tc, hot_dT=0.05 * Tc,
               hot_x0=nx / 3, hot_sigma=2.0, theta_bot_deg=70.0, theta_top_deg=100.0, gy=-1e-4)
    from workloads import Workload
    w = Workload("random open top", p, rho, ux, uy, T, 20)
    _, _, got, exp, err = _run(lbm, orc, w, 20, lbm.LBM_FP64, f"random open top {nx}x{ny}")
    assert err["rho"] <= 1e-11 and err["T"] <= 1e-13 and max(err["ux"], err["uy"]) <= 1e-12
