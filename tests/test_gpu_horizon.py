"""FP32 GPU runs of the benchmark configurations at their stated sizes and horizons, against the FP64
oracle on the same seeded inputs (and, where the oracle cannot follow, against properties that hold
at any size).

  * Evaporation, 512 x 512, R = 64, edges at 1.1 T_sat, 20 000 steps, checkpoints every 2000 steps:
    L2-rel(rho) <= 1e-3, L2-rel(T) <= 1e-4 and the liquid area (r^2) within 0.5 % at every one.
  * The D^2-law set-up of Section 4.1 with the paper's values (vapour and edges at 1.0 Tc,
    lambda = 1/3): at D_0 = 20 on 64^2 the GPU's area curve stays within 0.5 % of the oracle's and
    is linear (R^2 >= 0.995, measured 0.9971 as the oracle's); at the paper's own size (D_0 = 60 on
    200^2, 600 000 steps, beyond what the oracle can follow here) the GPU alone follows the D^2 law
    with R^2 >= 0.99 (measured 0.9947: the line bends slightly more in the first tenth of the run).
  * Nucleate boiling, 1024 x 2048: as stated (pool half full, g = 2e-5) the closed box's vapour
    column is compressed past its spinodal after about 1300 steps (the oracle fails the same way,
    see the design notes), so it is compared at 500 and 1000 steps; with the head-limited fill the
    comparison runs over the first 2000 steps.  L2-rel(rho, T) <= 1e-4 at each checkpoint.  Then
    24 000 steps against the FP64 GPU path: mass, vapour fraction and mean temperature.

FP32 populations lose about 6e-8 per rounding; a step adds O(10) roundings to each population and
interfaces amplify them by O(10^2), so over thousands of steps the differences grow to the 1e-6 ..
1e-5 level and stay far below these bounds unless an operation is wrong.  L2-rel is
||GPU - oracle||_2 / ||oracle||_2 over the grid."""
import time

import numpy as np
import pytest

from workloads import Params, boiling, evaporation, head_limited_fill

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
    rl, rg, ps = orc.maxwell(base, 0.86 * Tc)
    return Tc, rl, rg, ps


def _l2rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _area(rho, rl, rg):
    """Liquid area: the excess of the density over the far-field vapour (the median), in units of
    rho_l - rho_v."""
    rv = float(np.median(rho))
    return float(np.clip((rho - rv) / (rl - rv), 0.0, 1.0).sum())


def _compare(lbm, orc, w, checkpoints, rl, rg, label, shape=None):
    s = lbm.Solver(w.params).init(w.rho, w.ux, w.uy, w.T)
    if shape is not None:
        s.set_shape(shape)
    o = orc.Oracle(w.params).init(w.rho, w.ux, w.uy, w.T)
    done, rows = 0, []
    t0 = time.perf_counter()
    for c in checkpoints:
        s.step(c - done)
        o.step(c - done)
        done = c
        g, e = s.fields(), o.fields()
        rows.append({"step": c, "rho": _l2rel(g[0], e[0]), "T": _l2rel(g[3], e[3]),
                     "area": abs(_area(g[0], rl, rg) / _area(e[0], rl, rg) - 1.0),
                     "rho_max_abs": float(np.abs(g[0] - e[0]).max()), "T_max_abs": float(np.abs(g[3] - e[3]).max())})
        r = rows[-1]
        print(f"   [{label}] step {c}: L2-rel rho {r['rho']:.2e} T {r['T']:.2e}; area {r['area']:.2e}; "
              f"max abs rho {r['rho_max_abs']:.2e} T {r['T_max_abs']:.2e} ({time.perf_counter() - t0:.0f} s)",
              flush=True)
    s.close()
    return rows


@pytest.mark.timeout(900)
def test_evaporation_config_fp32_20000_steps(lbm, orc):
    Tc, rl, rg, _ = _sat(orc)
    w = evaporation(Tc, rl, rg, nx=512, ny=512, R=64.0, superheat=1.10)
    print("\n[case] evaporation 512x512 R=64 fp32, 20000 steps vs oracle", flush=True)
    rows = _compare(lbm, orc, w, range(2000, 20001, 2000), rl, rg, "evaporation")
    for r in rows:
        assert r["rho"] <= 1e-3 and r["T"] <= 1e-4 and r["area"] <= 5e-3, r


def _d2_curve(step, fields, n_checks, every, A0, rl):
    t, a = [], []
    for _ in range(n_checks):
        step(every)
        rho = fields()
        t.append(len(t) * every + every)
        rv = float(np.median(rho))
        a.append(np.clip((rho - rv) / (rl - rv), 0, 1).sum() / A0)
        if a[-1] < 0.15:
            break
    return np.array(t), np.array(a)


def _linear_r2(t, a):
    sel = (a <= 0.9) & (a >= 0.2)
    slope, icpt = np.polyfit(t[sel], a[sel], 1)
    fit = slope * t[sel] + icpt
    return slope, 1 - ((a[sel] - fit) ** 2).sum() / ((a[sel] - a[sel].mean()) ** 2).sum(), int(sel.sum())


@pytest.mark.timeout(600)
def test_d2_law_fp32_against_oracle_and_at_the_papers_size(lbm, orc):
    Tc, rl, rg, _ = _sat(orc)
    w = evaporation(Tc, rl, rg, nx=64, ny=64, R=10.0, superheat=1.0 / 0.86, hot_vapour=True)
    A0 = np.clip((w.rho - rg) / (rl - rg), 0, 1).sum()
    print("\n[case] D^2 law 64x64 D0=20 fp32 vs oracle", flush=True)
    s = lbm.Solver(w.params).init(w.rho, w.ux, w.uy, w.T)
    o = orc.Oracle(w.params).init(w.rho, w.ux, w.uy, w.T)
    tg, ag = _d2_curve(s.step, lambda: s.fields()[0], 320, 250, A0, rl)
    to, ao = _d2_curve(o.step, lambda: o.fields()[0], len(tg), 250, A0, rl)
    s.close()
    m = min(len(ag), len(ao))
    dev = float(np.abs(ag[:m] / ao[:m] - 1).max())
    slope, r2, npts = _linear_r2(tg, ag)
    print(f"   GPU vs oracle area: max rel dev {dev:.2e}; GPU D^2 fit R^2 {r2:.5f} over {npts} points", flush=True)
    assert dev <= 5e-3
    assert slope < 0 and npts >= 100 and r2 >= 0.995
    # the paper's size: D0 = 60 on 200 x 200 (nine times the evaporation time)
    w = evaporation(Tc, rl, rg, nx=200, ny=200, R=30.0, superheat=1.0 / 0.86, hot_vapour=True)
    A0 = np.clip((w.rho - rg) / (rl - rg), 0, 1).sum()
    print("[case] D^2 law 200x200 D0=60 fp32 (GPU alone)", flush=True)
    s = lbm.Solver(w.params).init(w.rho, w.ux, w.uy, w.T)
    tg, ag = _d2_curve(s.step, lambda: s.fields()[0], 400, 2000, A0, rl)
    s.close()
    slope, r2, npts = _linear_r2(tg, ag)
    print(f"   area {ag[0]:.3f} -> {ag[-1]:.3f} over {tg[-1]} steps; D^2 fit R^2 {r2:.5f} over {npts} points",
          flush=True)
    assert slope < 0 and npts >= 50 and r2 >= 0.99  # measured 0.9947


@pytest.mark.timeout(900)
def test_boiling_config_fp32_first_steps(lbm, orc):
    Tc, rl, rg, ps = _sat(orc)
    w = boiling(Tc, rl, rg, nx=1024, ny=2048, gravity=2e-5, seed=1, fill=0.5)
    print("\n[case] boiling 1024x2048 as stated (fill 0.5) fp32 vs oracle", flush=True)
    for r in _compare(lbm, orc, w, (500, 1000), rl, rg, "boiling fill 0.5"):
        assert r["rho"] <= 1e-4 and r["T"] <= 1e-4, r
    fill = head_limited_fill(rl, rg, ps, 2e-5, 2048)
    w = boiling(Tc, rl, rg, nx=1024, ny=2048, gravity=2e-5, seed=1, fill=fill)
    # the benchmark's configuration: this workload, FP32, the 64 x 8 one-step tile shape its autotuner
    # picks (every shape gives the same bits, test_gpu_shapes.py)
    print(f"[case] boiling 1024x2048 head-limited fill {fill:.3f} fp32 (shape 2) vs oracle", flush=True)
    for r in _compare(lbm, orc, w, (500, 1000, 2000), rl, rg, "boiling head-limited", shape=2):
        assert r["rho"] <= 1e-4 and r["T"] <= 1e-4, r


def test_boiling_config_fp32_long_run_against_fp64(lbm, orc):
    """24 000 steps of the head-limited pool, FP32 against the FP64 GPU path (which matches the oracle
    to rounding wherever both run; the oracle itself would need about 15 minutes here): mass within
    1e-5 relative, vapour fraction and mean temperature within 2 %, L2-rel(rho) <= 1e-2 (the pool
    boils, so pointwise agreement decays while the integrals stay).  Later, from about step 26 000,
    a cold dense blob forms in the plume above the hot spot and rises while cooling and compressing
    until the pseudopotential is undefined near step 35 000, identically in FP32 and FP64 (a property
    of the scheme at this configuration, see the design notes), so the run stops before it."""
    Tc, rl, rg, ps = _sat(orc)
    fill = head_limited_fill(rl, rg, ps, 2e-5, 2048)
    w = boiling(Tc, rl, rg, nx=1024, ny=2048, gravity=2e-5, seed=1, fill=fill)
    print(f"\n[case] boiling 1024x2048 head-limited fill {fill:.3f}, 24000 steps, fp32 vs fp64", flush=True)
    runs = [lbm.Solver(w.params, precision=p).init(w.rho, w.ux, w.uy, w.T) for p in (lbm.LBM_FP32, lbm.LBM_FP64)]
    m0 = [s.diagnostics()[0] for s in runs]
    rmid = 0.5 * (rl + rg)
    for k in range(3):
        for s in runs:
            s.step(8000)
        (r32, _, _, T32), (r64, _, _, T64) = (s.fields() for s in runs)
        m = [s.diagnostics()[0] for s in runs]
        drift = [abs(a / b - 1) for a, b in zip(m, m0)]
        vf = [float((r < rmid).mean()) for r in (r32, r64)]
        print(f"   step {(k + 1) * 8000}: mass drift fp32 {drift[0]:.2e} fp64 {drift[1]:.2e}; vapour fraction "
              f"{vf[0]:.5f} / {vf[1]:.5f}; mean T {T32.mean() / Tc:.5f} / {T64.mean() / Tc:.5f} Tc; "
              f"L2-rel rho {_l2rel(r32, r64):.2e}; max rho {r32.max():.3f}", flush=True)
        assert drift[0] <= 1e-5 and drift[1] <= 1e-12
        assert vf[0] == pytest.approx(vf[1], rel=2e-2) and T32.mean() == pytest.approx(T64.mean(), rel=2e-2)
        assert _l2rel(r32, r64) <= 1e-2
    for s in runs:
        s.close()
