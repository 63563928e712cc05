"""FP32 GPU runs against the FP64 oracle over long horizons, on scaled-down versions of the
benchmark workloads (default tile shape: two steps per launch where the grid allows).

Tolerances (stated per workload, measured values printed beside them):
  evaporation 256 x 256, 4000 steps: L2-rel(rho) <= 1e-3, L2-rel(T) <= 1e-4, droplet area within
      0.5 % at every checkpoint, total mass drift (FP64 sum) <= 1e-6 relative;
  boiling 256 x 512 (walls, gravity, hot spot), 2000 steps: L2-rel(rho) <= 1e-4, L2-rel(T) <= 1e-4
      at every checkpoint, mass drift <= 1e-6.
FP32 populations lose about 6e-8 per rounding; a step adds O(10) roundings to each population and
interfaces amplify them by O(10^2), so over thousands of steps the differences grow to the 1e-5
level and stay far below these bounds unless an operation is wrong.
"""
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


def _l2rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _area(rho, rl, rg):
    return float(np.clip((rho - rg) / (rl - rg), 0.0, 1.0).sum())


def _compare(lbm, orc, w, checkpoints, rl, rg):
    s = lbm.Solver(w.params).init(w.rho, w.ux, w.uy, w.T)
    o = orc.Oracle(w.params).init(w.rho, w.ux, w.uy, w.T)
    m0, _ = s.diagnostics()
    done = 0
    rows = []
    for c in checkpoints:
        s.step(c - done)
        o.step(c - done)
        done = c
        g, e = s.fields(), o.fields()
        rows.append({"step": c, "rho": _l2rel(g[0], e[0]), "T": _l2rel(g[3], e[3]),
                     "area": abs(_area(g[0], rl, rg) / _area(e[0], rl, rg) - 1.0),
                     "rho_max_abs": float(np.abs(g[0] - e[0]).max()), "T_max_abs": float(np.abs(g[3] - e[3]).max())})
        r = rows[-1]
        print(f"   step {c}: L2-rel rho {r['rho']:.2e} T {r['T']:.2e}; area {r['area']:.2e}; "
              f"max abs rho {r['rho_max_abs']:.2e} T {r['T_max_abs']:.2e}", flush=True)
    m1, _ = s.diagnostics()
    drift = abs(m1 - m0) / m0
    print(f"   mass drift {drift:.2e}, tile shape {lbm.shapes(lbm.LBM_FP32)[s.shape]}", flush=True)
    s.close()
    return rows, drift


def test_evaporation_fp32_long_horizon(lbm, orc):
    base = Params()
    Tc = orc.Tc(base)
    rl, rg, _ = orc.maxwell(base, 0.86 * Tc)
    w = evaporation(Tc, rl, rg, nx=256, ny=256, R=32.0, superheat=1.10)
    print("\n[case] evaporation 256x256 fp32 4000 steps vs oracle", flush=True)
    rows, drift = _compare(lbm, orc, w, (1000, 2000, 3000, 4000), rl, rg)
    for r in rows:
        assert r["rho"] <= 1e-3 and r["T"] <= 1e-4 and r["area"] <= 5e-3, r
    assert drift <= 1e-6


def test_boiling_fp32_long_horizon(lbm, orc):
    base = Params()
    Tc = orc.Tc(base)
    rl, rg, ps = orc.maxwell(base, 0.86 * Tc)
    fill = head_limited_fill(rl, rg, ps, 2e-5, 512)
    w = boiling(Tc, rl, rg, nx=256, ny=512, hot_width=8.0, gravity=2e-5, fill=fill, seed=21)
    print(f"\n[case] boiling 256x512 (fill {fill:.3f}) fp32 2000 steps vs oracle", flush=True)
    rows, drift = _compare(lbm, orc, w, (500, 1000, 2000), rl, rg)
    for r in rows:
        assert r["rho"] <= 1e-4 and r["T"] <= 1e-4, r
    assert drift <= 1e-6
