"""Device vapour-row counts of the bubble-departure readout: exact agreement with counts from
the field readout (the density compared with the threshold in the working precision), for
windows that wrap around the periodic x boundary, in FP32 and FP64."""
import numpy as np
import pytest

from workloads import Params, boiling, evaporation

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_00686_amd as lbm
    return lbm


def test_vapour_rows_match_field_readout(lbm):
    base = Params()
    Tc = lbm.critical_temperature(base)
    rl, rg, _ = lbm.coexistence(base, 0.86 * Tc)
    thr = 0.5 * (rl + rg)
    cases = [(evaporation(Tc, rl, rg, nx=200, ny=130, R=30.0), lbm.LBM_FP32, np.float32),
             (boiling(Tc, rl, rg, nx=150, ny=120, hot_width=2.0, dT_rel=0.19, gravity=3e-5), lbm.LBM_FP32, np.float32),
             (evaporation(Tc, rl, rg, nx=90, ny=70, R=14.0), lbm.LBM_FP64, np.float64)]
    for w, prec, dt in cases:
        nx = w.params.nx
        s = lbm.Solver(w.params, precision=prec).init(w.rho, w.ux, w.uy, w.T)
        s.step(60)
        rho = s.fields()[0].astype(dt)
        for lo, hi in ((0, nx), (nx // 2, nx // 2 + nx // 3), (nx - 10, nx + 25), (-17, 40)):
            print(f"\n[case] vapour rows {nx}x{w.params.ny} window [{lo}, {hi})", flush=True)
            got = s.vapour_rows(thr, lo, hi)
            cols = np.arange(lo, hi) % nx
            exp = (rho[:, cols] < dt(thr)).sum(axis=1)
            assert np.array_equal(got, exp.astype(np.int32))
        assert s.vapour_rows(thr).sum() > 0
        for lo, hi in ((5, 5), (0, nx + 1)):
            with pytest.raises(lbm.LbmError):
                s.vapour_rows(thr, lo, hi)
        s.close()


def test_departure_diameter_follows_fritz(lbm):
    """The paper's boiling study (Section 4.3): bubbles departing from a heated spot have
    D_d ~ g^(-1/2).  Three gravities of the sweep, first departure each, one batch."""
    from paper_2205_00686_amd import fritz
    from workloads import head_limited_fill

    base = Params()
    Tc = lbm.critical_temperature(base)
    rl, rg, ps = lbm.coexistence(base, 0.86 * Tc)
    gs = (3e-5, 4e-5, 6e-5)
    fill = head_limited_fill(rl, rg, ps, 6e-5, 300)
    ws = [boiling(Tc, rl, rg, nx=150, ny=300, gravity=g, dT_rel=0.19, hot_width=8.0, fill=fill, noise=0.0)
          for g in gs]
    print("\n[case] departure sweep 150x300, g = 3e-5, 4e-5, 6e-5", flush=True)
    res = fritz.sweep(ws, rl, rg, max_steps=40000, check_every=250)
    for r in res:
        print(f"   g {r.gravity:.1e}: step {r.step}, D {r.diameter:.1f}", flush=True)
    assert all(r.step > 0 for r in res)
    assert res[0].diameter > res[1].diameter > res[2].diameter
    slope, _, r2 = fritz.fit_power([r.gravity for r in res], [r.diameter for r in res])
    print(f"   slope {slope:.3f}, R^2 {r2:.4f}", flush=True)
    assert -0.6 <= slope <= -0.4 and r2 >= 0.98
