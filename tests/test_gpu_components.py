"""Vapour components labelled on the device (lbm_vapour_components, the departure readout of
Section 4.3) against the oracle's flood-fill labelling of the density that lbm_read_fields returns
for the same state: component roots, areas, bounds and row sums equal as integers.  Vapour is
decided in FP64 on both sides from the same working-precision density, so the masks are identical.

Cases: random masks (scattered and blob-like, percolating at about half vapour) on ragged grids
and row windows, FP32 and FP64; a boiling pool with a bubble, before and after departure; the state
unchanged by the labelling (it uses buffers the next step overwrites); errors and the batch guard."""
import numpy as np
import pytest

from oracle.components import vapour_components
from workloads import Params, boiling, droplet, head_limited_fill

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_00686_amd as lbm
    return lbm


@pytest.fixture(scope="module")
def sat(lbm):
    base = Params()
    Tc = lbm.critical_temperature(base)
    rl, rg, ps = lbm.coexistence(base, 0.86 * Tc)
    return Tc, rl, rg, ps


def _mask(rng, ny, nx, p, smooth):
    r = rng.random((ny, nx))
    if smooth:  # blobs: a few passes of a periodic box filter
        for _ in range(smooth):
            r = sum(np.roll(np.roll(r, dy, 0), dx, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)) / 9.0
        return r < np.quantile(r, p)
    return r < p


def _solver(lbm, sat, mask, precision):
    Tc, rl, rg, _ = sat
    ny, nx = mask.shape
    w = droplet(Tc, rl, rg, nx=nx, ny=ny, R=4.0)
    rho = np.where(mask, rg, rl)
    return lbm.Solver(w.params, precision=precision).init(rho, w.ux, w.uy, w.T)


@pytest.mark.parametrize("nx,ny,p,smooth,prec", [
    (64, 48, 0.45, 0, 0), (97, 61, 0.3, 0, 0), (150, 300, 0.5, 3, 0), (301, 77, 0.55, 1, 0),
    (256, 129, 0.45, 0, 1), (3, 5, 0.5, 0, 0), (1000, 40, 0.4, 2, 0)])
def test_random_masks_match_the_oracle(lbm, sat, nx, ny, p, smooth, prec):
    rng = np.random.default_rng(nx * 1000 + ny)
    precision = lbm.LBM_FP64 if prec else lbm.LBM_FP32
    s = _solver(lbm, sat, _mask(rng, ny, nx, p, smooth), precision)
    thr = 0.5 * (sat[1] + sat[2])
    rho = s.fields()[0]
    for lo, hi in ((0, ny), (1, ny - 1), (ny // 3, ny // 3 + 2), (ny - 1, ny)):
        if hi <= lo:
            continue
        print(f"\n[case] components {nx}x{ny} p={p} smooth={smooth} prec={prec} rows [{lo}, {hi})", flush=True)
        got = s.vapour_components(thr, lo, hi)
        exp = vapour_components(rho, thr, lo, hi)
        assert got == exp
        assert sum(c["area"] for c in got) == int((rho[lo:hi] < thr).sum())
    s.close()


def test_boiling_bubble_components_and_unchanged_state(lbm, sat):
    Tc, rl, rg, ps = sat
    thr = 0.5 * (rl + rg)
    fill = head_limited_fill(rl, rg, ps, 6e-5, 300)
    w = boiling(Tc, rl, rg, nx=150, ny=300, gravity=6e-5, dT_rel=0.19, hot_width=8.0, fill=fill, noise=0.0)
    print("\n[case] boiling 150x300 g=6e-5: components every 1000 steps vs oracle labelling", flush=True)
    a = lbm.Solver(w.params).init(w.rho, w.ux, w.uy, w.T)
    b = lbm.Solver(w.params).init(w.rho, w.ux, w.uy, w.T)
    y_surface = int(fill * 300) - 12
    seen_departed = False
    for k in range(16):
        a.step(1000)
        b.step(1000)
        got = a.vapour_components(thr, 0, y_surface + 1)
        rho = b.fields()[0]  # the field of the run that was never labelled
        assert got == vapour_components(rho, thr, 0, y_surface + 1)
        inner = [c for c in got if c["y_min"] > 0 and c["y_max"] < y_surface]
        seen_departed = seen_departed or bool(inner)
    fa, ga, ha = a.state(absolute=False)
    fb, gb, hb = b.state(absolute=False)
    assert np.array_equal(fa, fb) and np.array_equal(ga, gb) and np.array_equal(ha, hb)
    assert seen_departed  # the bubble left the wall within the 16 000 steps (it does near 13 750)
    a.close()
    b.close()


def test_errors_and_the_batch_guard(lbm, sat):
    Tc, rl, rg, _ = sat
    thr = 0.5 * (rl + rg)
    w = droplet(Tc, rl, rg, nx=64, ny=40, R=8.0)
    s = lbm.Solver(w.params).init(w.rho, w.ux, w.uy, w.T)
    t = lbm.Solver(w.params).init(w.rho, w.ux, w.uy, w.T)
    print("\n[case] component errors and batch guard", flush=True)
    for lo, hi in ((-1, 10), (0, 41), (10, 10), (12, 5)):
        with pytest.raises(lbm.LbmError) as e:
            s.vapour_components(thr, lo, hi)
        assert e.value.status == -1  # LBM_E_INVAL
    with pytest.raises(lbm.LbmError):
        s.vapour_components(float("nan"))
    assert len(s.vapour_components(thr)) == 1
    b = lbm.Batch([s, t])
    b.set_budget(0, 10)
    b.set_budget(1, 10)
    b.step(10)
    for call in (lambda: s.vapour_components(thr), s.fields, lambda: s.step(1), s.diagnostics, s.save_state):
        with pytest.raises(lbm.LbmError) as e:
            call()
        assert e.value.status == -5  # LBM_E_STATE
    assert b.sync() == [0, 0]
    assert len(s.vapour_components(thr)) == 1
    b.set_budget(0, 5)
    b.step(5)
    b.close()  # brings the members up to date first
    assert s.steps == 15 and t.steps == 10
    s.fields()
    s.close()
    t.close()
