"""Persistent batched launches (one kernel per group of steps, grid barriers between launches):
bit-identical to the launch-per-step batch for uneven members, budgets and tile shapes, including
open-top members (whose boundary pass runs between two barriers) and FP64; and a barrier wait
forced to time out from the host (a spin limit of one poll) ends every workgroup normally and is
reported as a device failure of every member, after which the GPU serves new work."""
import numpy as np
import pytest

from workloads import Params, boiling, droplet, evaporation, heated_droplet

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_00686_amd as lbm
    return lbm


def _sat(lbm):
    base = Params()
    Tc = lbm.critical_temperature(base)
    rl, rg, _ = lbm.coexistence(base, 0.86 * Tc)
    return Tc, rl, rg


def _raw(s):
    f, g, h = s.state(absolute=False)
    return np.concatenate([f.ravel(), g.ravel(), h.ravel()])


def _run(lbm, ws, budgets, persistent, shape=None, precision=0):
    sols = [lbm.Solver(w.params, precision=precision).init(w.rho, w.ux, w.uy, w.T) for w in ws]
    b = lbm.Batch(sols)
    if shape is not None:
        b.set_shape(shape)
    if persistent:
        b.set_persistent(True)
    for i, n in enumerate(budgets):
        b.set_budget(i, n)
    b.step(70)
    b.step(max(budgets))
    assert b.sync() == [0] * len(ws)
    b.close()
    out = [_raw(s) for s in sols]
    for s, n in zip(sols, budgets):
        assert s.steps == n
        s.close()
    return out


@pytest.mark.parametrize("shape,precision", [(6, 0), (2, 0), (0, 1)])
def test_persistent_equals_launch_per_step(lbm, shape, precision):
    Tc, rl, rg = _sat(lbm)
    ws = [boiling(Tc, rl, rg, nx=160, ny=96, gravity=3e-5, dT_rel=0.25, hot_width=8.0, seed=1),
          evaporation(Tc, rl, rg, nx=100, ny=80, R=15.0, superheat=1.15),
          droplet(Tc, rl, rg, nx=96, ny=64, R=16.0)]
    if shape != 6:  # an open-top member (one-step shapes only)
        ws.append(heated_droplet(Tc, rl, rg, nx=90, ny=48, R=14.0, T_h_rel=0.95, gy=-5e-5))
    budgets = [150, 97, 64, 131][:len(ws)]
    print(f"\n[case] persistent vs launch-per-step, shape {shape}, precision {precision}", flush=True)
    ref = _run(lbm, ws, budgets, False, shape, precision)
    got = _run(lbm, ws, budgets, True, shape, precision)
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)


def test_persistent_barrier_timeout_is_reported(lbm):
    Tc, rl, rg = _sat(lbm)
    print("\n[case] persistent barrier forced to time out (spin limit 1)", flush=True)
    ws = [boiling(Tc, rl, rg, nx=512, ny=256, gravity=2e-5, hot_width=8.0, seed=2, fill=0.7)]
    sols = [lbm.Solver(w.params).init(w.rho, w.ux, w.uy, w.T) for w in ws]
    b = lbm.Batch(sols).set_persistent(True, spin_limit=1)
    b.set_budget(0, 64)
    b.step(64)
    with pytest.raises(lbm.LbmError) as e:
        b.sync()
    assert e.value.status == -3
    with pytest.raises(lbm.LbmError) as e:
        sols[0].step(1)
    assert e.value.status == -5
    b.close()
    sols[0].close()
    # the device serves new work: a healthy persistent batch afterwards
    sols = [lbm.Solver(w.params).init(w.rho, w.ux, w.uy, w.T) for w in ws]
    b = lbm.Batch(sols).set_persistent(True)
    b.set_budget(0, 64)
    b.step(64)
    assert b.sync() == [0]
    b.close()
    sols[0].close()
