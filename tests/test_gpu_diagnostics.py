"""Diagnostics every k steps (FP64 mass and thermal energy, deterministic wavefront-shuffle
reduction enqueued by lbm_step between launches): the records land at the multiples of k, equal
the on-demand lbm_diagnostics at those steps bit for bit, match the FP64 oracle's mass and energy
(relative 1e-13 and 1e-12: both sum FP64 populations that agree to rounding, in different orders),
and leave the simulation's bits unchanged."""
import numpy as np
import pytest

from workloads import Params, boiling, heated_droplet

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_00686_amd as lbm
    return lbm


def _raw(s):
    f, g, h = s.state(absolute=False)
    return np.concatenate([f.ravel(), g.ravel(), h.ravel()])


@pytest.mark.parametrize("k,calls", [(50, (537,)), (130, (100, 333, 2))])
@pytest.mark.parametrize("kind", ["boiling", "open_top"])
def test_every_k_diagnostics(lbm, orc, k, calls, kind):
    base = Params()
    Tc = orc.Tc(base)
    rl, rg, _ = orc.maxwell(base, 0.86 * Tc)
    if kind == "boiling":
        w = boiling(Tc, rl, rg, nx=96, ny=80, gravity=5e-5, hot_width=6.0, seed=3)
    else:
        w = heated_droplet(Tc, rl, rg, nx=80, ny=48, R=14.0, T_h_rel=0.95, gy=-5e-5)
    print(f"\n[case] diagnostics every {k} steps, calls {calls}, {kind}", flush=True)
    total = sum(calls)
    marks = list(range(k, total + 1, k))
    # the logged run (FP64)
    s = lbm.Solver(w.params, precision=lbm.LBM_FP64).init(w.rho, w.ux, w.uy, w.T)
    s.set_diagnostics_interval(k)
    for n in calls:
        s.step(n)
    log = s.diagnostics_log()
    assert [r[0] for r in log] == marks
    # the same run without the log, with on-demand diagnostics at the marks
    t = lbm.Solver(w.params, precision=lbm.LBM_FP64).init(w.rho, w.ux, w.uy, w.T)
    o = orc.Oracle(w.params).init(w.rho, w.ux, w.uy, w.T)
    done = 0
    for (step, m, e) in log:
        t.step(step - done)
        o.step(step - done)
        done = step
        mt, et = t.diagnostics()
        assert (m, e) == (mt, et)
        mo, eo, _, _ = o.diagnostics()
        assert m == pytest.approx(mo, rel=1e-13) and e == pytest.approx(eo, rel=1e-12)
    t.step(total - done)
    assert np.array_equal(_raw(s), _raw(t))
    if kind == "open_top":
        assert abs(log[-1][1] - log[0][1]) > 1e-9 * log[0][1]  # mass crosses the open top
    # the log was read: the next read is empty; k = 0 stops it
    assert s.diagnostics_log() == []
    s.set_diagnostics_interval(0)
    s.step(3 * k)
    assert s.diagnostics_log() == []
    s.close()
    t.close()


@pytest.mark.parametrize("persistent", [False, True])
def test_batch_diagnostics_every_k(lbm, orc, persistent):
    """Every-k diagnostics of batch members: records at multiples of k batch steps, where a member's
    budget ends inside an interval, and where the last budget ends; each equals lbm_diagnostics of
    the member run alone to that step, bit for bit; the members' results are unchanged."""
    base = Params()
    Tc = orc.Tc(base)
    rl, rg, _ = orc.maxwell(base, 0.86 * Tc)
    ws = [boiling(Tc, rl, rg, nx=96, ny=80, gravity=5e-5, hot_width=6.0, seed=3),
          heated_droplet(Tc, rl, rg, nx=80, ny=48, R=14.0, T_h_rel=0.95, gy=-5e-5),
          boiling(Tc, rl, rg, nx=130, ny=70, gravity=3e-5, hot_width=5.0, seed=5)]
    budgets, k = (260, 123, 310), 50
    print(f"\n[case] batch diagnostics every {k}, budgets {budgets}, persistent {persistent}", flush=True)
    sols = [lbm.Solver(w.params).init(w.rho, w.ux, w.uy, w.T) for w in ws]
    b = lbm.Batch(sols).set_persistent(persistent).set_diagnostics_interval(k)
    for i, n in enumerate(budgets):
        b.set_budget(i, n)
    b.step(70)
    b.step(max(budgets))
    assert b.sync() == [0, 0, 0]
    for i, (w, n) in enumerate(zip(ws, budgets)):
        log = sols[i].diagnostics_log()
        expect = list(range(k, n + 1, k)) + ([n] if n % k else [])
        assert [r[0] for r in log] == expect, (i, [r[0] for r in log])
        alone = lbm.Solver(w.params).init(w.rho, w.ux, w.uy, w.T)
        done = 0
        for step, m, e in log:
            alone.step(step - done)
            done = step
            assert (m, e) == alone.diagnostics(), (i, step)
        assert np.array_equal(_raw(alone), _raw(sols[i]))
        alone.close()
    b.close()
    for s in sols:
        s.close()
