"""Continuous-batching server: every request's result is bit-identical to running it alone, also
when admission is limited by the HBM budget and requests join while others run, under either
admission order; a failing request does not disturb the others."""
import numpy as np
import pytest

from workloads import Params, boiling, droplet, evaporation

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_00686_amd as lbm
    return lbm


def _mix(lbm):
    base = Params()
    Tc = lbm.critical_temperature(base)
    rl, rg, _ = lbm.coexistence(base, 0.86 * Tc)
    return [
        (0.00, 300, lambda: droplet(Tc, rl, rg, nx=96, ny=80, R=20.0)),
        (0.00, 130, lambda: evaporation(Tc, rl, rg, nx=128, ny=100, R=16.0, superheat=1.2)),
        (0.01, 257, lambda: boiling(Tc, rl, rg, nx=130, ny=140, hot_width=8.0, seed=4)),
        (0.02, 64, lambda: droplet(Tc, rl, rg, nx=70, ny=70, R=12.0)),
        (0.02, 190, lambda: boiling(Tc, rl, rg, nx=64, ny=200, gravity=4e-5, hot_width=6.0, seed=5)),
        (0.03, 75, lambda: evaporation(Tc, rl, rg, nx=90, ny=90, R=12.0, superheat=1.3, hot_vapour=True)),
    ]


@pytest.mark.parametrize("policy", ["arrival", "shortest"])
def test_served_results_equal_alone(lbm, policy):
    from paper_2205_00686_amd import serve
    mix = _mix(lbm)
    alone = []
    for _, steps, make in mix:
        w = make()
        s = lbm.Solver(w.params).init(w.rho, w.ux, w.uy, w.T)
        s.step(steps)
        alone.append(s.fields())
        s.close()
    # budget for about three of these at once: admission waits, later requests join mid-run
    fp = max(lbm.footprint_bytes(make().params) for _, _, make in mix)
    server = serve.Server(hbm_budget=3 * fp, max_slots=3, chunk=64, policy=policy)
    reqs = [serve.Request(rid=i, arrival=a, steps=n, make=m) for i, (a, n, m) in enumerate(mix)]
    done, summary = server.run(reqs, realtime=False)
    print(f"\n[case] serve mix, {policy} admission:", summary, flush=True)
    assert summary["completed"] == len(mix)
    for r in done:
        for got, exp in zip(r.result, alone[r.rid]):
            assert np.array_equal(got, exp), r.rid
    # FIFO baseline gives the same bits too
    reqs = [serve.Request(rid=i, arrival=a, steps=n, make=m) for i, (a, n, m) in enumerate(mix)]
    done, _ = serve.fifo(reqs, realtime=False)
    for r in done:
        for got, exp in zip(r.result, alone[r.rid]):
            assert np.array_equal(got, exp), r.rid


def test_failing_request_is_isolated(lbm):
    from paper_2205_00686_amd import serve
    base = Params()
    Tc = lbm.critical_temperature(base)
    rl, rg, _ = lbm.coexistence(base, 0.86 * Tc)
    good = lambda: droplet(Tc, rl, rg, nx=64, ny=64, R=14.0)  # noqa: E731
    bad = lambda: droplet(Tc, rl, rg, nx=64, ny=64, R=14.0, cv=0.1)  # noqa: E731  (rho c_v < 1: rejected)
    reqs = [serve.Request(rid=0, arrival=0.0, steps=100, make=good),
            serve.Request(rid=1, arrival=0.0, steps=100, make=bad),
            serve.Request(rid=2, arrival=0.0, steps=150, make=good)]
    done, summary = serve.Server(hbm_budget=1 << 30, max_slots=4, chunk=64).run(reqs, realtime=False)
    assert summary["completed"] == 2 and summary["failed"] == 1
    assert done[1].error is not None and done[0].error is None and done[2].error is None
    w = good()
    s = lbm.Solver(w.params).init(w.rho, w.ux, w.uy, w.T)
    s.step(150)
    assert np.array_equal(s.fields()[0], done[2].result[0])


def test_batch_orders_member_streams(lbm):
    """Members initialised on streams of their own, batched on a third stream and, after the
    batch is gone, advanced on their own streams again: same bits as one stream throughout."""
    import torch
    base = Params()
    Tc = lbm.critical_temperature(base)
    rl, rg, _ = lbm.coexistence(base, 0.86 * Tc)
    makes = [lambda: evaporation(Tc, rl, rg, nx=160, ny=120, R=20.0, superheat=1.2),
             lambda: boiling(Tc, rl, rg, nx=128, ny=160, hot_width=8.0, seed=9)]
    alone = []
    for make in makes:
        w = make()
        s = lbm.Solver(w.params).init(w.rho, w.ux, w.uy, w.T)
        s.step(90)
        s.step(33)
        alone.append(s.fields())
        s.close()
    streams = [torch.cuda.Stream() for _ in makes]
    sols = []
    for make, st in zip(makes, streams):
        w = make()
        sols.append(lbm.Solver(w.params, stream=st).init(w.rho, w.ux, w.uy, w.T))
    b = lbm.Batch(sols, stream=torch.cuda.Stream())
    for i in range(len(sols)):
        b.set_budget(i, 90)
    b.step(90)
    assert b.sync() == [0] * len(sols)
    b.close()
    for s in sols:
        s.step(33)
    for s, exp in zip(sols, alone):
        assert s.steps == 123
        for got, e in zip(s.fields(), exp):
            assert np.array_equal(got, e)
    # members may be destroyed before their batch once it is synchronised
    b = lbm.Batch(sols)
    b.sync()
    for s in sols:
        s.close()
    b.close()
