"""Tile shapes of the step kernel and their autotuner: every shape gives bit-identical results
(single runs, a shape change in mid-run, batches), and tuning restores the simulation's state
exactly and records its choice."""
import json

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


@pytest.fixture(scope="module")
def sat(lbm):
    base = Params()
    Tc = lbm.critical_temperature(base)
    rl, rg, _ = lbm.coexistence(base, 0.86 * Tc)
    return Tc, rl, rg


def _cases(sat, lbm):
    Tc, rl, rg = sat
    return [
        ("evaporation 200x130 FP32", evaporation(Tc, rl, rg, nx=200, ny=130, R=30.0), lbm.LBM_FP32, 100),
        ("boiling 300x200 FP32", boiling(Tc, rl, rg, nx=300, ny=200, hot_width=10.0, gravity=3e-5), lbm.LBM_FP32, 100),
        ("droplet 40x36 FP32", droplet(Tc, rl, rg, nx=40, ny=36, R=9.0), lbm.LBM_FP32, 70),
        ("droplet 70x50 FP64", droplet(Tc, rl, rg, nx=70, ny=50, R=12.0), lbm.LBM_FP64, 100),
        ("boiling 130x70 FP64", boiling(Tc, rl, rg, nx=130, ny=70, hot_width=6.0, gravity=3e-5), lbm.LBM_FP64, 70),
    ]


def _run(lbm, w, prec, n, shape):
    s = lbm.Solver(w.params, precision=prec).init(w.rho, w.ux, w.uy, w.T)
    s.set_shape(shape)
    assert s.shape == shape
    s.step(n)
    s.sync()
    out = s.save_state()
    s.close()
    return out


def test_every_shape_gives_identical_bits(lbm, sat):
    for name, w, prec, n in _cases(sat, lbm):
        ref = _run(lbm, w, prec, n, 0)
        for k in range(1, len(lbm.shapes(prec))):
            if not lbm.shape_fits(w.params, k, prec):
                continue
            print(f"\n[case] {name} shape {k} {lbm.shapes(prec)[k]}", flush=True)
            assert _run(lbm, w, prec, n, k) == ref, (name, k)
            assert _run(lbm, w, prec, n + 1, k) == _run(lbm, w, prec, n + 1, 0), (name, k, "odd")


def test_shapes_identical_on_grids_of_many_workgroup_waves(lbm, sat):
    """More tiles than the GPU holds at once: workgroups of later waves read halos that earlier
    workgroups of the same launch have finished with (regression: the temperature history of a
    neighbour's nodes must not be overwritten within a launch)."""
    Tc, rl, rg = sat
    for name, w in (("evaporation 1024x512", evaporation(Tc, rl, rg, nx=1024, ny=512, R=100.0)),
                    ("boiling 512x1024", boiling(Tc, rl, rg, nx=512, ny=1024, hot_width=16.0))):
        ref = _run(lbm, w, lbm.LBM_FP32, 7, 0)
        for k in range(1, len(lbm.shapes(lbm.LBM_FP32))):
            print(f"\n[case] {name} shape {k}", flush=True)
            assert _run(lbm, w, lbm.LBM_FP32, 7, k) == ref, (name, k)


def test_two_step_shape_rejected_on_small_grid(lbm, sat):
    Tc, rl, rg = sat
    w = droplet(Tc, rl, rg, nx=40, ny=36, R=9.0)
    two = [k for k, sh in enumerate(lbm.shapes(lbm.LBM_FP32)) if sh[3] == 2]
    s = lbm.Solver(w.params).init(w.rho, w.ux, w.uy, w.T)
    for k in two:
        assert not lbm.shape_fits(w.params, k)
        with pytest.raises(lbm.LbmError) as e:
            s.set_shape(k)
        assert e.value.status == -1
    s.close()


def test_shape_change_mid_run(lbm, sat):
    Tc, rl, rg = sat
    w = boiling(Tc, rl, rg, nx=256, ny=160, hot_width=10.0, gravity=3e-5)
    ref = _run(lbm, w, lbm.LBM_FP32, 150, 0)
    s = lbm.Solver(w.params).init(w.rho, w.ux, w.uy, w.T)
    assert s.shape in range(len(lbm.shapes(lbm.LBM_FP32)))
    s.set_shape(3).step(70)
    s.set_shape(6).step(33)   # two steps per launch, odd count: the last launch does one
    s.set_shape(4).step(3)
    s.set_shape(7).step(1)
    s.set_shape(6).step(2)
    s.set_shape(-1).step(41)
    s.sync()
    assert s.steps == 150
    assert s.save_state() == ref
    s.close()


def test_batch_shapes_give_identical_bits(lbm, sat):
    Tc, rl, rg = sat
    ws = [evaporation(Tc, rl, rg, nx=200, ny=130, R=30.0),
          boiling(Tc, rl, rg, nx=300, ny=200, hot_width=10.0, gravity=3e-5),
          droplet(Tc, rl, rg, nx=96, ny=80, R=20.0)]
    budgets = [91, 60, 33]  # uneven and odd: two-step launches end some members with one step
    alone = [_run(lbm, w, lbm.LBM_FP32, n, 0) for w, n in zip(ws, budgets)]
    for k in range(len(lbm.shapes(lbm.LBM_FP32))):
        print(f"\n[case] batch shape {k}", flush=True)
        sol = [lbm.Solver(w.params).init(w.rho, w.ux, w.uy, w.T) for w in ws]
        b = lbm.Batch(sol).set_shape(k)
        assert b.shape == k
        for i, n in enumerate(budgets):
            b.set_budget(i, n)
        b.step(45)
        b.step(7)
        b.step(100)
        assert b.sync() == [0] * len(sol)
        b.close()
        for s, ref, n in zip(sol, alone, budgets):
            assert s.steps == n
            assert s.save_state() == ref, k
            s.close()


def test_autotune_solver_restores_state_and_caches(lbm, sat, tmp_path, monkeypatch):
    from paper_2205_00686_amd import autotune
    monkeypatch.setenv("LBM_SHAPE_CACHE", str(tmp_path / "shapes.json"))
    Tc, rl, rg = sat
    w = evaporation(Tc, rl, rg, nx=256, ny=192, R=40.0)
    s = lbm.Solver(w.params).init(w.rho, w.ux, w.uy, w.T)
    s.step(37)
    before = s.save_state()
    res = autotune.tune_solver(s, steps=16, repeats=2)
    print("\n[case] autotune solver", res, flush=True)
    assert not res.cached and res.shape == s.shape
    assert set(res.ms_per_step) == set(range(len(lbm.shapes(lbm.LBM_FP32))))
    assert all(v > 0 for v in res.ms_per_step.values())
    assert s.steps == 37 and s.save_state() == before
    # continuing after tuning gives the same bits as never tuning
    s.step(40)
    ref = lbm.Solver(w.params).init(w.rho, w.ux, w.uy, w.T)
    ref.step(77)
    assert s.save_state() == ref.save_state()
    data = json.load(open(tmp_path / "shapes.json"))
    assert data[res.key]["shape"] == res.shape
    s2 = lbm.Solver(w.params).init(w.rho, w.ux, w.uy, w.T)
    again = autotune.tune_solver(s2)
    assert again.cached and again.shape == res.shape and s2.shape == res.shape
    for x in (s, ref, s2):
        x.close()


def test_autotune_batch_leaves_members_untouched(lbm, sat, tmp_path, monkeypatch):
    from paper_2205_00686_amd import autotune
    monkeypatch.setenv("LBM_SHAPE_CACHE", str(tmp_path / "shapes.json"))
    Tc, rl, rg = sat
    ws = [boiling(Tc, rl, rg, nx=128, ny=256, hot_width=8.0, gravity=1e-5, seed=3),
          evaporation(Tc, rl, rg, nx=192, ny=160, R=30.0),
          boiling(Tc, rl, rg, nx=256, ny=128, hot_width=8.0, gravity=2e-5, seed=4)]
    sol = [lbm.Solver(w.params).init(w.rho, w.ux, w.uy, w.T) for w in ws]
    b = lbm.Batch(sol)
    for i in range(3):
        b.set_budget(i, 50)
    b.step(20)
    b.sync()
    before = [s.save_state() for s in sol]
    res = autotune.tune_batch(b, steps=16, repeats=2)
    print("\n[case] autotune batch", res, flush=True)
    assert b.shape == res.shape and not res.cached
    assert [s.save_state() for s in sol] == before
    assert [b.remaining(i) for i in range(3)] == [30, 30, 30]
    b.step(30)
    assert b.sync() == [0, 0, 0]
    b.close()
    for w, s in zip(ws, sol):
        ref = lbm.Solver(w.params).init(w.rho, w.ux, w.uy, w.T)
        ref.step(50)
        assert s.save_state() == ref.save_state()
        ref.close()
        s.close()


def test_tile_orders_give_identical_bits(lbm, sat):
    """The order in which workgroups take the tiles (whole rows, strips of k tile columns, changed in
    mid-run, in a batch) does not change a bit: every node's arithmetic is the same."""
    Tc, rl, rg = sat
    w = boiling(Tc, rl, rg, nx=600, ny=260, hot_width=10.0, gravity=3e-5)  # 10 tile columns, ragged
    ref = None
    for shape in (6, 2):
        for order in (1, 2, 3, 8, 0):
            print(f"\n[case] tile order {order} shape {shape}", flush=True)
            s = lbm.Solver(w.params).init(w.rho, w.ux, w.uy, w.T).set_shape(shape).set_tile_order(order)
            assert s.tile_order == (10 if order == 1 else order if order else s.tile_order)
            s.step(37)
            s.set_tile_order(3 if order != 3 else 1)
            s.step(40)
            out = s.save_state()
            s.close()
            ref = ref or out
            assert out == ref, (shape, order)
    sols = [lbm.Solver(w.params).init(w.rho, w.ux, w.uy, w.T).set_tile_order(o) for o in (2, 1)]
    b = lbm.Batch(sols)
    for i in range(2):
        b.set_budget(i, 77)
    b.step(77)
    assert b.sync() == [0, 0]
    b.close()
    for s in sols:
        assert s.save_state() == ref
        s.close()
