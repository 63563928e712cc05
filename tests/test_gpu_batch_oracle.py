"""Batched and served runs against the FP64 oracle (not only against the same GPU kernel run alone):
every member of a batch of uneven grids, parameters and step budgets, in FP32 and FP64, and every
request of a continuous-batching mix, compared element by element with its own oracle run.

Bounds: FP64 members agree to rounding (rho <= 1e-11, T and u <= 1e-13, as the single-run FP64
parity); FP32 members stay within the single-run FP32 bounds (after up to 300 steps rho within
2e-4 rho_l, T within 2e-6 relative, u within 1e-5), which follow from the FP32 unit roundoff
accumulated over the collisions.

Also: a saved state is rejected by a context of another precision, grid or thermal lattice, and a
truncated buffer is rejected (2-D and 3-D)."""
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


def _sat(orc):
    base = Params()
    Tc = orc.Tc(base)
    rl, rg, _ = orc.maxwell(base, 0.86 * Tc)
    return Tc, rl, rg


def _errors(got, exp):
    return {n: float(np.abs(g - e).max()) for n, g, e in zip(("rho", "ux", "uy", "T"), got, exp)}


def _oracle_fields(orc, w, steps):
    o = orc.Oracle(w.params).init(w.rho, w.ux, w.uy, w.T)
    o.step(steps)
    return o.fields()


def _assert_fp32(err, exp):
    Tmax = float(np.abs(exp[3]).max())
    assert err["rho"] <= 2e-4 * 6.5 and err["T"] <= 2e-6 * Tmax and max(err["ux"], err["uy"]) <= 1e-5, err


def _assert_fp64(err):
    assert err["rho"] <= 1e-11 and err["T"] <= 1e-13 and max(err["ux"], err["uy"]) <= 1e-13, err


def _batch_run(lbm, ws, budgets, precision, pre=None):
    sols = [lbm.Solver(w.params, precision=precision).init(w.rho, w.ux, w.uy, w.T) for w in ws]
    pre = pre or [0] * len(ws)
    for s, n in zip(sols, pre):  # some members take plain steps first: the batch continues them
        if n:
            s.step(n)
    b = lbm.Batch(sols)
    for i, n in enumerate(budgets):
        b.set_budget(i, n - pre[i])
    b.step(70)
    b.step(max(budgets))
    assert b.sync() == [0] * len(ws)
    b.close()
    for s, n in zip(sols, budgets):
        assert s.steps == n
    return sols


def test_batch_members_match_oracle_fp32(lbm, orc):
    Tc, rl, rg = _sat(orc)
    ws = [boiling(Tc, rl, rg, nx=128, ny=96, gravity=3e-5, dT_rel=0.25, hot_width=8.0, seed=1),
          evaporation(Tc, rl, rg, nx=100, ny=70, R=15.0, superheat=1.15),
          droplet(Tc, rl, rg, nx=64, ny=64, R=16.0),
          boiling(Tc, rl, rg, nx=70, ny=130, gravity=1e-5, dT_rel=0.1, hot_width=5.0, seed=2)]
    budgets = [150, 97, 64, 200]
    print("\n[case] FP32 batch of 4 uneven members vs oracle", flush=True)
    sols = _batch_run(lbm, ws, budgets, lbm.LBM_FP32, pre=[0, 0, 0, 10])
    for i, (s, w, n) in enumerate(zip(sols, ws, budgets)):
        exp = _oracle_fields(orc, w, n)
        err = _errors(s.fields(), exp)
        print(f"   member {i} {w.params.nx}x{w.params.ny} {n} steps: " +
              " ".join(f"{k}={v:.2e}" for k, v in err.items()), flush=True)
        _assert_fp32(err, exp)
        s.close()


def test_batch_fp64_uneven_members_match_oracle(lbm, orc):
    """FP64 batch of uneven grids, boundary kinds (periodic, Dirichlet box, walls with gravity and
    a hot spot, open top) and budgets (odd and even, one below a graph's worth of steps)."""
    Tc, rl, rg = _sat(orc)
    ws = [boiling(Tc, rl, rg, nx=96, ny=72, gravity=5e-5, dT_rel=0.2, hot_width=6.0, seed=3),
          evaporation(Tc, rl, rg, nx=70, ny=90, R=14.0, superheat=1.2, hot_vapour=True),
          droplet(Tc, rl, rg, nx=65, ny=33, R=9.0),
          heated_droplet(Tc, rl, rg, nx=80, ny=40, R=12.0, T_h_rel=0.95, gy=-5e-5)]
    budgets = [131, 80, 41, 150]
    print("\n[case] FP64 batch of 4 uneven members vs oracle", flush=True)
    sols = _batch_run(lbm, ws, budgets, lbm.LBM_FP64, pre=[0, 3, 0, 0])
    for i, (s, w, n) in enumerate(zip(sols, ws, budgets)):
        exp = _oracle_fields(orc, w, n)
        err = _errors(s.fields(), exp)
        print(f"   member {i} {w.params.nx}x{w.params.ny} {n} steps: " +
              " ".join(f"{k}={v:.2e}" for k, v in err.items()), flush=True)
        _assert_fp64(err)
        s.close()


def test_served_results_match_oracle(lbm, orc):
    """Requests arriving while others run (admission limited to three at a time by the HBM budget):
    each served result against its own oracle run."""
    from paper_2205_00686_amd import serve
    Tc, rl, rg = _sat(orc)
    mix = [
        (0.00, 300, lambda: droplet(Tc, rl, rg, nx=96, ny=80, R=20.0)),
        (0.00, 130, lambda: evaporation(Tc, rl, rg, nx=128, ny=100, R=16.0, superheat=1.2)),
        (0.01, 257, lambda: boiling(Tc, rl, rg, nx=130, ny=140, hot_width=8.0, seed=4)),
        (0.02, 64, lambda: droplet(Tc, rl, rg, nx=70, ny=70, R=12.0)),
        (0.02, 190, lambda: boiling(Tc, rl, rg, nx=64, ny=200, gravity=4e-5, hot_width=6.0, seed=5)),
        (0.03, 75, lambda: heated_droplet(Tc, rl, rg, nx=90, ny=50, R=14.0, T_h_rel=0.95)),
    ]
    fp = max(lbm.footprint_bytes(make().params) for _, _, make in mix)
    server = serve.Server(hbm_budget=3 * fp, max_slots=3, chunk=64)
    reqs = [serve.Request(rid=i, arrival=a, steps=n, make=m) for i, (a, n, m) in enumerate(mix)]
    done, summary = server.run(reqs, realtime=False)
    print("\n[case] served mix vs oracle:", summary, flush=True)
    assert summary["completed"] == len(mix)
    for r in done:
        _, steps, make = mix[r.rid]
        exp = _oracle_fields(orc, make(), steps)
        err = _errors(r.result, exp)
        print(f"   request {r.rid} ({steps} steps): " + " ".join(f"{k}={v:.2e}" for k, v in err.items()), flush=True)
        _assert_fp32(err, exp)


def test_saved_state_of_another_context_is_rejected(lbm, orc):
    Tc, rl, rg = _sat(orc)
    w = droplet(Tc, rl, rg, nx=40, ny=32, R=8.0)
    a = lbm.Solver(w.params, precision=lbm.LBM_FP64).init(w.rho, w.ux, w.uy, w.T)
    a.step(5)
    blob64 = a.save_state()
    b = lbm.Solver(w.params, precision=lbm.LBM_FP32).init(w.rho, w.ux, w.uy, w.T)
    blob32 = b.save_state()
    for bad in (blob64, blob32[:-8], blob32 + b"\0" * 8):
        with pytest.raises(lbm.LbmError) as e:
            b.load_state(bad)
        assert e.value.status == -1
    # same byte count, another grid: 40x32 FP32 vs 32x40 FP32
    w2 = droplet(Tc, rl, rg, nx=32, ny=40, R=8.0)
    c = lbm.Solver(w2.params).init(w2.rho, w2.ux, w2.uy, w2.T)
    assert c.state_bytes() == b.state_bytes()
    with pytest.raises(lbm.LbmError) as e:
        c.load_state(blob32)
    assert e.value.status == -1
    # the D2Q9 thermal lattice: another layout
    w9 = droplet(Tc, rl, rg, nx=40, ny=32, R=8.0, thermal_q=9)
    d = lbm.Solver(w9.params).init(w9.rho, w9.ux, w9.uy, w9.T)
    with pytest.raises(lbm.LbmError):
        d.load_state(blob32)
    # a good one still loads and resumes
    b.load_state(blob32)
    assert b.steps == 0
    # 3-D
    from paper_2205_00686_amd import three_d
    from workloads import droplet3d
    w3 = droplet3d(Tc, rl, rg, n=16, R=5.0)
    s3 = three_d.Solver3D(w3.params).init(w3.rho, w3.ux, w3.uy, w3.uz, w3.T)
    blob3 = s3.save_state()
    t3 = three_d.Solver3D(w3.params, precision=lbm.LBM_FP64).init(w3.rho, w3.ux, w3.uy, w3.uz, w3.T)
    for bad in (blob3, blob3[:-4]):
        with pytest.raises(Exception):
            t3.load_state(bad)
    s3.load_state(blob3)
