"""Host-side scheduling of the continuous-batching server, with stand-in solvers (no GPU):
admission in arrival order within the slot and HBM-budget limits, each request advanced exactly its
own step count, oversize and failing requests isolated, latency measured from arrival."""
import types

import pytest

from paper_2205_00686_amd import serve


class FakeSolver:
    live_bytes = 0
    peak_bytes = 0
    live = 0
    peak_live = 0

    def __init__(self, params, precision=None, stream=None):
        self.params = params
        self.steps = 0
        if params.get("bad"):
            raise RuntimeError("rejected by lbm_init")

    def init(self, rho, ux, uy, T):
        cls = type(self)
        cls.live_bytes += self.params["fp"]
        cls.live += 1
        cls.peak_bytes = max(cls.peak_bytes, cls.live_bytes)
        cls.peak_live = max(cls.peak_live, cls.live)
        return self

    def fields(self):
        return (self.steps,)

    def close(self):
        cls = type(self)
        cls.live_bytes -= self.params["fp"]
        cls.live -= 1
        self.closed = True


class FakeBatch:
    launches = []

    def __init__(self, solvers, stream=None):
        self.solvers = list(solvers)
        self.budget = [0] * len(self.solvers)

    def set_budget(self, i, n):
        self.budget[i] = n

    def step(self, k):
        type(self).launches.append(len(self.solvers))
        for s, b in zip(self.solvers, self.budget):
            s.steps += min(b, k)
            if s.params.get("nan_after") is not None and s.steps >= s.params["nan_after"]:
                s.failed = True

    def sync(self):
        return [-4 if getattr(s, "failed", False) else 0 for s in self.solvers]

    def close(self):
        # the server releases a batch before any of its members
        assert not any(getattr(s, "closed", False) for s in self.solvers)


@pytest.fixture
def fake(monkeypatch):
    FakeSolver.live_bytes = FakeSolver.peak_bytes = FakeSolver.live = FakeSolver.peak_live = 0
    FakeBatch.launches = []
    monkeypatch.setattr(serve, "Solver", FakeSolver)
    monkeypatch.setattr(serve, "Batch", FakeBatch)
    monkeypatch.setattr(serve, "footprint_bytes", lambda p, prec: p["fp"])
    monkeypatch.setattr(serve, "_new_stream", lambda: None)
    import torch
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)
    return serve


def _req(rid, steps, fp, arrival=0.0, **extra):
    w = types.SimpleNamespace(params=dict(fp=fp, **extra), rho=None, ux=None, uy=None, T=None, nodes=fp)
    return serve.Request(rid=rid, arrival=arrival, steps=steps, make=lambda: w)


def test_every_request_gets_its_steps_within_limits(fake):
    reqs = [_req(i, steps=100 + 37 * i, fp=10 + (i % 3) * 5) for i in range(12)]
    done, summary = fake.Server(hbm_budget=40, max_slots=3, chunk=64).run(reqs, realtime=False)
    assert summary["completed"] == 12 and summary["failed"] == 0
    for r in done:
        assert r.result == (r.steps,)
        assert r.latency >= 0.0 and r.t_admit <= r.t_done
    assert FakeSolver.peak_bytes <= 40
    assert FakeSolver.peak_live <= 3
    assert FakeSolver.live == 0
    # continuous batching: several requests shared launches
    assert max(FakeBatch.launches) > 1
    assert summary["node_updates"] == sum(r.nodes * r.steps for r in done)


def test_batch_released_before_members_when_all_finish_together(fake):
    # two rounds in which every running request finishes in the same chunk
    reqs = [_req(i, steps=64, fp=10) for i in range(2)] + [_req(2 + i, steps=128, fp=10, arrival=0.0) for i in range(2)]
    done, summary = fake.Server(hbm_budget=20, max_slots=2, chunk=64).run(reqs, realtime=False)
    assert summary["completed"] == 4 and FakeSolver.live == 0


def test_admission_is_in_arrival_order(fake):
    reqs = [_req(i, steps=64, fp=10) for i in range(6)]
    done, _ = fake.Server(hbm_budget=20, max_slots=8, chunk=64).run(reqs, realtime=False)
    admits = [r.t_admit for r in sorted(done, key=lambda r: r.rid)]
    assert admits == sorted(admits)


def test_oversize_and_failing_requests_are_isolated(fake):
    reqs = [_req(0, 200, 10), _req(1, 200, 1000), _req(2, 300, 10, bad=True), _req(3, 500, 10, nan_after=130),
            _req(4, 250, 10)]
    done, summary = fake.Server(hbm_budget=50, max_slots=4, chunk=64).run(reqs, realtime=False)
    by = {r.rid: r for r in done}
    assert by[1].error == "footprint exceeds the HBM budget"
    assert "rejected" in by[2].error
    assert by[3].error == "numerical failure" and by[3].result is None
    for i in (0, 4):
        assert by[i].error is None and by[i].result == (by[i].steps,)
    assert summary["completed"] == 2 and summary["failed"] == 3
    assert FakeSolver.live == 0


def test_oversize_request_does_not_block_the_queue(fake):
    # request 1 can never fit; it is rejected when it reaches the head of the queue, while request 0
    # runs, so request 2 is admitted next to request 0 instead of waiting for the server to drain
    reqs = [_req(0, 640, 30), _req(1, 64, 1000), _req(2, 64, 10)]
    done, summary = fake.Server(hbm_budget=50, max_slots=4, chunk=64).run(reqs, realtime=False)
    by = {r.rid: r for r in done}
    assert by[1].error == "footprint exceeds the HBM budget"
    assert by[1].t_done <= by[0].t_done
    assert by[2].t_admit <= by[0].t_done and by[2].t_done <= by[0].t_done
    assert summary["completed"] == 2 and summary["failed"] == 1


@pytest.mark.parametrize("policy", ["arrival", "shortest"])
def test_request_whose_fields_cannot_be_built_fails_alone(fake, policy):
    def broken():
        raise ValueError("no such workload")
    reqs = [_req(0, 128, 10), serve.Request(rid=1, arrival=0.0, steps=64, make=broken), _req(2, 64, 10)]
    done, summary = fake.Server(hbm_budget=50, max_slots=4, chunk=64, policy=policy).run(reqs, realtime=False)
    by = {r.rid: r for r in done}
    assert "no such workload" in by[1].error
    assert by[0].result == (128,) and by[2].result == (64,)
    assert summary["completed"] == 2 and summary["failed"] == 1


def test_fifo_isolates_a_request_whose_fields_cannot_be_built(fake, monkeypatch):
    class Plain(FakeSolver):
        def step(self, n):
            self.steps += n

    def broken():
        raise ValueError("no such workload")
    monkeypatch.setattr(serve, "Solver", Plain)
    reqs = [_req(0, 50, 10), serve.Request(rid=1, arrival=0.0, steps=64, make=broken), _req(2, 70, 10)]
    done, summary = fake.fifo(reqs, realtime=False)
    by = {r.rid: r for r in done}
    assert "no such workload" in by[1].error
    assert by[0].result == (50,) and by[2].result == (70,)
    assert summary["completed"] == 2 and summary["failed"] == 1


def test_fifo_baseline_runs_one_at_a_time(fake, monkeypatch):
    class Plain(FakeSolver):
        def step(self, n):
            self.steps += n

    monkeypatch.setattr(serve, "Solver", Plain)
    reqs = [_req(i, steps=50 * (i + 1), fp=10) for i in range(4)]
    done, summary = fake.fifo(reqs, realtime=False)
    assert summary["completed"] == 4
    assert all(r.result == (r.steps,) for r in done)
    assert Plain.peak_live == 1
    assert all(r.latency >= 0.0 for r in done)
