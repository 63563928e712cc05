"""Admission order of the continuous-batching server (host logic, no GPU): which queued request is
admitted next under the arrival and shortest-work policies."""
import concurrent.futures as cf
from collections import deque
from types import SimpleNamespace

import pytest

from paper_2205_00686_amd import serve


def _queue(specs):
    """specs: (rid, t_arrive, steps, nodes or None while its fields are being prepared)."""
    queued, prep = deque(), {}
    for rid, t, steps, nodes in specs:
        r = serve.Request(rid=rid, arrival=t, steps=steps, make=None)
        r.t_arrive = t
        fut = cf.Future()
        if nodes is not None:
            fut.set_result(SimpleNamespace(nodes=nodes))
        queued.append(r)
        prep[rid] = fut
    return queued, prep


def test_arrival_order_waits_for_the_head():
    s = serve.Server(hbm_budget=1, policy="arrival")
    q, prep = _queue([(0, 0.0, 100, None), (1, 0.1, 10, 50)])
    assert s._next(q, prep, 1.0) is None
    q, prep = _queue([(0, 0.0, 100, 4000), (1, 0.1, 10, 50)])
    assert s._next(q, prep, 1.0).rid == 0


def test_shortest_work_first_among_ready_requests():
    s = serve.Server(hbm_budget=1, policy="shortest", max_wait=5.0)
    q, prep = _queue([(0, 0.0, 1000, 4000), (1, 0.1, 100, 4000), (2, 0.2, 50, None), (3, 0.3, 100, 5000)])
    assert s._next(q, prep, 1.0).rid == 1  # 4e5 node updates; request 2 is not ready yet
    prep[2].set_result(SimpleNamespace(nodes=100))
    assert s._next(q, prep, 1.0).rid == 2
    # the oldest request has waited max_wait: it goes first whatever its size
    assert s._next(q, prep, 5.0).rid == 0
    q, prep = _queue([(0, 0.0, 1000, None), (1, 0.1, 10, 10)])
    assert s._next(q, prep, 6.0) is None  # ... and is waited for while its fields are prepared


def test_unknown_policy_is_rejected():
    with pytest.raises(ValueError):
        serve.Server(hbm_budget=1, policy="random")
