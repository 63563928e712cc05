"""The allocation-free batch entry point (lbm_batch_create_noalloc, for callers that cannot allocate
device memory): called through the C ABI, its batch gives the same bits as a batch made by
lbm_batch_create over caller memory, on two calls in a row, the second with fewer and smaller
members; a second such batch on the device is refused while the first exists, and oversized
requests are refused."""
import ctypes

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


def _raw(s):
    f, g, h = s.state(absolute=False)
    return np.concatenate([f.ravel(), g.ravel(), h.ravel()])


def _run(lbm, ws, budgets, noalloc):
    sols = [lbm.Solver(w.params).init(w.rho, w.ux, w.uy, w.T) for w in ws]
    b = lbm.Batch(sols, noalloc=noalloc)
    assert (b.mem is None) == noalloc
    for i, n in enumerate(budgets):
        b.set_budget(i, n)
    b.step(70)
    b.step(max(budgets))
    st = b.sync()
    b.close()
    out = [(_raw(s), s.fields(), s.steps) for s in sols]
    for s in sols:
        s.close()
    return st, out


def _compare(lbm, ws, budgets):
    st_ref, ref = _run(lbm, ws, budgets, noalloc=False)
    st, got = _run(lbm, ws, budgets, noalloc=True)
    assert st == st_ref == [0] * len(ws)
    for (ra, fa, na), (rb, fb, nb), n in zip(got, ref, budgets):
        assert na == nb == n
        assert np.array_equal(ra, rb)
        for x, y in zip(fa, fb):
            assert np.array_equal(x, y)


def test_noalloc_batch_equals_caller_memory_batch(lbm):
    base = Params()
    Tc = lbm.critical_temperature(base)
    rl, rg, _ = lbm.coexistence(base, 0.86 * Tc)
    print("\n[case] noalloc batch: 3 members, then 2 smaller ones", flush=True)
    first = [boiling(Tc, rl, rg, nx=128, ny=96, gravity=3e-5, hot_width=8.0, seed=1),
             evaporation(Tc, rl, rg, nx=100, ny=70, R=15.0, superheat=1.15),
             droplet(Tc, rl, rg, nx=64, ny=64, R=16.0)]
    _compare(lbm, first, [150, 97, 64])
    second = [droplet(Tc, rl, rg, nx=48, ny=40, R=10.0),
              evaporation(Tc, rl, rg, nx=40, ny=36, R=8.0, superheat=1.2)]
    _compare(lbm, second, [41, 80])


def test_noalloc_batch_limits(lbm):
    from paper_2205_00686_amd import _native
    L = _native.lib()
    base = Params()
    Tc = lbm.critical_temperature(base)
    rl, rg, _ = lbm.coexistence(base, 0.86 * Tc)
    w = droplet(Tc, rl, rg, nx=32, ny=32, R=8.0)
    sols = [lbm.Solver(w.params).init(w.rho, w.ux, w.uy, w.T) for _ in range(2)]
    arr = (ctypes.c_void_p * 2)(*[s.handle.value for s in sols])
    stream = ctypes.c_void_p(sols[0].stream.cuda_stream)
    h1, h2 = ctypes.c_void_p(), ctypes.c_void_p()
    assert L.lbm_batch_create_noalloc(arr, 2, stream, ctypes.byref(h1)) == 0
    # one static batch per device at a time
    assert L.lbm_batch_create_noalloc(arr, 2, stream, ctypes.byref(h2)) == -5
    assert L.lbm_batch_destroy(h1) == 0
    assert L.lbm_batch_create_noalloc(arr, 2, stream, ctypes.byref(h2)) == 0
    assert L.lbm_batch_destroy(h2) == 0
    # sizes beyond the area, and empty batches, are refused without touching the device
    big = (ctypes.c_void_p * 257)(*([sols[0].handle.value] * 257))
    assert L.lbm_batch_create_noalloc(big, 257, stream, ctypes.byref(h2)) == -1
    assert L.lbm_batch_create_noalloc(arr, 0, stream, ctypes.byref(h2)) == -1
    for s in sols:
        s.close()
