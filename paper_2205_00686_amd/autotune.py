"""Autotuner of the step kernel's tile shape.

The library holds several workgroup shapes of the fused step (``shapes(precision)``).  Which one
is fastest depends on the grid.  A grid of few tiles is a single wave of workgroups, so the
latency of one workgroup sets the step time.  A large grid runs best with two workgroups resident
per compute unit, so that one workgroup's memory traffic overlaps the other's arithmetic.  The
tuner times every shape on the actual simulation (or batch) with HIP events on its stream.  It
then restores the exact state, keeps the fastest shape, and records the choice per (device,
precision, grid, boundary kind) in a JSON cache.  Every shape gives bit-identical results, so
tuning never changes an answer.

The cache file is ``$LBM_SHAPE_CACHE`` if set, else ``~/.cache/paper_2205_00686_amd/shapes.json``.
"""
from __future__ import annotations

import json
import os
import tempfile
import threading
from dataclasses import dataclass, field

from . import Batch, Solver, shape_fits, shapes

_lock = threading.Lock()


@dataclass
class TuneResult:
    shape: int                          # chosen shape index
    ms_per_step: dict = field(default_factory=dict)  # shape index -> measured ms per step
    key: str = ""
    cached: bool = False                # True: taken from the cache, nothing was timed

    def describe(self, precision) -> str:
        tx, ty, w, d = shapes(precision)[self.shape]
        return f"{tx}x{ty} tile, {w} wavefronts, {d} step(s) per launch"


def cache_path() -> str:
    return os.environ.get("LBM_SHAPE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache",
                                                               "paper_2205_00686_amd", "shapes.json")


def _load_cache(path):
    try:
        with open(path) as fh:
            data = json.load(fh)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def _store(path, key, value):
    with _lock:
        data = _load_cache(path)
        data[key] = value
        d = os.path.dirname(path) or "."
        os.makedirs(d, exist_ok=True)
        fd, tmp = tempfile.mkstemp(dir=d, prefix=".shapes.", suffix=".json")
        with os.fdopen(fd, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)


_build_id = None


def _library_id() -> str:
    """Digest of the built library: a rebuilt kernel invalidates earlier measurements."""
    global _build_id
    if _build_id is None:
        import hashlib
        from ._native import LIB_PATH
        with open(LIB_PATH, "rb") as fh:
            _build_id = hashlib.sha1(fh.read()).hexdigest()[:12]
    return _build_id


def _device_tag(device) -> str:
    import torch
    p = torch.cuda.get_device_properties(device)
    return f"{p.name}|{getattr(p, 'gcnArchName', '')}|cu{p.multi_processor_count}|lib{_library_id()}"


def solver_key(s: Solver) -> str:
    c = s.params
    return (f"{_device_tag(s.mem.device)}|p{s.precision}|q{s.q}|{s.nx}x{s.ny}|walls{int(c.y_walls)}"
            f"|box{int(c.thermal_box)}")


def batch_key(b: Batch) -> str:
    s0 = b.solvers[0]
    sizes = sorted(f"{s.nx}x{s.ny}w{int(s.params.y_walls)}b{int(s.params.thermal_box)}" for s in b.solvers)
    # grids of a batch enter through their multiset; a long list is summarised by a digest
    import hashlib
    digest = hashlib.sha1(",".join(sizes).encode()).hexdigest()[:16]
    return f"{_device_tag(s0.mem.device)}|p{s0.precision}|q{s0.q}|batch{len(sizes)}|{digest}"


def _time(step, stream, steps, repeats):
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = []
    for _ in range(repeats):
        e0.record(stream)
        step(steps)
        e1.record(stream)
        e1.synchronize()
        best.append(e0.elapsed_time(e1) / steps)
    best.sort()
    return best[len(best) // 2]


def _valid(entry, n):
    return isinstance(entry, dict) and isinstance(entry.get("shape"), int) and 0 <= entry["shape"] < n


def tune_solver(s: Solver, candidates=None, steps: int = 64, repeats: int = 3, use_cache: bool = True,
                force: bool = False) -> TuneResult:
    """Pick the fastest tile shape for Solver s and set it.  The simulation's state (populations,
    history, step count) is saved before timing and restored afterwards, bit for bit.  Shapes
    that do not fit the grid are not candidates."""
    n = len(shapes(s.precision))
    cands = list(range(n)) if candidates is None else [int(k) for k in candidates]
    cands = [k for k in cands if shape_fits(s.prm, k, s.precision)]
    key = solver_key(s)
    path = cache_path()
    if use_cache and not force:
        entry = _load_cache(path).get(key)
        if _valid(entry, n) and entry["shape"] in cands:
            s.set_shape(entry["shape"])
            return TuneResult(entry["shape"], {int(k): v for k, v in entry.get("ms_per_step", {}).items()}, key,
                              cached=True)
    snap = s.save_state()
    times = {}
    try:
        for k in cands:
            s.set_shape(k)
            s.step(steps)  # warm-up; builds this shape's graph
            times[k] = _time(s.step, s.stream, steps, repeats)
    finally:
        s.load_state(snap)
    best = min(times, key=times.get)
    s.set_shape(best)
    if use_cache:
        _store(path, key, {"shape": best, "ms_per_step": {str(k): v for k, v in times.items()}})
    return TuneResult(best, times, key)


def tune_batch(b: Batch, candidates=None, steps: int = 64, repeats: int = 3, use_cache: bool = True,
               force: bool = False) -> TuneResult:
    """Pick the fastest tile shape for the batched launches of b and set it.  Timing runs on
    clones of the members (same parameters, exact copies of their states), so neither the
    members nor the batch's budgets are touched; the clones need as much device memory again."""
    prec = b.solvers[0].precision
    n = len(shapes(prec))
    cands = list(range(n)) if candidates is None else [int(k) for k in candidates]
    cands = [k for k in cands if all(shape_fits(x.prm, k, prec) for x in b.solvers)]
    key = batch_key(b)
    path = cache_path()
    if use_cache and not force:
        entry = _load_cache(path).get(key)
        if _valid(entry, n) and entry["shape"] in cands:
            b.set_shape(entry["shape"])
            return TuneResult(entry["shape"], {int(k): v for k, v in entry.get("ms_per_step", {}).items()}, key,
                              cached=True)
    b.stream.synchronize()
    clones = []
    tb = None
    try:
        for s in b.solvers:
            c = Solver(s.prm, precision=s.precision, device=s.mem.device, stream=b.stream)
            c.load_state(s.save_state())
            clones.append(c)
        tb = Batch(clones, stream=b.stream)
        times = {}
        budget = steps * (repeats + 1)
        for k in cands:
            tb.set_shape(k)
            for i in range(len(clones)):
                tb.set_budget(i, budget)
            tb.step(steps)
            times[k] = _time(tb.step, b.stream, steps, repeats)
            tb.sync()
    finally:
        if tb is not None:
            tb.close()
        for c in clones:
            c.close()
    best = min(times, key=times.get)
    b.set_shape(best)
    if use_cache:
        _store(path, key, {"shape": best, "ms_per_step": {str(k): v for k, v in times.items()}})
    return TuneResult(best, times, key)
