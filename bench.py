"""Benchmark of the fused thermal LBM step on one MI355X.

Headline workload: the nucleate-boiling pool of the paper's Section 4.3 set-up at 1024 x 2048, FP32
populations: walls at the bottom (contact angle 75, Gaussian hot spot of width 32 and 0.2 Tc) and
top (90), gravity 2e-5, saturated liquid at 0.86 Tc with 1e-3 density noise (seed 1).  The pool is
filled to the head limit of the closed box: at the stated fill 0.5 the vapour column above it is
compressed past its spinodal within about 1500 steps.  One benchmark step is one time step of the
whole coupled D2Q9 + D2Q5 update over the grid (fused kernels, one or two steps per launch as the
autotuned tile shape has it).

Prints one JSON line: MLUPS of exactly K steps in one call, the roofline of the step kernel
(algorithmic 128 bytes per node update in FP32 over the kernel's average launch duration from HIP
events on the library's stream), the batched gravity sweep against plain launches, a served request
stream against FIFO service (p50/p99 latency), and the FP64 CPU oracle timed on a bounded sample of
the same workload.

  python bench.py [--gpus 1] [--steps 2000] [--warmup 100] [--no-cpu-baseline] [--no-batched] [--no-served]
  python bench.py --workload evaporation --nx 512 --ny 512       the droplet-evaporation workload instead
  python bench.py --mode batch [--instances 64 --steps 10000]    batched gravity sweep vs plain
  python bench.py --mode serve [--requests 256 --rate 20]        continuous batching vs FIFO
  python bench.py --mode fritz [--gravities 1e-5,...,6e-5]       bubble departure diameter vs gravity
  python bench.py --mode lattice                                 thermal lattice: D2Q5 MRT / BGK vs D2Q9
  python bench.py --mode heated                                  droplet evaporation on a heated surface
  python bench.py --mode 3d                                      three-dimensional extension (D3Q19 + D3Q7)
  python bench.py --mode ceiling                                 HBM copy ceiling (hand-written copy kernel)
  python bench.py --mode cpu-baseline                            the FP64 oracle timed on the parity configurations
  python bench.py --mode readout                                 cost of the readouts (vapour rows and components, fields)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS (D2Q9+D2Q5 node updates/s) & % HBM roofline; batched vs plain; p50/p99"
HBM_PEAK_GBS = 8000.0
BYTES_PER_LU = {"f32": 128, "f64": 256}  # f 9+9, g 5+5, history 2+2 values per node update
# Measured HBM bytes per launch of the fused 3-D kernel (FETCH_SIZE x 2 + WRITE_SIZE, calibrated on a
# plain copy): (edge, path, z_chunk) -> bytes, for the kernel as profiled
TRAFFIC3D = {(256, 0, 0): {"bytes": 3976907571, "kernel_sha": "dd5e74b3f1075cb1"}}
KERNEL3D_SOURCES = ("lbm3d.hip", "lbm_device.hpp")
# HBM bytes per launch of the step kernel from rocprofv3 FETCH_SIZE / WRITE_SIZE passes, scaled by the
# same counters read for a plain copy of known size (profiles/): (workload, nx, ny, shape, dtype) ->
# bytes and the digest of the kernel sources profiled (reported only while the sources match)
TRAFFIC = {("boiling", 1024, 2048, 2, "f32"): {"bytes": 272334848, "kernel_sha": "d5db904e983c3fd3"},
           ("evaporation", 4096, 4096, 6, "f32"): {"bytes": 2301070336, "kernel_sha": "d5db904e983c3fd3"},
           ("evaporation", 4096, 4096, 2, "f32"): {"bytes": 2325466624, "kernel_sha": "d5db904e983c3fd3"}}


def build_workload(nx=512, ny=512, steps=20000, kind="evaporation"):
    """evaporation: the benchmark workload.  boiling: the nucleate-boiling pool (walls, hot spot of
    width 32 and dT 0.2 Tc, g = 2e-5, noise from seed 1); its pool is filled to the head limit of
    the closed box (workloads.head_limited_fill) so that it stays stable over a long timed run."""
    import paper_2205_00686_amd as lbm
    from workloads import Params, boiling, evaporation, head_limited_fill

    base = Params()
    Tc = lbm.critical_temperature(base)
    rl, rg, ps = lbm.coexistence(base, 0.86 * Tc)
    if kind == "boiling":
        return boiling(Tc, rl, rg, nx=nx, ny=ny, gravity=2e-5, seed=1, steps=steps,
                       fill=head_limited_fill(rl, rg, ps, 2e-5, ny))
    return evaporation(Tc, rl, rg, nx=nx, ny=ny, R=64.0 * nx / 512, superheat=1.10, steps=steps)


def _host_cpu() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, steps):
    """The FP64 oracle on the same workload for a bounded number of steps, on all host cores
    (OpenMP), then on one core for a sixteenth of the steps."""
    import oracle

    oracle.build(force=False)
    o = oracle.Oracle(w.params).init(w.rho, w.ux, w.uy, w.T)
    o.step(2)  # warm caches
    cores = oracle.num_threads()
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    steps1 = max(1, steps // 16)
    oracle.set_threads(1)
    try:
        t1 = time.perf_counter()
        o.step(steps1)
        dt1 = time.perf_counter() - t1
    finally:
        oracle.set_threads(cores)
    return {"value": w.nodes * steps / dt / 1e6, "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": f"{w.params.nx}x{w.params.ny} {w.name}, FP64, {steps} steps after 2 warm-up steps "
                      f"({dt:.1f} s)",
            "single_core": {"value": w.nodes * steps1 / dt1 / 1e6, "steps": steps1, "seconds": round(dt1, 2)},
            "host": {"cpu": _host_cpu(), "logical_cpus": os.cpu_count()}}


def run_cpu_baseline_mode(args):
    """The FP64 oracle timed on the configurations of the parity tests, as a CPU reference: the
    static droplet (64 x 64, 2000 steps) and the evaporation box (512 x 512, 20 000 steps) in full,
    the boiling pool (1024 x 2048) over its first 2000 steps with the time for 50 000 steps
    extrapolated; each on all host cores (OpenMP) and, for a stated sample, on one core."""
    import oracle
    import paper_2205_00686_amd as lbm
    from workloads import Params, droplet

    oracle.build(force=False)
    base = Params()
    Tc = lbm.critical_temperature(base)
    rl, rg, _ = lbm.coexistence(base, 0.86 * Tc)
    full = args.cpu_scale
    cases = [
        ("static droplet 64x64, FP64", droplet(Tc, rl, rg, nx=64, ny=64, R=16.0), int(2000 * full), 2000,
         int(2000 * full)),
        ("evaporation 512x512, FP64", build_workload(512, 512, 20000, "evaporation"), int(20000 * full), 20000,
         max(1, int(200 * full))),
        ("boiling 1024x2048 (head-limited fill), FP64", build_workload(1024, 2048, 50000, "boiling"),
         max(2, int(2000 * full)), 50000, max(1, int(20 * full))),
    ]
    cores = oracle.num_threads()
    runs = []
    gpu = _gpu_available()
    for name, w, steps, horizon, steps1 in cases:
        o = oracle.Oracle(w.params).init(w.rho, w.ux, w.uy, w.T)
        t0 = time.perf_counter()
        o.step(steps)
        dt = time.perf_counter() - t0
        oracle.set_threads(1)
        try:
            o1 = oracle.Oracle(w.params).init(w.rho, w.ux, w.uy, w.T)
            t1 = time.perf_counter()
            o1.step(steps1)
            dt1 = time.perf_counter() - t1
        finally:
            oracle.set_threads(cores)
        run = {"config": name, "nodes": w.nodes, "steps": steps, "seconds": round(dt, 2),
               "mlups": round(w.nodes * steps / dt / 1e6, 2), "horizon_steps": horizon,
               "horizon_seconds": round(dt * horizon / steps, 1) if steps else None,
               "horizon_measured": steps == horizon,
               "single_core": {"steps": steps1, "seconds": round(dt1, 2),
                               "mlups": round(w.nodes * steps1 / dt1 / 1e6, 2)}}
        if gpu:  # the same steps on the GPU, the library's default tile shape; FP64 only for the droplet
            prec = lbm.LBM_FP64 if "droplet" in name else lbm.LBM_FP32
            sg = lbm.Solver(w.params, precision=prec).init(w.rho, w.ux, w.uy, w.T)
            sg.step(min(steps, 64))
            ms = _timed_steps(sg, steps)
            sg.sync()
            sg.close()
            run["gpu"] = {"precision": "fp64" if prec == lbm.LBM_FP64 else "fp32", "steps": steps,
                          "seconds": round(ms / 1e3, 4), "us_per_step": round(ms * 1e3 / steps, 2),
                          "horizon_seconds": round(ms / 1e3 * horizon / steps, 3)}
        runs.append(run)
        print(f"[bench] {json.dumps(run)}", file=sys.stderr, flush=True)
    print(json.dumps({"metric": "FP64 oracle MLUPS on the host (CPU reference)", "unit": "MLUPS", "kind": "oracle",
                      "cores": cores, "host": {"cpu": _host_cpu(), "logical_cpus": os.cpu_count()},
                      "runs": runs}))


def _gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except ImportError:
        return False


def run_readout_mode(args):
    """Cost of the readouts of a running simulation, on the boiling pool (1024 x 2048, FP32) after
    args.steps steps: the per-row vapour counts of the departure trigger, the vapour components of
    the band below the pool surface and of the whole grid (the vapour above the pool is one component
    of about a million nodes), all fields to the host, and the FP64 diagnostics.  Each call is timed
    on the host around the synchronising call (median of 5 after one untimed call)."""
    import paper_2205_00686_amd as lbm
    from workloads import Params

    base = Params()
    Tc = lbm.critical_temperature(base)
    rl, rg, _ = lbm.coexistence(base, 0.86 * Tc)
    w = build_workload(args.nx, args.ny, args.steps, "boiling")
    s = lbm.Solver(w.params).init(w.rho, w.ux, w.uy, w.T)
    s.step(args.steps)
    s.sync()
    mid = 0.5 * (rl + rg)
    y_surface = int(min(w.meta["fill"], 1.0) * args.ny) - 12
    calls = {
        "vapour_rows (all rows, all columns)": lambda: s.vapour_rows(mid, 0, args.nx),
        f"vapour_components rows 0..{y_surface}": lambda: s.vapour_components(mid, 0, y_surface + 1),
        f"vapour_components rows 0..{args.ny}": lambda: s.vapour_components(mid, 0, args.ny),
        "read_fields (4 FP64 fields to the host)": lambda: s.fields(),
        "diagnostics (FP64 mass and energy)": lambda: s.diagnostics(),
    }
    out = {}
    for name, fn in calls.items():
        res = fn()
        ts = []
        for _ in range(5):
            t0 = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t0)
        out[name] = {"ms": round(sorted(ts)[2] * 1e3, 3)}
        if name.startswith("vapour_components"):
            out[name]["components"] = len(res)
            out[name]["largest_area"] = max((c["area"] for c in res), default=0)
        print(f"[bench] {name}: {json.dumps(out[name])}", file=sys.stderr, flush=True)
    s.close()
    print(json.dumps({"metric": "readout cost (ms per call)", "mode": "readouts",
                      "config": {"workload": f"boiling pool {args.nx}x{args.ny}, FP32, after {args.steps} steps"},
                      "calls": out}))


def shape_text(lbm, precision, k):
    tx, ty, w, d = lbm.shapes(precision)[k]
    return f"{tx}x{ty} tile, {w} wavefronts, {d} step{'s' if d > 1 else ''} per launch (shape {k})"


def choose_shape(s, shape):
    """Tile shape of a solver: 'auto' times every shape (autotune), an integer fixes one.
    Returns the measured ms per step per shape ({} when fixed)."""
    from paper_2205_00686_amd import autotune

    if shape == "auto":
        r = autotune.tune_solver(s, use_cache=False)
        return {str(k): round(v, 6) for k, v in sorted(r.ms_per_step.items())}
    s.set_shape(int(shape))
    return {}


def sweep_workloads(n, steps, lbm):
    """The batched gravity sweep: boiling instances on grids of three sizes, gravity log-uniform in
    [5e-6, 5e-5], hot-spot dT uniform in [0.1, 0.3] Tc (workloads.gravity_sweep, seed 2).  The pool
    is half full unless the vapour head of that pool would exceed p_sat / 2; then it is filled
    further (workloads.head_limited_fill), which keeps every instance inside the model's stable
    range for the whole run."""
    from workloads import Params, boiling, gravity_sweep, head_limited_fill

    base = Params()
    Tc = lbm.critical_temperature(base)
    rl, rg, ps = lbm.coexistence(base, 0.86 * Tc)
    out = []
    for spec in gravity_sweep(n=n, steps=steps):
        fill = head_limited_fill(rl, rg, ps, spec["gravity"], spec["ny"])
        out.append(boiling(Tc, rl, rg, nx=spec["nx"], ny=spec["ny"], gravity=spec["gravity"],
                           dT_rel=spec["dT_rel"], seed=spec["seed"], steps=steps, fill=fill))
    return out


def run_batch_mode(args):
    """Batched (one launch per step over all instances, graph-replayed) against sequential plain runs."""
    import torch

    import paper_2205_00686_amd as lbm

    ws = sweep_workloads(args.instances, args.steps, lbm)
    nodes = sum(w.nodes for w in ws)
    print(f"[bench] batch of {len(ws)} boiling instances, {nodes} nodes, {args.steps} steps", file=sys.stderr,
          flush=True)
    from paper_2205_00686_amd import autotune

    # plain: one simulation after the other, each with the tile shape tuned for its grid
    solvers = [lbm.Solver(w.params).init(w.rho, w.ux, w.uy, w.T) for w in ws]
    stream = solvers[0].stream
    for s in solvers:
        s.step(args.warmup)
    plain_shapes = {}
    for s in solvers:
        r = autotune.tune_solver(s)
        plain_shapes[f"{s.nx}x{s.ny}"] = shape_text(lbm, lbm.LBM_FP32, r.shape)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for s in solvers:
        s.step(args.steps)
    e1.record(stream)
    e1.synchronize()
    for s in solvers:
        s.sync()
    plain_ms = e0.elapsed_time(e1)
    plain_state = [s.save_state() for s in solvers[:4]]
    for s in solvers:
        s.close()
    # batched
    solvers = [lbm.Solver(w.params).init(w.rho, w.ux, w.uy, w.T) for w in ws]
    b = lbm.Batch(solvers)
    for i in range(len(solvers)):
        b.set_budget(i, args.warmup)
    b.step(args.warmup)
    b.sync()
    bt = autotune.tune_batch(b, use_cache=False)
    print(f"[bench] batch tile shape {b.shape}: {bt.ms_per_step}", file=sys.stderr, flush=True)
    for i in range(len(solvers)):
        b.set_budget(i, args.steps)
    torch.cuda.synchronize()
    e0.record(stream)
    b.step(args.steps)
    e1.record(stream)
    e1.synchronize()
    st = b.sync()
    batch_ms = e0.elapsed_time(e1)
    same = all(s.save_state() == p for s, p in zip(solvers[:4], plain_state))
    lu = nodes * args.steps
    out = {"metric": METRIC, "mode": "batched vs plain", "unit": "MLUPS", "n_gpus": 1, "dtype": "f32",
           "config": {"workload": f"gravity sweep: {len(ws)} boiling instances on 256x512/384x768/512x1024 grids, "
                                  f"g log-uniform [5e-6, 5e-5], dT uniform [0.1, 0.3] Tc, pool fill 0.5 or head-limited",
                      "instances": len(ws), "nodes": nodes, "steps": args.steps, "warmup": args.warmup,
                      "batch_tile_shape": shape_text(lbm, lbm.LBM_FP32, b.shape),
                      "plain_tile_shapes": plain_shapes},
           "batched_mlups": round(lu / (batch_ms * 1e-3) / 1e6, 1),
           "plain_sequential_mlups": round(lu / (plain_ms * 1e-3) / 1e6, 1),
           "speedup": round(plain_ms / batch_ms, 3),
           "batched_roofline_frac": round(lu * 128 / (batch_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "batched_equals_plain_bitwise_first4": same, "failed_instances": sum(1 for x in st if x != 0)}
    print(json.dumps(out), flush=True)


def run_serve_mode(args):
    """Continuous batching of a Poisson request stream against one-at-a-time FIFO service."""
    import paper_2205_00686_amd as lbm
    from paper_2205_00686_amd import serve
    from workloads import Params, boiling, droplet, evaporation, head_limited_fill, request_stream

    base = Params()
    Tc = lbm.critical_temperature(base)
    rl, rg, ps = lbm.coexistence(base, 0.86 * Tc)

    def make(spec):
        nx, ny, seed = spec["nx"], spec["ny"], spec["seed"]
        if spec["kind"] == "droplet":
            return lambda: droplet(Tc, rl, rg, nx=nx, ny=ny, R=min(nx, ny) / 4.0)
        if spec["kind"] == "evaporation":
            return lambda: evaporation(Tc, rl, rg, nx=nx, ny=ny, R=min(nx, ny) / 8.0)
        fill = head_limited_fill(rl, rg, ps, 2e-5, ny)
        return lambda: boiling(Tc, rl, rg, nx=nx, ny=ny, seed=seed, fill=fill)

    specs = request_stream(n=args.requests, rate=args.rate, steps_range=(args.min_steps, args.max_steps))
    mk = lambda: [serve.Request(rid=sp["id"], arrival=sp["arrival"], steps=sp["steps"], make=make(sp),  # noqa: E731
                                meta={"kind": sp["kind"], "nx": sp["nx"], "ny": sp["ny"]}) for sp in specs]
    print(f"[bench] serve {args.requests} requests at {args.rate}/s, budget {args.hbm_budget_gb} GB, "
          f"{args.slots} slots", file=sys.stderr, flush=True)
    server = serve.Server(hbm_budget=int(args.hbm_budget_gb * 2**30), max_slots=args.slots, chunk=args.chunk,
                          keep_results=False)
    _, served = server.run(mk())
    print(f"[bench] served: {json.dumps(served)}", file=sys.stderr, flush=True)
    # the same stream with shortest-work-first admission (the oldest request goes first after max_wait)
    shortest = serve.Server(hbm_budget=int(args.hbm_budget_gb * 2**30), max_slots=args.slots, chunk=args.chunk,
                            keep_results=False, policy="shortest", max_wait=args.max_wait)
    _, served_sw = shortest.run(mk())
    print(f"[bench] served, shortest work first: {json.dumps(served_sw)}", file=sys.stderr, flush=True)
    _, base_line = serve.fifo(mk(), keep_results=False)
    out = {"metric": METRIC, "mode": "served (continuous batching) vs FIFO plain", "unit": "MLUPS", "n_gpus": 1,
           "dtype": "f32",
           "config": {"workload": f"Poisson stream of {args.requests} mixed droplet/evaporation/boiling requests at "
                                  f"{args.rate} req/s, grids log-uniform 128x128..1024x2048, steps uniform "
                                  f"[{args.min_steps}, {args.max_steps}]",
                      "hbm_budget_gb": args.hbm_budget_gb, "slots": args.slots, "chunk": args.chunk},
           "served": served, "served_shortest_first": dict(served_sw, max_wait_s=args.max_wait), "fifo": base_line}
    print(json.dumps(out), flush=True)


LATTICES = (("D2Q5-MRT", {}), ("D2Q5-BGK", {"flags": 8}), ("D2Q9-BGK", {"thermal_q": 9}))


def _time_solver(s, steps):
    """ms per step of Solver s over `steps` graph-replayed steps (HIP events on its stream)."""
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s.stream)
    s.step(steps)
    e1.record(s.stream)
    e1.synchronize()
    s.sync()
    return e0.elapsed_time(e1) / steps


def _pulse_error(lbm, kw, rho0, n=128, s0=8.0, A=0.005, steps=400):
    """Frozen-flow Gaussian temperature pulse on the GPU (FP32) against the exact diffusion
    solution with D = lambda / (rho c_v): max |T - T_exact| / A, or the step of a numerical failure."""
    import numpy as np
    from workloads import FREEZE_FLOW, Params
    p = Params(nx=n, ny=n, **kw)
    p = p.replace(flags=p.flags | FREEZE_FLOW)
    T0 = 0.86 * lbm.critical_temperature(p)
    y, x = np.mgrid[0:n, 0:n].astype(float)
    r2 = (x - n / 2) ** 2 + (y - n / 2) ** 2
    T = T0 + A * np.exp(-r2 / (2 * s0 ** 2))
    s = lbm.Solver(p).init(np.full((n, n), rho0), 0 * T, 0 * T, T)
    try:
        for k in range(steps // 50):
            s.step(50)
            s.sync()
    except lbm.LbmError:
        s.close()
        return {"diverged_by_step": (k + 1) * 50}
    Tn = s.fields()[3]
    s.close()
    D = p.lambda_ / (rho0 * p.cv)
    s2 = s0 ** 2 + 2 * D * steps
    Ta = T0 + A * s0 ** 2 / s2 * np.exp(-r2 / (2 * s2))
    return {"max_err_over_A": float(np.abs(Tn - Ta).max() / A)}


def run_lattice_mode(args):
    """Thermal-lattice ablation (the paper's efficiency argument for the D2Q5 lattice): the
    D2Q5 model with the MRT collision of Eq. (39), its BGK variant (Eq. 21) and the D2Q9
    thermal lattice with the BGK collision, on the evaporation workload at 512 x 512 and at
    2048 x 2048 (a working set far beyond the 256 MB Infinity Cache), FP32.  Each variant runs at
    its best one-step tile shape (D2Q9 has no two-step shape), and the D2Q5 MRT also at its best
    shape overall.  Plus the frozen-flow Gaussian pulse error of each variant at rho c_v = 5 and 1."""
    import paper_2205_00686_amd as lbm
    from paper_2205_00686_amd import autotune
    from workloads import Params, evaporation

    base = Params()
    Tc = lbm.critical_temperature(base)
    rl, rg, _ = lbm.coexistence(base, 0.86 * Tc)
    one_step = [k for k, sh in enumerate(lbm.shapes(lbm.LBM_FP32)) if sh[3] == 1]
    rows = []
    for nx, ny in ((512, 512), (2048, 2048)):
        steps = args.steps if nx == 512 else max(200, args.steps // 16)
        for name, kw in LATTICES:
            w = evaporation(Tc, rl, rg, nx=nx, ny=ny, R=nx / 8.0, superheat=1.10, **kw)
            bytes_lu = 160 if kw.get("thermal_q") == 9 else 128
            s = lbm.Solver(w.params).init(w.rho, w.ux, w.uy, w.T)
            s.step(args.warmup)
            cand = [("one-step", one_step)] + ([("any", None)] if name == "D2Q5-MRT" else [])
            for label, c in cand:
                r = autotune.tune_solver(s, candidates=c, use_cache=False)
                ms = _time_solver(s, steps)
                rows.append({"grid": f"{nx}x{ny}", "lattice": name, "shapes": label,
                             "shape": shape_text(lbm, lbm.LBM_FP32, r.shape), "bytes_per_lu": bytes_lu,
                             "us_per_step": round(ms * 1e3, 3), "mlups": round(w.nodes / (ms * 1e-3) / 1e6, 1),
                             "roofline_frac": round(w.nodes * bytes_lu / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)})
                print(f"[bench] {rows[-1]}", file=sys.stderr, flush=True)
            s.close()
    pulses = {}
    for name, kw in LATTICES:
        for rho0 in (1.0, 0.2):
            pulses[f"{name} rho_cv={rho0 * 5:g}"] = _pulse_error(lbm, kw, rho0)
    print(f"[bench] pulse errors {pulses}", file=sys.stderr, flush=True)
    out = {"metric": METRIC, "mode": "thermal-lattice ablation", "unit": "MLUPS", "n_gpus": 1, "dtype": "f32",
           "config": {"workload": "droplet evaporation (R = nx/8, edges at 1.1 T_sat), FP32, 512x512 and 2048x2048",
                      "steps_512": args.steps, "warmup": args.warmup},
           "runs": rows, "gaussian_pulse": pulses}
    print(json.dumps(out), flush=True)


def run_fritz_mode(args):
    """Bubble departure diameter against gravity (the study of Section 4.3): one batched sweep,
    the first departure per gravity, and the least-squares slope of log D_d against log g."""
    import paper_2205_00686_amd as lbm
    from paper_2205_00686_amd import fritz
    from workloads import Params, boiling, head_limited_fill

    base = Params()
    Tc = lbm.critical_temperature(base)
    rl, rg, ps = lbm.coexistence(base, 0.86 * Tc)
    gs = [float(x) for x in args.gravities.split(",")]
    if args.open_top:
        # the paper's setting: the enclosure full of saturated liquid under an open top
        fill, extra, box = 1.05, {"open_top": 1}, "open top, full of liquid"
    else:
        fill, extra, box = head_limited_fill(rl, rg, ps, max(gs), args.ny), {}, "closed box"
    ws = [boiling(Tc, rl, rg, nx=args.nx, ny=args.ny, gravity=g, dT_rel=args.dT_rel, hot_width=args.hot_width,
                  fill=fill, noise=0.0, seed=1, **extra) for g in gs]
    print(f"[bench] fritz sweep: {len(gs)} gravities on {args.nx}x{args.ny}, {box}, fill {fill:.3f}, "
          f"hot spot dT {args.dT_rel} Tc (width {args.hot_width})", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    res = fritz.sweep(ws, rl, rg, max_steps=args.steps, check_every=args.check_every,
                      log=lambda r: print(f"[bench] g={r.gravity:.2e}: departure at step {r.step}, "
                                          f"D={r.diameter:.1f}", file=sys.stderr, flush=True))
    wall = time.perf_counter() - t0
    ok = [r for r in res if r.step > 0]
    fit = fritz.fit_power([r.gravity for r in ok], [r.diameter for r in ok]) if len(ok) >= 2 else (None, None, None)
    out = {"metric": "bubble departure diameter vs gravity (Fritz: D_d ~ g^-0.5)", "mode": "fritz",
           "config": {"workload": f"nucleate boiling {args.nx}x{args.ny}, T_sat 0.86 Tc, hot spot dT {args.dT_rel} Tc "
                                  f"(Gaussian width {args.hot_width}), contact angle 75, lambda 2/3, {box}, "
                                  f"fill {fill:.3f}", "precision": "fp32", "max_steps": args.steps,
                      "check_every": args.check_every},
           "departures": [{"g": r.gravity, "step": r.step, "area": r.area, "D": round(r.diameter, 3),
                           "y_centroid": round(r.y_centroid, 1), **r.meta} for r in res],
           "slope": None if fit[0] is None else round(fit[0], 4), "r2": None if fit[2] is None else round(fit[2], 4),
           "wall_s": round(wall, 2)}
    print(json.dumps(out), flush=True)


def _liquid(rho, rho_mid):
    """Liquid mass (sum of rho over nodes above the mid density), base half-width on the first
    fluid row and height of the liquid region on the wall, in lattice units."""
    import numpy as np
    liq = rho > rho_mid
    mass = float(rho[liq].sum())
    cols = np.nonzero(liq[0])[0]
    a = 0.5 * len(cols)
    h = float(liq.any(axis=1).nonzero()[0].max() + 1) if liq.any() else 0.0
    return mass, a, h


def run_heated_mode(args):
    """Droplet evaporation on a heated surface (Section 4.2): the heated_droplet workload (200 x 100,
    half disk of R = 35 on the wall, contact angle 90, open top at T_sat, lambda = 0.08).  Stage 1
    runs without heating (wall at T_sat) until the shape settles; its state is then loaded into a
    context whose wall is at T_h, and the liquid mass is followed until a fraction of it is left.
    Contact angle of the settled droplet from its base half-width a and height h (circular cap):
    cos(theta) = 1 - h / R with R = (a^2 + h^2) / (2 h)."""
    import math

    import paper_2205_00686_amd as lbm
    from workloads import Params, heated_droplet

    base = Params()
    Tc = lbm.critical_temperature(base)
    rl, rg, _ = lbm.coexistence(base, 0.86 * Tc)
    mid = 0.5 * (rl + rg)
    cold = heated_droplet(Tc, rl, rg, T_h_rel=0.86)
    s = lbm.Solver(cold.params).init(cold.rho, cold.ux, cold.uy, cold.T)
    t0 = time.perf_counter()
    s.step(args.pre_steps)
    m_pre, a, h = _liquid(s.fields()[0], mid)
    R = (a * a + h * h) / (2 * h)
    theta = math.degrees(math.acos(max(-1.0, min(1.0, 1 - h / R))))
    raw = s.save_state()
    s.close()
    hot = heated_droplet(Tc, rl, rg, T_h_rel=args.T_h)
    s = lbm.Solver(hot.params).init(cold.rho, cold.ux, cold.uy, cold.T)
    s.load_state(raw)
    curve = [(0, 1.0)]
    m0 = m_pre
    done = 0
    while done < args.steps:
        s.step(args.check_every)
        done += args.check_every
        m = _liquid(s.fields()[0], mid)[0]
        curve.append((done, round(m / m0, 5)))
        if m / m0 < args.stop_fraction:
            break
    wall = time.perf_counter() - t0
    s.close()
    half = next((t for t, f in curve if f <= 0.5), None)
    print(f"[bench] heated droplet: contact angle {theta:.1f} after {args.pre_steps} unheated steps; "
          f"half the liquid gone at step {half}", file=sys.stderr, flush=True)
    out = {"metric": "normalised droplet mass against time, droplet on a heated surface", "mode": "heated",
           "config": {"workload": "heated_droplet 200x100, R 35 on the wall, contact angle 90, open top at T_sat, "
                                  f"wall at {args.T_h} Tc after {args.pre_steps} unheated steps, lambda 0.08, FP32",
                      "check_every": args.check_every},
           "contact_angle_deg": round(theta, 1), "base_half_width": a, "height": h,
           "half_mass_step": half, "curve": curve[:: max(1, len(curve) // 40)], "wall_s": round(wall, 2)}
    print(json.dumps(out), flush=True)


def run_3d_mode(args):
    """The three-dimensional extension (include/lbm3d.h): an evaporating droplet of radius 16 in a
    Dirichlet temperature box, FP32, at 128^3 and 256^3.  (A droplet started from the tanh profile
    sends an inward pressure wave that focuses at its centre; from R = 32 on it pushes the density
    past the EOS limit within about 35 steps, in the FP64 oracle as on the GPU.)  Algorithmic bytes per node update:
    f 19 + 19, g 7 + 7, history 2 + 2 values = 224 B in FP32.  Both step paths are timed: the fused
    kernel (one per step) and the per-node kernels (three per step, whose per-node fields, 15
    planes, also pass through HBM); --z-chunk sets the fused path's planes per workgroup."""
    import torch

    import paper_2205_00686_amd as lbm
    from paper_2205_00686_amd import three_d
    from workloads import Params, evaporation3d

    base = Params()
    Tc = lbm.critical_temperature(base)
    rl, rg, _ = lbm.coexistence(base, 0.86 * Tc)
    rows = []
    if args.calibration_copy_mib > 0:
        calibration_copy(lbm, args.calibration_copy_mib)
    grids = [int(v) for v in args.grids3d.split(",")]
    paths = [{"fused": 0, "per-node": 1}[v] for v in args.paths3d.split(",")]
    for path, n in [(pa, g) for pa in paths for g in grids]:
        steps = args.steps if n <= 128 else max(20, args.steps * 128 ** 3 // n ** 3)
        w = evaporation3d(Tc, rl, rg, n=n, R=16.0, superheat=1.1)
        w.params = w.params.replace(path=path, z_chunk=args.z_chunk if path == 0 else 0)
        s = three_d.Solver3D(w.params).init(w.rho, w.ux, w.uy, w.uz, w.T)
        s.step(10)
        s.sync()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s.stream)
        s.step(steps)
        e1.record(s.stream)
        e1.synchronize()
        s.sync()
        ms = e0.elapsed_time(e1) / steps
        mass, _ = s.diagnostics()
        prof = TRAFFIC3D.get((n, path, args.z_chunk))
        traffic = prof["bytes"] if prof and prof["kernel_sha"] == _kernel_source_sha(KERNEL3D_SOURCES) else None
        achieved = w.nodes * 224 / (ms * 1e-3) / 1e9  # algorithmic GB/s (one launch per step on the fused path)
        rows.append({"grid": f"{n}^3", "path": "fused" if path == 0 else "per-node", "steps": steps,
                     "us_per_step": round(ms * 1e3, 2),
                     "mlups": round(w.nodes / (ms * 1e-3) / 1e6, 1),
                     "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                  "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                                  "kernel_sha": _kernel_source_sha(KERNEL3D_SOURCES)},
                     "mass_drift": abs(mass / float(w.rho.sum()) - 1.0)})
        print(f"[bench] 3d {rows[-1]}", file=sys.stderr, flush=True)
        s.close()
    out = {"metric": METRIC, "mode": "three-dimensional extension", "unit": "MLUPS", "n_gpus": 1, "dtype": "f32",
           "config": {"workload": "droplet (R 16) evaporating in a Dirichlet temperature box, D3Q19 + D3Q7, FP32",
                      "bytes_per_lu": 224},
           "runs": rows}
    print(json.dumps(out), flush=True)


def run_ceiling_mode(args):
    """Practical HBM ceiling: device-to-device copies of 64 MiB to 4 GiB with the library's
    streaming copy kernel (16-byte lanes, lbm_device_copy) and, for comparison, torch's copy, each
    counted as bytes read plus bytes written.  The sizes up to 128 MiB fit the 256 MB Infinity
    Cache with their destination; the larger ones stream from HBM."""
    import torch

    import paper_2205_00686_amd as lbm

    rows = []
    stream = torch.cuda.current_stream()
    for mib in (64, 128, 256, 1024, 4096):
        n = mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        row = {"copy_mib": mib}
        for name, fn in (("hip_copy16", lambda: lbm.device_copy(src, dst, stream)), ("torch_copy", lambda: dst.copy_(src))):
            for _ in range(3):
                fn()
            torch.cuda.synchronize()
            reps = max(5, 4096 // mib)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                fn()
            e1.record(stream)
            e1.synchronize()
            ms = e0.elapsed_time(e1) / reps
            row[name] = {"ms": round(ms, 4), "tb_per_s": round(2 * n * 4 / (ms * 1e-3) / 1e12, 3)}
        assert torch.equal(src, dst)
        rows.append(row)
        print(f"[bench] ceiling {rows[-1]}", file=sys.stderr, flush=True)
        del src, dst
        torch.cuda.empty_cache()
    print(json.dumps({"mode": "HBM copy ceiling", "unit": "TB/s", "peak_tb_per_s": HBM_PEAK_GBS / 1000, "runs": rows}),
          flush=True)


def calibration_copy(lbm, mib):
    """One copy of `mib` MiB with the library's streaming copy kernel: a kernel of known traffic
    (mib MiB read, mib MiB written) whose byte counters calibrate those of a profile."""
    import torch
    src = torch.ones(mib * (1 << 20) // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    lbm.device_copy(src, dst)
    torch.cuda.synchronize()
    del src, dst


def _kernel_source_sha(names=("lbm_step.hpp", "lbm_device.hpp")) -> str:
    """Digest of a kernel's sources (default: the two-dimensional step kernel; the fused
    three-dimensional kernel is lbm3d.hip with lbm_device.hpp): a profile's traffic figure applies
    only to sources with the digest it was taken with."""
    import hashlib
    h = hashlib.sha1()
    for name in names:
        with open(os.path.join(ROOT, "paper_2205_00686_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _timed_steps(s, n):
    """ms of one s.step(n) call from HIP events on the solver's stream, bracketed by device syncs."""
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s.stream)
    s.step(n)
    e1.record(s.stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def batched_summary(lbm, instances, steps, warmup):
    """The batched gravity sweep (64 boiling instances on 256x512 / 384x768 / 512x1024 grids): one
    batched, graph-replayed launch per step over every instance, against the same instances run one
    after the other with plain lbm_step calls (each grid size at its own autotuned tile shape).  Same
    steps for both; the first four instances are compared bit for bit."""
    import torch

    from paper_2205_00686_amd import autotune

    ws = sweep_workloads(instances, steps, lbm)
    nodes = sum(w.nodes for w in ws)
    print(f"[bench] batched: {len(ws)} boiling instances, {nodes} nodes, {steps} steps", file=sys.stderr, flush=True)
    solvers = [lbm.Solver(w.params).init(w.rho, w.ux, w.uy, w.T) for w in ws]
    stream = solvers[0].stream
    plain_shapes = {}
    for s in solvers:
        key = f"{s.nx}x{s.ny}"
        if key not in plain_shapes:
            plain_shapes[key] = autotune.tune_solver(s, use_cache=False).shape
        s.set_shape(plain_shapes[key])
        s.step(warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for s in solvers:
        s.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    for s in solvers:
        s.sync()
    plain_ms = e0.elapsed_time(e1)
    plain_state = [s.save_state() for s in solvers[:4]]
    for s in solvers:
        s.close()
    solvers = [lbm.Solver(w.params).init(w.rho, w.ux, w.uy, w.T) for w in ws]
    b = lbm.Batch(solvers)
    for i in range(len(solvers)):
        b.set_budget(i, warmup)
    b.step(warmup)
    b.sync()
    bt = autotune.tune_batch(b, use_cache=False)
    for i in range(len(solvers)):
        b.set_budget(i, steps)
    torch.cuda.synchronize()
    e0.record(b.stream)
    b.step(steps)
    e1.record(b.stream)
    torch.cuda.synchronize()
    st = b.sync()
    batch_ms = e0.elapsed_time(e1)
    same = all(s.save_state() == p for s, p in zip(solvers[:4], plain_state))
    b.close()
    for s in solvers:
        s.close()
    # the same batch as persistent launches (one kernel per graph replay, grid barriers between steps)
    solvers = [lbm.Solver(w.params).init(w.rho, w.ux, w.uy, w.T) for w in ws]
    b = lbm.Batch(solvers).set_shape(bt.shape).set_persistent(True)
    for i in range(len(solvers)):
        b.set_budget(i, warmup + steps)
    b.step(warmup)
    b.sync()
    torch.cuda.synchronize()
    e0.record(b.stream)
    b.step(steps)
    e1.record(b.stream)
    torch.cuda.synchronize()
    b.sync()
    pers_ms = e0.elapsed_time(e1)
    same_p = all(s.save_state() == p for s, p in zip(solvers[:4], plain_state))
    b.close()
    for s in solvers:
        s.close()
    lu = nodes * steps
    return {"workload": f"gravity sweep: {len(ws)} boiling instances on 256x512/384x768/512x1024 grids, g log-uniform "
                        f"[5e-6, 5e-5], hot-spot dT uniform [0.1, 0.3] Tc, pool fill 0.5 or head-limited, FP32",
            "instances": len(ws), "nodes": nodes, "steps": steps, "warmup": warmup,
            "batched_mlups": round(lu / (batch_ms * 1e-3) / 1e6, 1),
            "plain_sequential_mlups": round(lu / (plain_ms * 1e-3) / 1e6, 1),
            "speedup": round(plain_ms / batch_ms, 3),
            "batched_roofline_frac": round(lu * BYTES_PER_LU["f32"] / (batch_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "batch_tile_shape": shape_text(lbm, lbm.LBM_FP32, bt.shape),
            "plain_tile_shapes": {k: shape_text(lbm, lbm.LBM_FP32, v) for k, v in plain_shapes.items()},
            "persistent_mlups": round(lu / (pers_ms * 1e-3) / 1e6, 1),
            "persistent_equal_bits_first4": same_p,
            "equal_bits_first4": same, "failed_instances": sum(1 for x in st if x != 0)}


def served_summary(lbm, requests, rate, min_steps, max_steps, budget_gb, slots, chunk):
    """A Poisson stream of mixed droplet / evaporation / boiling requests (grids log-uniform between
    128x128 and 1024x2048): continuous batching (admission by HBM footprint, state kept on the device,
    requests joining between chunks) against one-at-a-time FIFO service with plain launches.
    Latency runs from arrival to fields on the host."""
    from paper_2205_00686_amd import serve
    from workloads import Params, boiling, droplet, evaporation, head_limited_fill, request_stream

    base = Params()
    Tc = lbm.critical_temperature(base)
    rl, rg, ps = lbm.coexistence(base, 0.86 * Tc)

    def make(spec):
        nx, ny, seed = spec["nx"], spec["ny"], spec["seed"]
        if spec["kind"] == "droplet":
            return lambda: droplet(Tc, rl, rg, nx=nx, ny=ny, R=min(nx, ny) / 4.0)
        if spec["kind"] == "evaporation":
            return lambda: evaporation(Tc, rl, rg, nx=nx, ny=ny, R=min(nx, ny) / 8.0)
        fill = head_limited_fill(rl, rg, ps, 2e-5, ny)
        return lambda: boiling(Tc, rl, rg, nx=nx, ny=ny, seed=seed, fill=fill)

    specs = request_stream(n=requests, rate=rate, steps_range=(min_steps, max_steps))
    mk = lambda: [serve.Request(rid=sp["id"], arrival=sp["arrival"], steps=sp["steps"], make=make(sp),  # noqa: E731
                                meta={"kind": sp["kind"], "nx": sp["nx"], "ny": sp["ny"]}) for sp in specs]
    print(f"[bench] served: {requests} requests at {rate}/s, budget {budget_gb} GB, {slots} slots",
          file=sys.stderr, flush=True)
    server = serve.Server(hbm_budget=int(budget_gb * 2**30), max_slots=slots, chunk=chunk, keep_results=False)
    _, served = server.run(mk())
    print(f"[bench] served {json.dumps(served)}", file=sys.stderr, flush=True)
    _, fifo = serve.fifo(mk(), keep_results=False)
    print(f"[bench] fifo {json.dumps(fifo)}", file=sys.stderr, flush=True)
    keep = ("completed", "failed", "latency_p50_s", "latency_p99_s", "makespan_s", "aggregate_mlups")
    return {"workload": f"Poisson stream of {requests} mixed droplet/evaporation/boiling requests at {rate} req/s, "
                        f"grids log-uniform 128x128..1024x2048, steps uniform [{min_steps}, {max_steps}], FP32",
            "hbm_budget_gb": budget_gb, "slots": slots, "chunk": chunk,
            "served": {k: (round(served[k], 4) if isinstance(served[k], float) else served[k]) for k in keep},
            "fifo": {k: (round(fifo[k], 4) if isinstance(fifo[k], float) else fifo[k]) for k in keep}}


def run_headline(args):
    """The benchmark line: the nucleate-boiling pool at 1024 x 2048 in FP32 (the largest
    single-GPU workload; its pool is filled to the head limit of the closed box, see
    workloads.head_limited_fill), W warm-up steps, tile shape autotuned, then exactly K steps in one
    lbm_step call timed with HIP events on the library's stream.  Beside it: repeats of the same call,
    the roofline of the step kernel, the batched sweep against plain launches, the served stream
    against FIFO, and the FP64 oracle on a bounded sample of the same workload."""
    import numpy as np
    import torch

    import paper_2205_00686_amd as lbm

    torch.cuda.set_device(0)
    w = build_workload(args.nx, args.ny, args.steps, args.workload)
    prec = lbm.LBM_FP64 if args.precision == "fp64" else lbm.LBM_FP32
    PREC = args.precision.upper()
    dtype = "f64" if prec == lbm.LBM_FP64 else "f32"
    s = lbm.Solver(w.params, precision=prec).init(w.rho, w.ux, w.uy, w.T)
    print(f"[bench] {args.nx}x{args.ny} {args.workload} {PREC}, warmup {args.warmup}, steps {args.steps}",
          file=sys.stderr, flush=True)
    if args.calibration_copy_mib > 0:
        calibration_copy(lbm, args.calibration_copy_mib)
    tune = choose_shape(s, args.shape)
    print(f"[bench] tile shape {s.shape}: {tune}", file=sys.stderr, flush=True)
    # untimed steps until the GPU has run settle_ms of them: after the autotuner's short calls and
    # host work the first launches run 8-10 % slower than in steady operation (clocks ramping up)
    settle_ms, settle_steps = 0.0, 0
    while settle_ms < args.settle_ms:
        settle_ms += _timed_steps(s, 64)
        settle_steps += 64
    s.step(args.warmup)
    s.sync()
    # ---- the timed region: exactly K steps in one call
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms = _timed_steps(s, args.steps)
    wall = time.perf_counter() - t0
    s.sync()  # raises if the device flagged a numerical failure
    nodes = w.nodes
    mlups = nodes * args.steps / (ms * 1e-3) / 1e6
    depth = lbm.shapes(prec)[s.shape][3]  # time steps per launch of the step kernel
    launches = -(-args.steps // depth)
    ms_per_launch = ms / launches
    # ---- repeats: separate calls of K steps, and calls repeated until 0.5 s of GPU time
    rep = sorted(nodes * args.steps / (_timed_steps(s, args.steps) * 1e-3) / 1e6 for _ in range(args.repeats))
    sus_ms, sus_steps = 0.0, 0
    while sus_ms < args.sustain_ms:
        sus_ms += _timed_steps(s, args.steps)
        sus_steps += args.steps
    s.sync()
    bytes_per_launch = BYTES_PER_LU[dtype] * nodes * depth
    achieved = bytes_per_launch / (ms_per_launch * 1e-3) / 1e9
    prof = TRAFFIC.get((args.workload, args.nx, args.ny, s.shape, dtype))
    sha = _kernel_source_sha()
    traffic = prof["bytes"] if prof and prof["kernel_sha"] == sha else None
    fields = s.fields()
    finite = all(bool(np.isfinite(f).all()) for f in fields)
    shape = s.shape
    s.close()
    if args.workload == "evaporation":
        wl = f"droplet evaporation in open space, {args.nx}x{args.ny}, R={64 * args.nx // 512}, edges at 1.1 T_sat"
    else:
        wl = (f"nucleate boiling on a heated wall, {args.nx}x{args.ny}, walls (75/90 deg), hot spot width 32 dT "
              f"0.2 Tc, g 2e-5, noise 1e-3 seed 1, pool fill {w.meta['fill']:.3f} (head limit of the closed box; "
              f"the stated fill 0.5 collapses the vapour column)")
    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": f"synthetic (seeded initial fields of the paper's {args.workload} problem)",
        "config": {"workload": f"{wl}, {PREC} populations", "nx": args.nx, "ny": args.ny,
                   "kernel": "fused D2Q9+D2Q5 step", "tile_shape": shape_text(lbm, prec, shape),
                   "tile_shape_ms_per_step": tune, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "algorithmic_bytes_per_launch": bytes_per_launch, "steps_per_launch": depth,
                     "kernel_ms_per_launch": round(ms_per_launch, 6),
                     "measured_hbm_gbs": round(traffic / (ms_per_launch * 1e-3) / 1e9, 1) if traffic else None,
                     "kernel_sha": sha},
        "settle": {"steps": settle_steps, "gpu_ms": round(settle_ms, 1)},
        "repeats": {"calls": args.repeats, "steps_each": args.steps,
                    "mlups_p50": round(rep[len(rep) // 2], 1) if rep else None,
                    "mlups_min": round(rep[0], 1) if rep else None, "mlups_max": round(rep[-1], 1) if rep else None},
        "sustained": {"steps": sus_steps, "gpu_s": round(sus_ms * 1e-3, 4),
                      "mlups": round(nodes * sus_steps / (sus_ms * 1e-3) / 1e6, 1) if sus_steps else None},
        "wall_s": round(wall, 4),
        "fields_finite": finite,
    }
    if not args.no_batched:
        out["batched"] = batched_summary(lbm, args.instances, args.batch_steps, args.batch_warmup)
    if not args.no_served:
        out["served"] = served_summary(lbm, args.serve_requests, args.rate, args.min_steps, args.max_steps,
                                       args.hbm_budget_gb, args.slots, args.chunk)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (FP64 oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_steps)
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mode", choices=["plain", "batch", "serve", "fritz", "lattice", "heated", "3d", "ceiling",
                                       "cpu-baseline", "readout"], default="plain")
    ap.add_argument("--cpu-scale", type=float, default=1.0,
                    help="cpu-baseline: fraction of each configuration's timed steps (1: as documented)")
    ap.add_argument("--gravities", default="1e-5,1.5e-5,2e-5,3e-5,4e-5,6e-5")
    ap.add_argument("--dT-rel", type=float, default=0.19)
    ap.add_argument("--hot-width", type=float, default=8.0)
    ap.add_argument("--open-top", action="store_true", help="fritz: the paper's open-top pool full of liquid")
    ap.add_argument("--T-h", type=float, default=0.95, help="heated: wall temperature / Tc")
    ap.add_argument("--pre-steps", type=int, default=20000, help="heated: unheated steps before the wall is heated")
    ap.add_argument("--stop-fraction", type=float, default=0.1, help="heated: stop when this much liquid is left")
    ap.add_argument("--check-every", type=int, default=250)
    ap.add_argument("--z-chunk", type=int, default=0, help="3d: z planes per workgroup of the fused kernel (0: auto)")
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32",
                    help="plain mode: working precision of the populations (FP64 moves 256 B per node update)")
    ap.add_argument("--grids3d", default="128,256", help="3d: edge lengths of the cubic grids")
    ap.add_argument("--paths3d", default="fused,per-node", help="3d: step paths to time")
    ap.add_argument("--instances", type=int, default=64)
    ap.add_argument("--requests", type=int, default=256)
    ap.add_argument("--rate", type=float, default=20.0)
    ap.add_argument("--min-steps", type=int, default=1000)
    ap.add_argument("--max-steps", type=int, default=20000)
    ap.add_argument("--hbm-budget-gb", type=float, default=8.0)
    ap.add_argument("--slots", type=int, default=64)
    ap.add_argument("--chunk", type=int, default=512)
    ap.add_argument("--max-wait", type=float, default=5.0,
                    help="serve: seconds after which the oldest queued request is admitted first (shortest-work policy)")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default 2000; 10000 with --mode batch)")
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--settle-ms", type=float, default=200.0,
                    help="plain mode: untimed steps for this much GPU time before the warm-up steps")
    ap.add_argument("--workload", choices=["evaporation", "boiling"], default="boiling",
                    help="plain mode: the boiling pool (default) or the evaporation workload")
    ap.add_argument("--nx", type=int, default=1024)
    ap.add_argument("--ny", type=int, default=2048)
    ap.add_argument("--repeats", type=int, default=5, help="plain mode: further timed calls of K steps")
    ap.add_argument("--sustain-ms", type=float, default=500.0,
                    help="plain mode: repeat K-step calls until this much GPU time for the sustained rate (0: skip)")
    ap.add_argument("--batch-steps", type=int, default=10000, help="plain mode: steps of the batched sweep")
    ap.add_argument("--batch-warmup", type=int, default=64)
    ap.add_argument("--serve-requests", type=int, default=256, help="plain mode: requests of the served stream")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=300)
    ap.add_argument("--shape", default="auto", help="tile shape index, or 'auto' to autotune (default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibration-copy-mib", type=int, default=0,
                    help="before the timed region, copy this many MiB device-to-device once (a plain copy "
                         "kernel of known size, used to scale the HBM byte counters of a profile)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the library runs each simulation on a single device "
              f"(--gpus {args.gpus} is not supported)", file=sys.stderr)
        sys.exit(2)
    if args.mode == "fritz":
        if args.nx == 1024 and args.ny == 2048:  # the paper's boiling domain unless a grid is given
            args.nx, args.ny = 150, 300
        args.steps = args.steps or 200000
        return run_fritz_mode(args)
    if args.mode == "3d":
        args.steps = args.steps or 400
        return run_3d_mode(args)
    if args.mode == "ceiling":
        return run_ceiling_mode(args)
    if args.mode == "cpu-baseline":
        return run_cpu_baseline_mode(args)
    if args.mode == "readout":
        args.steps = args.steps or 2000
        return run_readout_mode(args)
    if args.mode == "heated":
        args.steps = args.steps or 400000
        if args.check_every == 250:
            args.check_every = 1000
        return run_heated_mode(args)
    if args.mode == "lattice":
        args.steps = args.steps or 4000
        return run_lattice_mode(args)
    if args.steps is None:
        args.steps = 10000 if args.mode == "batch" else 2000
    if args.mode == "batch":
        return run_batch_mode(args)
    if args.mode == "serve":
        return run_serve_mode(args)

    return run_headline(args)


if __name__ == "__main__":
    main()
