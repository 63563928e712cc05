"""Benchmark of the fused thermal LBM step on one MI355X.

Workload: droplet evaporation in open space -- 512 x 512 grid, FP32 populations, droplet of
radius 64 at the Maxwell densities of T_sat = 0.86 Tc in saturated vapour, box edges held at
1.1 T_sat, initial T uniform at T_sat, periodic flow.  One benchmark step is one time step of the
whole coupled D2Q9 + D2Q5 update (one fused kernel launch) over the grid.

Prints one JSON line: MLUPS over the timed steps, the roofline of the step kernel (algorithmic
128 bytes per node update in FP32 divided by the kernel's average duration from HIP events on
the library's stream), and the FP64 CPU oracle timed on a bounded sample of the same workload.

  python bench.py [--gpus 1] [--steps 20000] [--warmup 500] [--no-cpu-baseline]
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
# HBM bytes per launch of the step kernel measured with rocprofv3 FETCH_SIZE / WRITE_SIZE passes,
# scaled by the same counters read for a plain copy of known size (profiles/); keyed by grid size,
# None where no measurement of the current kernel exists
TRAFFIC = {(512, 512): 35257214}


def build_workload(nx=512, ny=512, steps=20000):
    import paper_2205_00686_amd as lbm
    from workloads import Params, evaporation

    base = Params()
    Tc = lbm.critical_temperature(base)
    rl, rg, _ = lbm.coexistence(base, 0.86 * Tc)
    return evaporation(Tc, rl, rg, nx=nx, ny=ny, R=64.0 * nx / 512, superheat=1.10, steps=steps)


def cpu_baseline(w, steps):
    """The FP64 oracle on the same workload for a bounded number of steps (host cores)."""
    import oracle

    oracle.build(force=False)
    o = oracle.Oracle(w.params).init(w.rho, w.ux, w.uy, w.T)
    o.step(2)  # warm caches
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    return {"value": w.nodes * steps / dt / 1e6, "unit": "MLUPS", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{w.params.nx}x{w.params.ny} evaporation, FP64, {steps} steps after 2 warm-up steps "
                      f"({dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--nx", type=int, default=512)
    ap.add_argument("--ny", type=int, default=512)
    ap.add_argument("--cpu-steps", type=int, default=2000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibration-copy-mib", type=int, default=0,
                    help="before the timed region, copy this many MiB device-to-device once (a plain copy "
                         "kernel of known size, used to scale the HBM byte counters of a profile)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the library runs each simulation on a single device "
              f"(--gpus {args.gpus} is not supported)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2205_00686_amd as lbm

    torch.cuda.set_device(0)
    w = build_workload(args.nx, args.ny, args.steps)
    s = lbm.Solver(w.params, precision=lbm.LBM_FP32).init(w.rho, w.ux, w.uy, w.T)
    stream = s.stream
    print(f"[bench] {args.nx}x{args.ny} evaporation FP32, warmup {args.warmup}, steps {args.steps}", file=sys.stderr,
          flush=True)

    if args.calibration_copy_mib > 0:
        n = args.calibration_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    s.step(args.warmup)
    s.sync()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    s.step(args.steps)
    ev1.record(stream)
    ev1.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    s.sync()  # raises if the device flagged a numerical failure
    ev_ms = ev0.elapsed_time(ev1)
    ms_per_step = ev_ms / args.steps
    nodes = w.nodes
    mlups = nodes * args.steps / (ev_ms * 1e-3) / 1e6

    # per-launch kernel duration from event pairs around single launches (no graph)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(200)]
    for a, b in evs:
        a.record(stream)
        s.step(1)
        b.record(stream)
    torch.cuda.synchronize()
    per_launch_ms = sorted(a.elapsed_time(b) for a, b in evs)
    launch_p50 = per_launch_ms[len(per_launch_ms) // 2]

    dtype = "f32"
    bytes_per_launch = BYTES_PER_LU[dtype] * nodes
    achieved = bytes_per_launch / (ms_per_step * 1e-3) / 1e9
    fields = s.fields()
    finite = all(bool((f == f).all()) for f in fields)

    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic (seeded initial fields of the paper's droplet-evaporation problem)",
        "config": {"workload": f"droplet evaporation in open space, {args.nx}x{args.ny}, FP32 populations, "
                               f"R={64 * args.nx // 512}, edges at 1.1 T_sat",
                   "nx": args.nx, "ny": args.ny, "precision": "fp32", "kernel": "fused D2Q9+D2Q5 step",
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": TRAFFIC.get((args.nx, args.ny)),
                     "bytes_per_launch": bytes_per_launch, "kernel_ms_timed_region": round(ms_per_step, 6),
                     "kernel_ms_single_launch_p50": round(launch_p50, 6)},
        "wall_s": round(wall, 4),
        "fields_finite": finite,
    }
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (FP64 oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
