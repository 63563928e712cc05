"""Bubble departure diameter against gravity (the nucleate-boiling study of Section 4.3).

Setting (the paper's problem, in a closed box):
- Saturated liquid pool at T_sat = 0.86 T_c on a wall at T_sat with a narrow hot spot at
  T_sat + dT in the middle, contact angle 75 degrees, lambda = 2/3, buoyancy (rho - rho_ave) g.
- A bubble nucleates on the hot spot, grows and departs.
- Fritz's analysis gives a departure diameter D_d proportional to g^(-1/2).

Measurement (every instance of the sweep runs in one batched launch per step):
- Every `check_every` steps the device counts, per row, the vapour nodes (rho below the mean of
  the coexistence densities) in a window around the hot spot (lbm_vapour_rows).
- A vapour row above a liquid gap, below the pool surface, triggers the measurement.
- The vapour components of the rows up to the surface are then labelled on the device
  (8-connected, periodic in x; lbm_vapour_components), and only their areas and bounds come
  back.  A component that touches neither the wall nor the vapour above the pool is a departed
  bubble; D = 2 sqrt(A / pi) from its area A.
- The first departure of each instance is kept.  The slope of log D_d against log g is fitted
  by least squares.

The pool is closed at the top here (the paper's top is open), so it is filled far enough that the
hydrostatic head of the vapour above it stays within half the saturation pressure at the largest
gravity of the sweep (workloads.head_limited_fill).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import LBM_FP32, Batch, Solver


def departed(components, y_surface: int, min_area: int = 12):
    """Departed bubbles among vapour components (dicts as Solver.vapour_components returns):
    those that touch neither the bottom row nor any row at or above y_surface and hold at least
    min_area nodes, as [(area, y_centroid, x_extent)], largest first."""
    out = []
    for c in components:
        if c["y_min"] == 0 or c["y_max"] >= y_surface or c["area"] < min_area:
            continue
        out.append((c["area"], c["y_sum"] / c["area"], c["x_max"] - c["x_min"] + 1))
    out.sort(reverse=True)
    return out


def gap_above_vapour(rows: np.ndarray, y_surface: int) -> bool:
    """Row profile trigger: some row below y_surface holds vapour above a row without any."""
    seen_gap = False
    for y in range(min(y_surface, len(rows))):
        if rows[y] == 0:
            seen_gap = True
        elif seen_gap:
            return True
    return False


@dataclass
class Departure:
    gravity: float
    step: int = -1          # first check at which a departed bubble was found (-1: none)
    area: int = 0
    diameter: float = float("nan")
    y_centroid: float = float("nan")
    profile_checks: int = 0
    meta: dict = field(default_factory=dict)


def fit_power(gs, ds):
    """Least-squares slope and R^2 of log d against log g."""
    x, y = np.log(np.asarray(gs, float)), np.log(np.asarray(ds, float))
    A = np.vstack([x, np.ones_like(x)]).T
    (a, b), *_ = np.linalg.lstsq(A, y, rcond=None)
    r2 = 1.0 - float(np.sum((y - (a * x + b)) ** 2) / np.sum((y - y.mean()) ** 2)) if len(x) > 2 else 1.0
    return float(a), float(b), r2


def sweep(workloads, rho_l: float, rho_g: float, max_steps: int = 60000, check_every: int = 250,
          window: int = None, surface_margin: int = 12, min_area: int = 12, precision: int = LBM_FP32, log=None):
    """Run the boiling `workloads` (one per gravity, same grid) as one batch until each shows its
    first departed bubble or max_steps pass.  Returns [Departure] in input order."""
    rho_mid = 0.5 * (rho_l + rho_g)
    sols = [Solver(w.params, precision=precision).init(w.rho, w.ux, w.uy, w.T) for w in workloads]
    b = Batch(sols)
    res = [Departure(gravity=-float(w.params.gy)) for w in workloads]
    for i in range(len(sols)):
        b.set_budget(i, max_steps)
    active = set(range(len(sols)))
    done = 0
    try:
        while active and done < max_steps:
            b.step(check_every)
            status = b.sync()
            done += check_every
            for i in sorted(active):
                w, s = workloads[i], sols[i]
                if status[i] != 0:
                    res[i].meta["failed_at"] = done
                    active.discard(i)
                    continue
                nx, ny = w.params.nx, w.params.ny
                x0 = int(round(w.params.hot_x0))
                half = (window or nx // 2) // 2
                y_surface = int(min(w.meta["fill"], 1.0) * ny) - surface_margin
                rows = s.vapour_rows(rho_mid, x0 - half, x0 + half)
                res[i].profile_checks += 1
                if not gap_above_vapour(rows, y_surface):
                    continue
                # components of the rows up to the surface, labelled on the device: one that reaches
                # row y_surface is excluded whether or not it continues above
                comps = s.vapour_components(rho_mid, 0, min(ny, y_surface + 1))
                found = departed(comps, y_surface, min_area)
                if not found:
                    continue
                area, yc, xext = found[0]
                res[i].step, res[i].area = done, area
                res[i].diameter = 2.0 * math.sqrt(area / math.pi)
                res[i].y_centroid, res[i].meta["x_extent"] = yc, xext
                b.set_budget(i, 0)
                active.discard(i)
                if log:
                    log(res[i])
    finally:
        b.close()
        for s in sols:
            s.close()
    return res
