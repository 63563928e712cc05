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
- The density field is then read back and its vapour components are labelled (8-connected,
  periodic in x).  A component that touches neither the wall nor the vapour above the pool is a
  departed bubble; D = 2 sqrt(A / pi) from its area A.
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


def label_vapour(vapour: np.ndarray) -> tuple[np.ndarray, int]:
    """8-connected components of a boolean [ny][nx] mask, periodic in x (labels 1..n)."""
    from scipy import ndimage

    lab, n = ndimage.label(vapour, structure=np.ones((3, 3), dtype=bool))
    if n == 0:
        return lab, 0
    # join components across the periodic x boundary (diagonal neighbours included)
    parent = list(range(n + 1))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    ny, nx = vapour.shape
    for y in range(ny):
        a = lab[y, nx - 1]
        if not a:
            continue
        for dy in (-1, 0, 1):
            yy = y + dy
            if 0 <= yy < ny and lab[yy, 0]:
                ra, rb = find(a), find(lab[yy, 0])
                if ra != rb:
                    parent[max(ra, rb)] = min(ra, rb)
    roots = np.array([find(i) for i in range(n + 1)])
    lab = roots[lab]
    uniq = np.unique(lab[lab > 0])
    remap = np.zeros(n + 1, dtype=lab.dtype)
    remap[uniq] = np.arange(1, len(uniq) + 1)
    return remap[lab], len(uniq)


def departed_bubbles(rho: np.ndarray, rho_mid: float, y_surface: int, min_area: int = 12):
    """Vapour components that touch neither the bottom row nor any row at or above y_surface:
    [(area, y_centroid, x_extent)] sorted by area, largest first."""
    lab, n = label_vapour(rho < rho_mid)
    out = []
    for k in range(1, n + 1):
        ys, xs = np.nonzero(lab == k)
        if ys.min() == 0 or ys.max() >= y_surface or len(ys) < min_area:
            continue
        out.append((int(len(ys)), float(ys.mean()), int(xs.max() - xs.min() + 1)))
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
                rho = s.fields()[0]
                found = departed_bubbles(rho, rho_mid, y_surface, min_area)
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
