"""Vapour components of a density field, for the bubble-departure readout of Section 4.3.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``): only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it.

The paper measures the diameter of a bubble when it leaves the heated wall (departure diameter
against gravity).  A departed bubble is a connected region of vapour that touches neither the wall
nor the vapour above the pool.  Here a node is vapour where its density is below a threshold (the
mean of the coexistence densities), two vapour nodes are connected when they are neighbours among
the eight lattice neighbours, and the domain is periodic in x (rows are not wrapped).

``vapour_components`` is the plain definition: a breadth-first flood fill from every unvisited
vapour node in increasing node order, in pure Python.  Pins (``tests/test_oracle_components.py``):
scipy's labelling on masks away from the x edges, brute-force transitive closure on tiny masks,
hand-made cases across the periodic edge, and counting identities.
"""
from __future__ import annotations

from collections import deque

import numpy as np


def vapour_components(rho: np.ndarray, thr: float, y_lo: int = 0, y_hi: int | None = None) -> list:
    """Components of {rho < thr} in rows [y_lo, y_hi) of rho[ny][nx]: a list of dicts with root
    (smallest node index y * nx + x), area, y_min, y_max, x_min, x_max and y_sum (sum of the
    rows), in increasing order of root."""
    ny, nx = rho.shape
    y_hi = ny if y_hi is None else y_hi
    vap = (np.asarray(rho, dtype=np.float64) < thr).tolist()
    seen = [[False] * nx for _ in range(ny)]
    out = []
    for y0 in range(y_lo, y_hi):
        for x0 in range(nx):
            if not vap[y0][x0] or seen[y0][x0]:
                continue
            seen[y0][x0] = True
            queue = deque([(y0, x0)])
            area, ysum = 0, 0
            ymin = ymax = y0
            xmin = xmax = x0
            while queue:
                y, x = queue.popleft()
                area += 1
                ysum += y
                ymin, ymax = min(ymin, y), max(ymax, y)
                xmin, xmax = min(xmin, x), max(xmax, x)
                for dy in (-1, 0, 1):
                    yy = y + dy
                    if yy < y_lo or yy >= y_hi:
                        continue
                    for dx in (-1, 0, 1):
                        xx = (x + dx) % nx
                        if vap[yy][xx] and not seen[yy][xx]:
                            seen[yy][xx] = True
                            queue.append((yy, xx))
            # the scan visits nodes in increasing index, so the first node of a component is its root
            out.append({"root": y0 * nx + x0, "area": area, "y_min": ymin, "y_max": ymax,
                        "x_min": xmin, "x_max": xmax, "y_sum": ysum})
    return out
