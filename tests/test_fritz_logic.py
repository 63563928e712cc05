"""Host side of the bubble-departure readout: selection of departed bubbles among vapour
components (labelled on the device; here by the oracle's labelling of the same rows), the
row-profile trigger, and the power-law fit."""
import math

import numpy as np

from oracle.components import vapour_components
from paper_2205_00686_amd import fritz

RL, RG = 6.5, 0.38
MID = 0.5 * (RL + RG)


def _pool(nx=120, ny=200, surface=160):
    rho = np.full((ny, nx), RL)
    rho[surface:, :] = RG
    return rho


def _disk(rho, x0, y0, r):
    ny, nx = rho.shape
    yy, xx = np.mgrid[0:ny, 0:nx]
    dx = (xx - x0 + nx / 2) % nx - nx / 2  # periodic in x
    rho[(dx ** 2 + (yy - y0) ** 2) <= r * r] = RG
    return rho


def _departed(rho, y_surface, min_area=12):
    # the components as the device returns them, here from the oracle's labelling of the same rows
    comps = vapour_components(rho, MID, 0, y_surface + 1)
    return fritz.departed(comps, y_surface, min_area)


def test_departed_bubble_area_and_exclusions():
    rho = _disk(_pool(), 60, 80, 10.0)
    found = _departed(rho, y_surface=150)
    assert len(found) == 1
    area, yc, xext = found[0]
    assert abs(area - math.pi * 100) < 0.05 * math.pi * 100 and abs(yc - 80) < 0.5 and xext == 21
    # attached to the wall: not departed
    assert _departed(_disk(_pool(), 60, 8, 10.0), y_surface=150) == []
    # merged with the vapour above the pool: not departed
    assert _departed(_disk(_pool(), 60, 155, 10.0), y_surface=150) == []
    # two bubbles: largest first; one below the area cut
    rho = _disk(_disk(_pool(), 30, 60, 8.0), 90, 100, 2.0)
    found = _departed(rho, y_surface=150, min_area=20)
    assert len(found) == 1 and abs(found[0][1] - 60) < 0.5
    found = _departed(rho, y_surface=150, min_area=1)
    assert len(found) == 2 and found[0][0] > found[1][0]


def test_rows_up_to_the_surface_give_the_departures_of_the_whole_field():
    # a component that reaches the surface row is excluded whether or not the labelled rows
    # continue above it, so labelling rows [0, y_surface] finds what labelling every row finds
    rng = np.random.default_rng(8)
    for _ in range(5):
        rho = _pool(nx=60, ny=80, surface=70)
        for _ in range(6):
            rho = _disk(rho, rng.uniform(0, 60), rng.uniform(0, 80), rng.uniform(1, 9))
        whole = fritz.departed(vapour_components(rho, MID), 64)
        assert _departed(rho, y_surface=64) == whole


def test_row_profile_trigger():
    assert not fritz.gap_above_vapour(np.array([5, 5, 3, 0, 0, 0, 9, 9]), y_surface=6)  # vapour only at/above the surface
    assert fritz.gap_above_vapour(np.array([5, 5, 0, 0, 4, 4, 0, 0]), y_surface=6)
    assert fritz.gap_above_vapour(np.array([0, 0, 0, 3, 0, 0]), y_surface=6)  # bubble away from a dry wall
    assert not fritz.gap_above_vapour(np.array([4, 4, 4, 4, 0, 0]), y_surface=6)  # attached only


def test_power_law_fit():
    g = np.array([1e-5, 2e-5, 4e-5, 8e-5])
    a, b, r2 = fritz.fit_power(g, 3.0 * g ** -0.5)
    assert abs(a + 0.5) < 1e-12 and abs(r2 - 1.0) < 1e-12
