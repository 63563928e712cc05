"""Pins of the oracle's vapour-component labelling (the departure readout of Section 4.3):
8-connected components of {rho < thr}, periodic in x, with integer statistics per component."""
import itertools

import numpy as np
import pytest
from scipy import ndimage

from oracle.components import vapour_components

THR = 1.0


def _field(mask):
    return np.where(mask, 0.5, 2.0)


def _closure_labels(mask):
    """Brute force: the connectivity relation of vapour nodes closed transitively by repeated
    squaring of the adjacency matrix (8 neighbours, periodic in x)."""
    ny, nx = mask.shape
    nodes = [(y, x) for y in range(ny) for x in range(nx) if mask[y, x]]
    n = len(nodes)
    A = np.eye(n, dtype=bool)
    for i, (y, x) in enumerate(nodes):
        for j, (yy, xx) in enumerate(nodes):
            dx = min((x - xx) % nx, (xx - x) % nx)
            if abs(y - yy) <= 1 and dx <= 1:
                A[i, j] = True
    while True:
        B = (A.astype(np.int64) @ A.astype(np.int64)) > 0
        if (B == A).all():
            break
        A = B
    comps = {}
    for i, (y, x) in enumerate(nodes):
        members = tuple(sorted(y2 * nx + x2 for j, (y2, x2) in enumerate(nodes) if A[i, j]))
        comps[members[0]] = members
    return comps


def test_matches_scipy_away_from_the_x_edges():
    rng = np.random.default_rng(11)
    for p in (0.2, 0.45, 0.6):
        m = rng.random((40, 50)) < p
        m[:, :1] = False
        m[:, -1:] = False  # no contact across the periodic edge: plain 8-connected labelling
        lab, n = ndimage.label(m, structure=np.ones((3, 3), dtype=bool))
        got = vapour_components(_field(m), THR)
        assert len(got) == n
        for c in got:
            ys, xs = np.nonzero(lab == lab.flat[c["root"]])
            assert c["area"] == len(ys) and c["y_sum"] == int(ys.sum())
            assert (c["y_min"], c["y_max"], c["x_min"], c["x_max"]) == (ys.min(), ys.max(), xs.min(), xs.max())
            assert c["root"] == int((ys * 50 + xs).min())


def test_matches_transitive_closure_on_tiny_masks():
    rng = np.random.default_rng(5)
    for shape in [(3, 3), (4, 5), (5, 4), (6, 7), (2, 9)]:
        for _ in range(25):
            m = rng.random(shape) < rng.uniform(0.2, 0.7)
            exp = _closure_labels(m)
            got = vapour_components(_field(m), THR)
            assert sorted(c["root"] for c in got) == sorted(exp)
            nx = shape[1]
            for c in got:
                members = exp[c["root"]]
                ys = [k // nx for k in members]
                assert c["area"] == len(members) and c["y_sum"] == sum(ys)


def test_all_masks_of_a_3x4_grid_against_the_closure():
    for bits in itertools.product((False, True), repeat=12):
        m = np.array(bits).reshape(3, 4)
        exp = _closure_labels(m)
        got = vapour_components(_field(m), THR)
        assert {c["root"]: c["area"] for c in got} == {r: len(v) for r, v in exp.items()}


def test_periodic_edge_and_diagonals():
    m = np.zeros((6, 10), dtype=bool)
    m[2, 0] = m[3, 9] = True  # diagonal contact across the x edge
    assert len(vapour_components(_field(m), THR)) == 1
    m = np.zeros((6, 10), dtype=bool)
    m[2, 0] = m[4, 9] = True  # two rows apart: separate
    assert len(vapour_components(_field(m), THR)) == 2
    m = np.zeros((6, 10), dtype=bool)
    m[0, 3] = m[5, 3] = True  # rows do not wrap
    assert len(vapour_components(_field(m), THR)) == 2
    m = np.zeros((8, 8), dtype=bool)
    m[::2, ::2] = True
    m[1::2, 1::2] = True  # a checkerboard is one component through its diagonals
    c = vapour_components(_field(m), THR)
    assert len(c) == 1 and c[0]["area"] == 32 and c[0]["root"] == 0


def test_row_window_and_threshold():
    rng = np.random.default_rng(2)
    rho = rng.uniform(0.0, 2.0, (30, 20))
    full = vapour_components(rho, 1.0)
    assert sum(c["area"] for c in full) == int((rho < 1.0).sum())
    win = vapour_components(rho, 1.0, 10, 20)
    assert sum(c["area"] for c in win) == int((rho[10:20] < 1.0).sum())
    assert all(10 <= c["y_min"] <= c["y_max"] < 20 for c in win)
    # a node exactly at the threshold is not vapour
    rho = np.full((4, 4), 2.0)
    rho[1, 1] = 1.0
    assert vapour_components(rho, 1.0) == []
    # components partition the vapour nodes whatever their number
    m = rng.random((30, 20)) < 0.5
    got = vapour_components(_field(m), THR)
    assert sum(c["area"] for c in got) == int(m.sum())


@pytest.mark.parametrize("nx", [1, 2])
def test_narrow_grids(nx):
    m = np.ones((3, nx), dtype=bool)
    c = vapour_components(_field(m), THR)
    assert len(c) == 1 and c[0]["area"] == 3 * nx
