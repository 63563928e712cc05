"""GPU runs at the largest grids.  Two dimensions: the largest grid the library accepts, one FP32
population plane of 65535 x 16383 nodes is 4 294 639 620 bytes, 320 KiB under the 2^32 - 1 bytes
that the step kernel's 32-bit byte offsets can address (the limit lbm_validate enforces).  Both
tile dimensions are ragged (65535 = 1023 x 64 + 63 columns, 16383 = 1023 x 16 + 15 rows).  In FP64
the same bytes hold 32767 x 16383 nodes (384 KiB under the limit, 511 x 64 + 63 columns).  Three
dimensions: grids whose planes are above 2^31 bytes, FP32 (184 GB of state) and FP64 (149 GB).

The oracle cannot run 1.07e9 nodes, so the test uses a property that holds at any size: the
update of a node depends only on its neighbourhood, so on a grid tiled with copies of a pattern
(periodic in x, and in y where the grid is periodic) the result is the same tiling of the
pattern's own result.  The pattern is run twice more, on the GPU and in the FP64 oracle:
  - the full grid must equal the tiled GPU pattern bit for bit, at every node (each node's
    arithmetic is fixed by the source, whatever the tile, shape or position);
  - the GPU pattern must match the oracle within the FP32 bounds of the parity tests.
The two global scalars of the state are made equal on both grids: the densities and temperatures
are multiples of 2^-19 and 2^-24, so the FP64 sums behind the mean density (buoyancy, Section 4.3)
and the temperature storage offset are exact and their means identical.

Each two-dimensional FP32 case steps twice with the two-step tile shape (one launch) and twice
with a one-step shape, so both kernels address the highest offsets (FP64, which has one-step
shapes only: 64 x 16 tiles, then 64 x 8); each three-dimensional case runs one
step path (fused or per-node) for four steps.  The largest case needs 184 GB of device memory and
about 70 GB of host memory.
"""
import numpy as np
import pytest

from workloads import Params, Workload

pytestmark = pytest.mark.gpu

NX, NY = 65535, 16383        # FP32: 255 x 257 columns, 127 x 129 rows
PX, PY = 255, 127            # pattern periods
NX64, PX64 = 32767, 217      # FP64 (8-byte values): 217 x 151 columns, 384 KiB under the limit
STEPS_TWO, STEPS_ONE = 2, 2


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_00686_amd as lbm
    return lbm


def _quantise(a, bits):
    return np.round(a * 2.0 ** bits) / 2.0 ** bits


def _pattern(orc, walls: bool, PX: int = PX):
    """Seeded pattern of PX columns: a periodic droplet cell (PY rows) or a full-height walled pool."""
    base = Params()
    Tc = orc.Tc(base)
    rl, rg, _ = orc.maxwell(base, 0.86 * Tc)
    ny = NY if walls else PY
    rng = np.random.default_rng(2205 + int(walls))
    y, x = np.mgrid[0:ny, 0:PX].astype(np.float64)
    if walls:
        rho = rg + 0.5 * (rl - rg) * (1.0 - np.tanh((y - 40.0) / 2.5))
        T = 0.9 * Tc - 0.04 * Tc * y / (ny - 1)
        p = Params(nx=PX, ny=ny, y_walls=1, T_bot=0.9 * Tc, T_top=0.86 * Tc, theta_bot_deg=75.0,
                   theta_top_deg=90.0, gy=-2e-5)
    else:
        dx = np.minimum(np.abs(x - PX / 2), PX - np.abs(x - PX / 2))
        dy = np.minimum(np.abs(y - PY / 2), PY - np.abs(y - PY / 2))
        rho = rg + 0.5 * (rl - rg) * (1.0 - np.tanh((np.hypot(dx, dy) - 30.0) / 2.5))
        T = 0.88 * Tc + 0.01 * Tc * np.sin(2 * np.pi * x / PX) + 0.005 * Tc * np.cos(2 * np.pi * y / PY)
        p = Params(nx=PX, ny=ny, gy=-2e-5)
    rho = _quantise(rho * (1.0 + 1e-3 * rng.uniform(-1, 1, rho.shape)), 19)
    T = _quantise(T * (1.0 + 1e-4 * rng.uniform(-1, 1, T.shape)), 24)
    ux = 1e-3 * rng.standard_normal(rho.shape)
    uy = 1e-3 * rng.standard_normal(rho.shape)
    return Workload("max-grid pattern", p, rho, ux, uy, T, STEPS_TWO + STEPS_ONE), rl


def _run(lbm, w, rows_rep, cols_rep, name, precision):
    """Solver on the pattern tiled rows_rep x cols_rep times.  FP32: the two-step shape, then shape 1;
    FP64 (one-step shapes only): shape 0 (64 x 16 tiles), then shape 1 (64 x 8)."""
    p = w.params.replace(nx=w.params.nx * cols_rep, ny=w.params.ny * rows_rep)
    s = lbm.Solver(p, precision=precision)
    s.init(*(np.tile(a, (rows_rep, cols_rep)) for a in (w.rho, w.ux, w.uy, w.T)))
    first = 0
    if precision == lbm.LBM_FP32:
        first = next(k for k, sh in enumerate(lbm.shapes(lbm.LBM_FP32)) if sh[3] == 2)
    assert lbm.shape_fits(p, first, precision) and lbm.shape_fits(p, 1, precision)
    s.set_shape(first).step(STEPS_TWO)
    s.set_shape(1).step(STEPS_ONE)
    print(f"   {name} {p.nx}x{p.ny}: stepped", flush=True)
    out = s.fields()
    s.close()
    return out


@pytest.mark.parametrize("fp64", [False, True], ids=["fp32", "fp64"])
@pytest.mark.parametrize("walls", [False, True], ids=["periodic", "walled"])
def test_largest_grid_equals_tiled_pattern(lbm, orc, walls, fp64):
    import torch

    nx, px, vb = (NX64, PX64, 8) if fp64 else (NX, PX, 4)
    precision = lbm.LBM_FP64 if fp64 else lbm.LBM_FP32
    assert nx % px == 0 and NY == PY * 129
    # the planes are within 384 KiB of the limit; a few more columns are rejected
    assert 2**32 - 1 - 2**19 < nx * NY * vb <= 2**32 - 1
    assert lbm.footprint_bytes(Params(nx=nx, ny=NY), precision) > 0
    assert lbm.footprint_bytes(Params(nx=(2**32 - 1) // (vb * NY) + 1, ny=NY), precision) == 0
    w, rl = _pattern(orc, walls, px)
    print(f"\n[case] largest grid {nx}x{NY} {'fp64' if fp64 else 'fp32'} {'walled' if walls else 'periodic'}",
          flush=True)

    small = _run(lbm, w, 1, 1, "pattern", precision)
    ref = orc.Oracle(w.params).init(w.rho, w.ux, w.uy, w.T)
    ref.step(STEPS_TWO + STEPS_ONE)
    exp = ref.fields()
    err = [float(np.abs(a - b).max()) for a, b in zip(small, exp)]
    print(f"   pattern vs oracle: rho={err[0]:.3e} ux={err[1]:.3e} uy={err[2]:.3e} T={err[3]:.3e}", flush=True)
    if fp64:  # rounding level, as the other FP64 parity tests
        assert err[0] <= 1e-11 and err[3] <= 1e-13 and max(err[1], err[2]) <= 1e-13
    else:
        assert err[0] <= 2e-4 * rl
        assert err[3] <= 2e-6 * float(np.abs(exp[3]).max())
        assert max(err[1], err[2]) <= 1e-5

    torch.cuda.empty_cache()
    rows_rep = 1 if walls else NY // PY
    big = _run(lbm, w, rows_rep, nx // px, "full grid", precision)
    torch.cuda.empty_cache()
    for name, b, s in zip(("rho", "ux", "uy", "T"), big, small):
        tiled = b.reshape(rows_rep, w.params.ny, nx // px, px)
        same = tiled == s[None, :, None, :]
        if not same.all():
            k = np.argwhere(~same)[0]
            raise AssertionError(f"{name} differs from the tiled pattern at tile ({k[0]}, {k[2]}), "
                                 f"pattern node ({k[3]}, {k[1]}): {tiled[tuple(k)]!r} vs {s[k[1], k[3]]!r}")
        del tiled, same
    print("   full grid equals the tiled pattern at every node", flush=True)


# ---- three dimensions.  A D3Q19 + D3Q7 state takes 276 bytes per node in FP32, so one GPU's memory
# runs out before the plane does: the grid 1020 x 1020 x 640 (plane 2 663 424 000 bytes, above the
# 2^31 bytes where a signed 32-bit offset would wrap; 184 GB) tiles a periodic 60 x 51 x 40 droplet
# cell.  Ragged column tiles in x (15 x 64 + 60) and y (127 x 8 + 4).
NX3, NY3, NZ3 = 1020, 1020, 640
PX3, PY3, PZ3 = 60, 51, 40
NZ3_64, PZ3_64 = 260, 52  # FP64 (552 bytes per node): plane 2 163 968 000 bytes, state 149 GB


def _pattern3(orc, pz: int = PZ3):
    from workloads import Params3D, Workload3D
    base = Params()
    Tc = orc.Tc(base)
    rl, rg, _ = orc.maxwell(base, 0.86 * Tc)
    rng = np.random.default_rng(22053)
    z, y, x = np.mgrid[0:pz, 0:PY3, 0:PX3].astype(np.float64)

    def per(a, n):
        return np.minimum(np.abs(a - n / 2), n - np.abs(a - n / 2))

    r = np.sqrt(per(x, PX3) ** 2 + per(y, PY3) ** 2 + per(z, pz) ** 2)
    rho = rg + 0.5 * (rl - rg) * (1.0 - np.tanh((r - 12.0) / 2.5))
    T = 0.88 * Tc + 0.01 * Tc * np.sin(2 * np.pi * x / PX3) + 0.005 * Tc * np.cos(2 * np.pi * z / pz)
    rho = _quantise(rho * (1.0 + 1e-3 * rng.uniform(-1, 1, rho.shape)), 19)
    T = _quantise(T * (1.0 + 1e-4 * rng.uniform(-1, 1, T.shape)), 24)
    u = [1e-3 * rng.standard_normal(rho.shape) for _ in range(3)]
    return Workload3D("max-grid pattern 3d", Params3D(nx=PX3, ny=PY3, nz=pz), rho, *u, T, 4), rl


def _run3(w, rep, path, name, precision=0):
    from paper_2205_00686_amd import three_d
    p = w.params.replace(nx=w.params.nx * rep[2], ny=w.params.ny * rep[1], nz=w.params.nz * rep[0], path=path)
    s = three_d.Solver3D(p, precision=precision)
    s.init(*(np.tile(a, rep) for a in (w.rho, w.ux, w.uy, w.uz, w.T)))
    s.step(w.steps)
    print(f"   {name} {p.nx}x{p.ny}x{p.nz} path {path}: stepped", flush=True)
    out = s.fields()
    s.close()
    return out


@pytest.mark.parametrize("fp64", [False, True], ids=["fp32", "fp64"])
@pytest.mark.parametrize("path", [0, 1], ids=["fused", "per_node"])
def test_largest_3d_grid_equals_tiled_pattern(lbm, orc, path, fp64):
    import torch
    from oracle import o3d
    from paper_2205_00686_amd import three_d
    from workloads import Params3D

    nz, pz, vb = (NZ3_64, PZ3_64, 8) if fp64 else (NZ3, PZ3, 4)
    rep = (nz // pz, NY3 // PY3, NX3 // PX3)
    assert (rep[0] * pz, rep[1] * PY3, rep[2] * PX3) == (nz, NY3, NX3)
    assert 2**31 < NX3 * NY3 * nz * vb <= 2**32 - 1
    assert three_d.footprint_bytes3(Params3D(nx=NX3, ny=NY3, nz=nz), int(fp64)) < 190e9
    w, rl = _pattern3(orc, pz)
    print(f"\n[case] largest 3d grid {NX3}x{NY3}x{nz} {'fp64' if fp64 else 'fp32'} path {path}", flush=True)

    small = _run3(w, (1, 1, 1), path, "pattern", int(fp64))
    ref = o3d.Oracle3D(w.params).init(w.rho, w.ux, w.uy, w.uz, w.T)
    ref.step(w.steps)
    exp = ref.fields()
    err = [float(np.abs(a - b).max()) for a, b in zip(small, exp)]
    print("   pattern vs oracle: " + " ".join(f"{v:.3e}" for v in err), flush=True)
    if fp64:
        assert err[0] <= 1e-11 and err[4] <= 1e-13 and max(err[1:4]) <= 1e-13
    else:
        assert err[0] <= 2e-4 * rl
        assert err[4] <= 2e-6 * float(np.abs(exp[4]).max())
        assert max(err[1:4]) <= 1e-5

    torch.cuda.empty_cache()
    big = _run3(w, rep, path, "full grid", int(fp64))
    torch.cuda.empty_cache()
    for name, b, s in zip(("rho", "ux", "uy", "uz", "T"), big, small):
        tiled = b.reshape(rep[0], pz, rep[1], PY3, rep[2], PX3)
        same = tiled == s[None, :, None, :, None, :]
        if not same.all():
            k = np.argwhere(~same)[0]
            raise AssertionError(f"{name} differs from the tiled pattern at tile ({k[0]}, {k[2]}, {k[4]}), "
                                 f"pattern node (z, y, x) = ({k[1]}, {k[3]}, {k[5]})")
        del tiled, same
    print("   full grid equals the tiled pattern at every node", flush=True)
