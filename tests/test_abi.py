"""The C-ABI library loads on a machine without a GPU, exports every symbol include/lbm.h
declares, and its host-only entry points behave (no device work is done here)."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = "".join(open(os.path.join(ROOT, "include", n)).read() for n in ("lbm.h", "lbm3d.h"))
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm(?:3d)?_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    from paper_2205_00686_amd import _native
    return _native.lib()


def test_every_declared_symbol_is_exported(L):
    from paper_2205_00686_amd import _native
    syms = _declared_symbols()
    assert len(syms) >= 20
    assert set(syms) == set(_native.EXPORTS)
    for s in syms:
        assert hasattr(L, s), s


def test_3d_validate_and_footprint(L):
    from paper_2205_00686_amd import _native
    p = _native.Lbm3dParams()
    L.lbm3d_params_default(ctypes.byref(p), 64, 48, 32)
    assert L.lbm3d_validate(ctypes.byref(p)) == 0
    n = 64 * 48 * 32
    assert 276 * n <= L.lbm3d_footprint_bytes(ctypes.byref(p)) <= 276 * n + 64 * 1024
    p.precision = 1
    assert 552 * n <= L.lbm3d_footprint_bytes(ctypes.byref(p)) <= 552 * n + 64 * 1024
    for field, bad in (("nz", 2), ("nu", 0.0), ("wdot", 1.0), ("precision", 3), ("flags", 8), ("s_e", 2.5),
                       ("z_chunk", -1), ("path", 2)):
        q = _native.Lbm3dParams()
        L.lbm3d_params_default(ctypes.byref(q), 16, 16, 16)
        setattr(q, field, bad)
        assert L.lbm3d_validate(ctypes.byref(q)) == -1, field
        assert L.lbm3d_footprint_bytes(ctypes.byref(q)) == 0
    q = _native.Lbm3dParams()
    L.lbm3d_params_default(ctypes.byref(q), 16, 16, 16)
    q.thermal_box = 1  # no box temperature
    assert L.lbm3d_validate(ctypes.byref(q)) == -1
    q.thermal_box, q.path, q.z_chunk = 0, _native.LBM3D_PATH_PER_NODE, 5
    assert L.lbm3d_validate(ctypes.byref(q)) == 0


def test_library_carries_gfx950_code_object():
    so = os.path.join(ROOT, "paper_2205_00686_amd", "liblbm.so")
    assert b"amdgcn-amd-amdhsa--gfx950" in open(so, "rb").read()


def test_validate_and_footprint(L):
    from paper_2205_00686_amd import _native
    p = _native.LbmParams()
    L.lbm_params_default(ctypes.byref(p), 512, 512)
    assert L.lbm_validate(ctypes.byref(p)) == 0
    n = 512 * 512
    fp = L.lbm_footprint_bytes(ctypes.byref(p))
    assert 128 * n <= fp <= 128 * n + 64 * 1024  # f, g and history twice, FP32, plus a small control block
    p.precision = 1
    assert 256 * n <= L.lbm_footprint_bytes(ctypes.byref(p)) <= 256 * n + 64 * 1024
    # D2Q9 thermal lattice: 4 more populations in two copies, 160 B per node in FP32
    p.thermal_q = 9
    assert 320 * n <= L.lbm_footprint_bytes(ctypes.byref(p)) <= 320 * n + 64 * 1024
    p.precision = 0
    assert 160 * n <= L.lbm_footprint_bytes(ctypes.byref(p)) <= 160 * n + 64 * 1024
    p.flags = _native.LBM_BGK | _native.LBM_NO_S
    assert L.lbm_validate(ctypes.byref(p)) == 0
    for field, bad in (("nx", 2), ("ny", 1), ("nu", -0.1), ("s_e", 2.0), ("wdot", 1.0), ("cv", 0.0),
                       ("precision", 7), ("lambda_", 0.0), ("thermal_q", 7), ("flags", 4)):
        q = _native.LbmParams()
        L.lbm_params_default(ctypes.byref(q), 64, 64)
        setattr(q, field, bad)
        assert L.lbm_validate(ctypes.byref(q)) == -1, field
        assert L.lbm_footprint_bytes(ctypes.byref(q)) == 0
    q = _native.LbmParams()
    L.lbm_params_default(ctypes.byref(q), 64, 64)
    q.y_walls = 1  # walls without wall temperatures
    assert L.lbm_validate(ctypes.byref(q)) == -1
    q.T_bot = q.T_top = 0.09
    assert L.lbm_validate(ctypes.byref(q)) == 0
    q.open_top = 1
    assert L.lbm_validate(ctypes.byref(q)) == 0
    q.y_walls = 0  # an open top needs the bottom wall
    assert L.lbm_validate(ctypes.byref(q)) == -1


def test_create_rejects_small_or_misaligned_buffers(L):
    from paper_2205_00686_amd import _native
    p = _native.LbmParams()
    L.lbm_params_default(ctypes.byref(p), 64, 64)
    h = ctypes.c_void_p()
    need = L.lbm_footprint_bytes(ctypes.byref(p))
    # host-side argument checks happen before any device call
    assert L.lbm_create(ctypes.byref(p), ctypes.c_void_p(4096), need - 1, None, ctypes.byref(h)) == -2
    assert L.lbm_create(ctypes.byref(p), ctypes.c_void_p(4097), need, None, ctypes.byref(h)) == -1
    assert L.lbm_create(ctypes.byref(p), None, need, None, ctypes.byref(h)) == -1


def test_default_parameters_are_the_papers(L):
    from paper_2205_00686_amd import _native
    p = _native.LbmParams()
    L.lbm_params_default(ctypes.byref(p), 10, 20)
    assert (p.nx, p.ny) == (10, 20)
    assert p.a == pytest.approx(3 / 49) and p.b == pytest.approx(2 / 21) and p.R == 1 and p.G == -1
    assert p.acentric == 0.344 and p.nu == 0.1 and p.cv == 5.0 and p.lambda_ == pytest.approx(1 / 3)
    assert math.isnan(p.rho_ave)


def test_critical_temperature_and_coexistence_agree_with_oracle(L, orc, base_params):
    """Two independent implementations of the Maxwell construction (library: Gauss-Legendre,
    golden section; oracle: Simpson, scan) agree."""
    import paper_2205_00686_amd as lbm
    Tc = lbm.critical_temperature(base_params)
    assert Tc == pytest.approx(orc.Tc(base_params), rel=1e-15)
    for tr in (0.8, 0.86, 0.9, 0.946):
        a = lbm.coexistence(base_params, tr * Tc)
        b = orc.maxwell(base_params, tr * Tc)
        assert a[0] == pytest.approx(b[0], rel=1e-9)
        assert a[1] == pytest.approx(b[1], rel=1e-8)
        assert a[2] == pytest.approx(b[2], rel=1e-8)
    with pytest.raises(lbm.LbmError):
        lbm.coexistence(base_params, 1.05 * Tc)


def test_strerror(L):
    for s in (0, -1, -2, -3, -4, -5):
        assert len(L.lbm_strerror(s)) > 0


def test_plane_size_limit(L):
    """A population plane must stay below 2^32 bytes (the step kernel's 32-bit byte offsets)."""
    from paper_2205_00686_amd import _native
    p = _native.LbmParams()
    L.lbm_params_default(ctypes.byref(p), 32768, 32767)  # 4 * 32768 * 32767 < 2^32
    assert L.lbm_validate(ctypes.byref(p)) == 0
    p.ny = 32768  # exactly 2^32 bytes
    assert L.lbm_validate(ctypes.byref(p)) == -1
    p.precision = 1
    p.ny = 16383  # 8 * 32768 * 16383 < 2^32
    assert L.lbm_validate(ctypes.byref(p)) == 0
    p.ny = 16384
    assert L.lbm_validate(ctypes.byref(p)) == -1


def test_tile_shapes_api(L):
    from paper_2205_00686_amd import shapes
    for prec in (0, 1):
        n = L.lbm_shape_count(prec)
        assert n >= 4
        got = shapes(prec)
        assert len(got) == n
        for tx, ty, w, d in got:
            assert tx == 64 and ty % w == 0 and 1 <= w <= 16 and ty in (4, 8, 16, 32) and d in (1, 2)
        assert len(set(got)) == n
        assert got[0][3] == 1 and (prec == 1) == all(d == 1 for *_, d in got)  # two-step shapes: FP32 only
        tx, ty, w, d = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        assert L.lbm_shape_info(prec, n, ctypes.byref(tx), ctypes.byref(ty), ctypes.byref(w), ctypes.byref(d)) == -1
        assert L.lbm_shape_info(prec, -1, None, None, None, None) == -1
        assert L.lbm_shape_info(prec, 0, None, None, None, None) == 0
    assert L.lbm_shape_count(7) == 0
    assert L.lbm_shape_info(7, 0, None, None, None, None) == -1
    # contexts and batches: NULL handles are rejected without touching a device
    assert L.lbm_set_shape(None, 0) == -1
    assert L.lbm_get_shape(None) == -1
    assert L.lbm_batch_set_shape(None, 0) == -1
    assert L.lbm_batch_get_shape(None) == -1


def test_two_step_shapes_need_a_grid_larger_than_their_halo(L):
    from paper_2205_00686_amd import _native, shape_fits, shapes
    from workloads import Params
    two = [k for k, s in enumerate(shapes(0)) if s[3] == 2]
    assert two
    for k in two:
        ty = shapes(0)[k][1]
        assert shape_fits(Params(nx=79, ny=ty + 11), k)
        assert not shape_fits(Params(nx=78, ny=ty + 11), k)
        assert not shape_fits(Params(nx=79, ny=ty + 10), k)
    assert all(shape_fits(Params(nx=3, ny=3), k) for k, s in enumerate(shapes(0)) if s[3] == 1)
    # the LDS of a two-step launch holds D2Q5 thermal populations only
    for k in two:
        assert not shape_fits(Params(nx=512, ny=512, thermal_q=9), k)
    assert all(shape_fits(Params(nx=512, ny=512, thermal_q=9), k) for k, s in enumerate(shapes(0)) if s[3] == 1)
    # an open top runs its boundary pass between steps: one-step shapes only
    op = Params(nx=512, ny=512, y_walls=1, open_top=1, T_bot=0.09, T_top=0.09)
    assert not any(shape_fits(op, k) for k in two)
    assert all(shape_fits(op, k) for k, s in enumerate(shapes(0)) if s[3] == 1)
    p = _native.LbmParams()
    L.lbm_params_default(ctypes.byref(p), 2, 64)  # invalid parameters
    assert L.lbm_shape_fits(ctypes.byref(p), 0) == 0


def test_3d_binding_carries_path_and_chunking(L):
    """three_d.params3_struct copies every field the parameter object names, including the step
    path and the z chunking of the fused kernel; defaults are the fused path, automatic chunking."""
    from paper_2205_00686_amd import _native, three_d
    from workloads import Params3D
    c = three_d.params3_struct(Params3D(nx=20, ny=12, nz=9))
    assert c.path == _native.LBM3D_PATH_FUSED and c.z_chunk == 0
    c = three_d.params3_struct(Params3D(nx=20, ny=12, nz=9, path=1, z_chunk=3), precision=_native.LBM_FP64)
    assert (c.nx, c.ny, c.nz, c.precision, c.path, c.z_chunk) == (20, 12, 9, 1, 1, 3)
    assert L.lbm3d_validate(ctypes.byref(c)) == 0
