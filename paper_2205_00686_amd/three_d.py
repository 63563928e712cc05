"""Three-dimensional extension through the C ABI of include/lbm3d.h (argument marshalling
only): D3Q19 pseudopotential flow coupled to the paper's temperature model on D3Q7."""
from __future__ import annotations

import ctypes

import numpy as np

from . import _native
from ._native import LBM_FP32, LBM_FP64


def params3_struct(prm, precision: int = LBM_FP32) -> _native.Lbm3dParams:
    """lbm3d_params from any object carrying the parameter names (e.g. workloads.Params3D)."""
    c = _native.Lbm3dParams()
    _native.lib().lbm3d_params_default(ctypes.byref(c), int(prm.nx), int(prm.ny), int(prm.nz))
    for name, _ in _native.Lbm3dParams._fields_:
        if name.startswith("reserved") or name == "precision":
            continue
        if hasattr(prm, name):
            setattr(c, name, getattr(prm, name))
    c.precision = int(precision)
    return c


def footprint_bytes3(prm, precision: int = LBM_FP32) -> int:
    return int(_native.lib().lbm3d_footprint_bytes(ctypes.byref(params3_struct(prm, precision))))


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Solver3D:
    """One three-dimensional simulation on the current GPU; fields are (nz, ny, nx) arrays."""

    def __init__(self, prm, precision: int = LBM_FP32, stream=None):
        import torch

        from . import LbmError, _check, default_stream
        self._check, self.LbmError = _check, LbmError
        L = _native.lib()
        self.params = params3_struct(prm, precision)
        self.precision = precision
        self.shape = (int(prm.nz), int(prm.ny), int(prm.nx))
        nbytes = int(L.lbm3d_footprint_bytes(ctypes.byref(self.params)))
        if nbytes == 0:
            raise LbmError(-1, "invalid parameters (lbm3d_validate)")
        dev = torch.device("cuda", torch.cuda.current_device())
        self.mem = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.stream = stream if stream is not None else default_stream(dev)
        self.mem.record_stream(self.stream)
        h = ctypes.c_void_p()
        _check(L.lbm3d_create(ctypes.byref(self.params), ctypes.c_void_p(self.mem.data_ptr()), nbytes,
                              ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self.handle = h
        self.footprint = nbytes

    def init(self, rho, ux, uy, uz, T):
        arrs = [np.ascontiguousarray(a, dtype=np.float64).reshape(self.shape) for a in (rho, ux, uy, uz, T)]
        self._status(_native.lib().lbm3d_init(self.handle, *(_dptr(a) for a in arrs)))
        return self

    def step(self, n: int = 1):
        self._status(_native.lib().lbm3d_step(self.handle, int(n)))
        return self

    def sync(self):
        self._status(_native.lib().lbm3d_sync(self.handle))

    @property
    def steps(self) -> int:
        return int(_native.lib().lbm3d_steps_done(self.handle))

    def fields(self):
        out = [np.empty(self.shape) for _ in range(5)]
        self._status(_native.lib().lbm3d_read_fields(self.handle, *(_dptr(a) for a in out)))
        return tuple(out)  # rho, ux, uy, uz, T

    def diagnostics(self):
        m, e = ctypes.c_double(), ctypes.c_double()
        self._status(_native.lib().lbm3d_diagnostics(self.handle, ctypes.byref(m), ctypes.byref(e)))
        return m.value, e.value

    def state_bytes(self) -> int:
        return int(_native.lib().lbm3d_state_bytes(self.handle))

    def save_state(self) -> bytes:
        """Raw state (f, g, history in the working precision, step count, T_ref) as bytes."""
        buf = ctypes.create_string_buffer(self.state_bytes())
        self._status(_native.lib().lbm3d_save_state(self.handle, buf, len(buf)))
        return buf.raw

    def load_state(self, data: bytes):
        buf = ctypes.create_string_buffer(data, len(data))
        self._status(_native.lib().lbm3d_load_state(self.handle, buf, len(data)))
        return self

    def _status(self, s):
        if s != 0:
            L = _native.lib()
            raise self.LbmError(s, L.lbm_strerror(s).decode())

    def close(self):
        if getattr(self, "handle", None):
            self.stream.synchronize()
            _native.lib().lbm3d_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
