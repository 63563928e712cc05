"""MI355X (gfx950) library for the thermal pseudopotential lattice Boltzmann model of
Wang, Huang & He, "A new thermal lattice Boltzmann model for liquid-vapor phase change"
(arXiv:2205.00686).

The hot path (one fused D2Q9 + D2Q5 time step per kernel launch) lives in the HIP library
``liblbm.so`` behind the C ABI of ``include/lbm.h``.  This package only marshals arguments:
``Solver`` wraps one simulation (device memory from a torch uint8 tensor, work on the current
torch stream), ``Batch`` advances many simulations per launch, ``serve.Server`` runs the
continuous-batching request loop.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np

from . import _native
from ._native import LBM_BGK, LBM_FP32, LBM_FP64, LBM_FREEZE_FLOW, LBM_NO_S, NativeLibraryMissing

__all__ = ["Solver", "Batch", "LbmError", "params_struct", "coexistence", "critical_temperature",
           "footprint_bytes", "shapes", "shape_fits", "device_copy", "LBM_FP32", "LBM_FP64", "LBM_FREEZE_FLOW", "LBM_NO_S", "LBM_BGK",
           "NativeLibraryMissing"]


class LbmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"[{status}] {msg}")
        self.status = status


def _check(status: int, handle=None):
    if status != 0:
        L = _native.lib()
        text = L.lbm_strerror(status).decode()
        if handle:
            text += ": " + (L.lbm_last_error(handle) or b"").decode()
        raise LbmError(status, text)


_FIELDS = [name for name, _ in _native.LbmParams._fields_ if not name.startswith("reserved")]


def params_struct(prm, precision: int = LBM_FP32) -> _native.LbmParams:
    """lbm_params from any object carrying the parameter names (e.g. workloads.Params)."""
    c = _native.LbmParams()
    _native.lib().lbm_params_default(ctypes.byref(c), int(prm.nx), int(prm.ny))
    for name in _FIELDS:
        if name == "precision":
            continue
        if hasattr(prm, name):
            setattr(c, name, getattr(prm, name))
    c.precision = int(precision)
    return c


def shapes(precision: int = LBM_FP32):
    """Tile shapes of the step kernel compiled into the library:
    [(tile_x, tile_y, waves, steps_per_launch), ...]."""
    L = _native.lib()
    out = []
    for k in range(int(L.lbm_shape_count(int(precision)))):
        tx, ty, w, d = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(L.lbm_shape_info(int(precision), k, ctypes.byref(tx), ctypes.byref(ty), ctypes.byref(w),
                                ctypes.byref(d)))
        out.append((tx.value, ty.value, w.value, d.value))
    return out


def shape_fits(prm, k: int, precision: int = LBM_FP32) -> bool:
    """Whether tile shape k can run the grid of prm (two-step shapes need a grid larger than
    their halo region)."""
    c = params_struct(prm, precision)
    return bool(_native.lib().lbm_shape_fits(ctypes.byref(c), int(k)))


def critical_temperature(prm) -> float:
    c = params_struct(prm)
    return _native.lib().lbm_critical_temperature(ctypes.byref(c))


def coexistence(prm, T: float):
    """(rho_l, rho_g, p_sat) of the Maxwell construction of the EOS at T (library, FP64 host)."""
    c = params_struct(prm)
    rl, rg, ps = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(_native.lib().lbm_eos_coexistence(ctypes.byref(c), float(T), ctypes.byref(rl), ctypes.byref(rg),
                                             ctypes.byref(ps)))
    return rl.value, rg.value, ps.value


def footprint_bytes(prm, precision: int = LBM_FP32) -> int:
    c = params_struct(prm, precision)
    return int(_native.lib().lbm_footprint_bytes(ctypes.byref(c)))


def device_copy(src, dst, stream=None):
    """Copy the bytes of torch tensor src into dst (same byte count, a multiple of 16) with the
    library's streaming copy kernel, on `stream` (default: the current torch stream)."""
    import torch
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("source and destination sizes differ")
    st = stream if stream is not None else torch.cuda.current_stream(src.device)
    _check(_native.lib().lbm_device_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), nbytes,
                                         ctypes.c_void_p(st.cuda_stream)))


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


_streams = {}


def default_stream(device):
    """A per-device torch stream (default priority) for the library's work.  The legacy null
    stream cannot be captured into a graph, so the library is given a stream of its own."""
    import torch
    key = torch.device(device).index
    if key not in _streams:
        _streams[key] = torch.cuda.Stream(device=device)
    return _streams[key]


class Solver:
    """One simulation on the current GPU.  Device memory is a torch uint8 tensor owned here; work
    is enqueued on ``stream`` (default: a library stream per device, see default_stream)."""

    def __init__(self, prm, precision: int = LBM_FP32, device=None, stream=None):
        import torch

        L = _native.lib()
        self.prm = prm
        self.precision = precision
        self.params = params_struct(prm, precision)
        self.nx, self.ny = int(prm.nx), int(prm.ny)
        self.q = 9 if int(self.params.thermal_q) == 9 else 5  # velocities of the thermal lattice
        nbytes = int(L.lbm_footprint_bytes(ctypes.byref(self.params)))
        if nbytes == 0:
            raise LbmError(-1, "invalid parameters (lbm_validate)")
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.mem = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.stream = stream if stream is not None else default_stream(dev)
        self.mem.record_stream(self.stream)  # the allocator must not reuse it while the stream runs
        h = ctypes.c_void_p()
        _check(L.lbm_create(ctypes.byref(self.params), ctypes.c_void_p(self.mem.data_ptr()), nbytes,
                            ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self.handle = h
        self.footprint = nbytes

    def close(self):
        if getattr(self, "handle", None):
            self.stream.synchronize()
            _native.lib().lbm_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init(self, rho, ux, uy, T):
        arrs = [np.ascontiguousarray(a, dtype=np.float64).reshape(self.ny, self.nx) for a in (rho, ux, uy, T)]
        _check(_native.lib().lbm_init(self.handle, *(_dptr(a) for a in arrs)), self.handle)
        return self

    def step(self, n: int = 1):
        _check(_native.lib().lbm_step(self.handle, int(n)), self.handle)
        return self

    def sync(self):
        _check(_native.lib().lbm_sync(self.handle), self.handle)

    @property
    def steps(self) -> int:
        return int(_native.lib().lbm_steps_done(self.handle))

    @property
    def shape(self) -> int:
        """Index (into shapes(precision)) of the tile shape used by later steps."""
        return int(_native.lib().lbm_get_shape(self.handle))

    def set_shape(self, k: int):
        """Tile shape k for later steps; -1 restores the library's choice.  Results do not change."""
        _check(_native.lib().lbm_set_shape(self.handle, int(k)), self.handle)
        return self

    @property
    def tile_order(self) -> int:
        """Tile columns per strip of the order in which workgroups take the tiles (see
        lbm_set_tile_order)."""
        return int(_native.lib().lbm_get_tile_order(self.handle))

    def set_tile_order(self, order: int):
        """0: the library's choice; 1: whole tile rows; k >= 2: strips of k tile columns.  Results do
        not change."""
        _check(_native.lib().lbm_set_tile_order(self.handle, int(order)), self.handle)
        return self

    def fields(self):
        out = [np.empty((self.ny, self.nx)) for _ in range(4)]
        _check(_native.lib().lbm_read_fields(self.handle, *(_dptr(a) for a in out)), self.handle)
        return tuple(out)

    def vapour_rows(self, rho_threshold: float, x_lo: int = 0, x_hi: int = None) -> np.ndarray:
        """Per row, the number of columns in [x_lo, x_hi) whose density is below rho_threshold
        (computed on the device from the current state)."""
        x_hi = self.nx if x_hi is None else int(x_hi)
        out = np.zeros(self.ny, dtype=np.int32)
        _check(_native.lib().lbm_vapour_rows(self.handle, float(rho_threshold), int(x_lo), x_hi,
                                             out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))), self.handle)
        return out

    def vapour_components(self, rho_threshold: float, y_lo: int = 0, y_hi: int = None) -> list:
        """Connected vapour components (8-connected, periodic in x) of rows [y_lo, y_hi), labelled
        on the device: a list of dicts (root, area, y_min, y_max, x_min, x_max, y_sum) in
        increasing order of root, the smallest node index y * nx + x of each component."""
        y_hi = self.ny if y_hi is None else int(y_hi)
        cap = _native.LBM_MAX_COMPONENTS
        out = (_native.LbmComponent * cap)()
        n = ctypes.c_int()
        _check(_native.lib().lbm_vapour_components(self.handle, float(rho_threshold), int(y_lo), y_hi, out, cap,
                                                   ctypes.byref(n)), self.handle)
        names = [f[0] for f in _native.LbmComponent._fields_]
        return [{k: int(getattr(out[i], k)) for k in names} for i in range(n.value)]

    def diagnostics(self):
        m, e = ctypes.c_double(), ctypes.c_double()
        _check(_native.lib().lbm_diagnostics(self.handle, ctypes.byref(m), ctypes.byref(e)), self.handle)
        return m.value, e.value

    def set_diagnostics_interval(self, k: int):
        """Record mass and energy every k steps during later step() calls (0: stop); clears the log."""
        _check(_native.lib().lbm_set_diagnostics_interval(self.handle, int(k)), self.handle)
        return self

    def diagnostics_log(self, max_records: int = 256):
        """[(step, mass, energy), ...] recorded since the last call, oldest first."""
        n = int(max_records)
        st = (ctypes.c_int64 * n)()
        m, e = np.empty(n), np.empty(n)
        c = ctypes.c_int()
        _check(_native.lib().lbm_read_diagnostics_log(self.handle, st, _dptr(m), _dptr(e), n, ctypes.byref(c)),
               self.handle)
        return [(int(st[i]), float(m[i]), float(e[i])) for i in range(c.value)]

    def state_bytes(self) -> int:
        return int(_native.lib().lbm_state_bytes(self.handle))

    def save_state(self) -> bytes:
        buf = ctypes.create_string_buffer(self.state_bytes())
        _check(_native.lib().lbm_save_state(self.handle, buf, len(buf)), self.handle)
        return buf.raw

    def load_state(self, data: bytes):
        buf = ctypes.create_string_buffer(data, len(data))
        _check(_native.lib().lbm_load_state(self.handle, buf, len(data)), self.handle)

    def state(self, absolute: bool = True):
        """(f[9], g[Q], history[2]) host copies (Q = 5 or 9).  absolute=True: the populations and
        T(t-1), T(t-2) in FP64 with the library's storage offset undone (lbm_read_state);
        absolute=False: the raw planes in the working precision, as stored (g_i - what_i T_ref,
        T - T_ref)."""
        n, Q = self.nx * self.ny, self.q
        if absolute:
            f = np.empty((9, self.ny, self.nx))
            g = np.empty((Q, self.ny, self.nx))
            h = np.empty((2, self.ny, self.nx))
            _check(_native.lib().lbm_read_state(self.handle, _dptr(f), _dptr(g), _dptr(h)), self.handle)
            return f, g, h
        raw = self.save_state()
        dt = np.float64 if self.precision == LBM_FP64 else np.float32
        planes = 9 + Q + 2
        a = np.frombuffer(raw, dtype=dt, count=planes * n)
        f = a[:9 * n].reshape(9, self.ny, self.nx)
        g = a[9 * n:(9 + Q) * n].reshape(Q, self.ny, self.nx)
        h = a[(9 + Q) * n:planes * n].reshape(2, self.ny, self.nx)
        return f, g, h


class Batch:
    """Many initialised Solvers (same precision) advanced together: one kernel launch per step
    covers the tiles of every instance with budget left.  noalloc=True: the batch's table lives in
    the library's static per-device area (lbm_batch_create_noalloc) instead of a torch allocation;
    one such batch per device at a time."""

    def __init__(self, solvers, stream=None, noalloc: bool = False):
        import torch

        L = _native.lib()
        self.solvers = list(solvers)
        n = len(self.solvers)
        self.stream = stream if stream is not None else self.solvers[0].stream
        for s in self.solvers:  # the members' memory is also used on the batch's stream
            s.mem.record_stream(self.stream)
        arr = (ctypes.c_void_p * n)(*[s.handle.value for s in self.solvers])
        h = ctypes.c_void_p()
        if noalloc:
            self.mem = None
            _check(L.lbm_batch_create_noalloc(arr, n, ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        else:
            nbytes = int(L.lbm_batch_footprint_bytes(n))
            self.mem = torch.empty(nbytes, dtype=torch.uint8, device=self.solvers[0].mem.device)
            self.mem.record_stream(self.stream)
            _check(L.lbm_batch_create(arr, n, ctypes.c_void_p(self.mem.data_ptr()), nbytes,
                                      ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self.handle = h

    def set_budget(self, i: int, steps: int):
        _check(_native.lib().lbm_batch_set_budget(self.handle, int(i), int(steps)))

    def step(self, k: int):
        _check(_native.lib().lbm_batch_step(self.handle, int(k)))

    def remaining(self, i: int) -> int:
        return int(_native.lib().lbm_batch_remaining(self.handle, int(i)))

    @property
    def shape(self) -> int:
        return int(_native.lib().lbm_batch_get_shape(self.handle))

    def set_shape(self, k: int):
        """Tile shape k of the batched launches; -1 restores the library's choice."""
        _check(_native.lib().lbm_batch_set_shape(self.handle, int(k)))
        return self

    def set_persistent(self, on: bool = True, spin_limit: int = 0):
        """Launch each group of steps as one persistent kernel with grid barriers (same results);
        spin_limit bounds each barrier wait (0: the library's default)."""
        _check(_native.lib().lbm_batch_set_persistent(self.handle, 1 if on else 0, int(spin_limit)))
        return self

    def set_diagnostics_interval(self, k: int):
        """Every k batch steps, each member that advanced gets a (step, mass, energy) record in its
        own diagnostics log (Solver.diagnostics_log, readable after sync); 0 stops."""
        _check(_native.lib().lbm_batch_set_diagnostics_interval(self.handle, int(k)))
        return self

    def sync(self):
        """Wait for the batch; per-member status (0, or -4 for a member parked after a numerical
        failure).  Raises LbmError if the wait itself failed or a persistent launch's barrier timed
        out (every member is then failed)."""
        n = len(self.solvers)
        st = (ctypes.c_int * n)()
        rc = _native.lib().lbm_batch_sync(self.handle, st)
        if rc not in (_native.LBM_OK, _native.LBM_E_NUMERIC):
            _check(rc, self.solvers[0].handle)
        return list(st)

    def close(self):
        """Release the batch.  While every member is still open, their steps are first brought up
        to date (lbm_batch_sync), so they can go on alone."""
        if getattr(self, "handle", None):
            L = _native.lib()
            if all(getattr(s, "handle", None) for s in self.solvers):
                L.lbm_batch_sync(self.handle, None)  # a failure stays recorded in each member
            self.stream.synchronize()
            rc = L.lbm_batch_destroy(self.handle)
            self.handle = None
            _check(rc)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
