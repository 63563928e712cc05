"""Plain FP64 CPU oracle of the three-dimensional extension (D3Q19 pseudopotential flow, the
paper's D3Q7 temperature model): TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``.  The
compute lives in ``lbm3d_oracle.c``; this module only marshals arguments.

Parity status (pins in ``tests/test_oracle_3d.py``): matrices (orthogonality, equilibrium
moments), mass and momentum conservation, the discrete energy identity, Gaussian diffusion in
three dimensions, uniform states, the two-dimensional limit of a one-axis profile, flat-interface
coexistence densities and the Laplace law of a spherical droplet.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm3d_oracle.c")
_LIB = os.path.join(_HERE, "liboracle3d.so")

FREEZE_FLOW = 1
NO_S = 2
FREEZE_THERMAL = 4


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Params3(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("a", ctypes.c_double), ("b", ctypes.c_double), ("R", ctypes.c_double), ("acentric", ctypes.c_double),
        ("G", ctypes.c_double),
        ("nu", ctypes.c_double), ("s_e", ctypes.c_double), ("s_eps", ctypes.c_double), ("sigma", ctypes.c_double),
        ("lambda_", ctypes.c_double), ("cv", ctypes.c_double), ("wdot", ctypes.c_double), ("vs3", ctypes.c_double),
        ("thermal_box", ctypes.c_int32), ("T_box", ctypes.c_double), ("flags", ctypes.c_uint32),
    ]


def _struct(prm) -> Params3:
    c = Params3()
    for name, _ in Params3._fields_:
        setattr(c, name, getattr(prm, name))
    return c


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(Params3)
        d, dp, vp = ctypes.c_double, ctypes.POINTER(ctypes.c_double), ctypes.c_void_p
        L.o3_eos_Tc.argtypes = [P]; L.o3_eos_Tc.restype = d
        L.o3_eos_p.argtypes = [P, d, d]; L.o3_eos_p.restype = d
        L.o3_feq.argtypes = [d, d, d, d, dp]; L.o3_feq.restype = None
        L.o3_new.argtypes = [P]; L.o3_new.restype = vp
        L.o3_free.argtypes = [vp]; L.o3_free.restype = None
        L.o3_init.argtypes = [vp, dp, dp, dp, dp, dp]; L.o3_init.restype = None
        L.o3_step.argtypes = [vp, ctypes.c_long]; L.o3_step.restype = ctypes.c_int
        L.o3_fields.argtypes = [vp, dp, dp, dp, dp, dp]; L.o3_fields.restype = ctypes.c_int
        L.o3_get_state.argtypes = [vp, dp, dp, dp]; L.o3_get_state.restype = None
        L.o3_diagnostics.argtypes = [vp, dp, dp, dp, dp]; L.o3_diagnostics.restype = None
        L.o3_matrices.argtypes = [vp, dp, dp]; L.o3_matrices.restype = None
        L.o3_steps.argtypes = [vp]; L.o3_steps.restype = ctypes.c_long
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def eos_p(prm, rho, T):
    return lib().o3_eos_p(ctypes.byref(_struct(prm)), float(rho), float(T))


def Tc(prm):
    return lib().o3_eos_Tc(ctypes.byref(_struct(prm)))


def feq(rho, ux, uy, uz):
    out = np.zeros(19)
    lib().o3_feq(rho, ux, uy, uz, _dp(out))
    return out


class Oracle3D:
    """One three-dimensional simulation on the CPU; fields are arrays of shape (nz, ny, nx)."""

    def __init__(self, prm):
        self.prm = prm
        self._c = _struct(prm)
        self.shape = (int(prm.nz), int(prm.ny), int(prm.nx))
        self._h = lib().o3_new(ctypes.byref(self._c))
        if not self._h:
            raise RuntimeError("invalid parameters")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().o3_free(h)
            self._h = None

    def init(self, rho, ux, uy, uz, T):
        arrs = [np.ascontiguousarray(a, dtype=np.float64).reshape(self.shape) for a in (rho, ux, uy, uz, T)]
        lib().o3_init(self._h, *(_dp(a) for a in arrs))
        return self

    def step(self, n=1):
        rc = lib().o3_step(self._h, int(n))
        if rc:
            raise RuntimeError(f"numerical failure (code {rc})")
        return self

    def fields(self):
        out = [np.zeros(self.shape) for _ in range(5)]
        rc = lib().o3_fields(self._h, *(_dp(a) for a in out))
        if rc:
            raise RuntimeError(f"numerical failure (code {rc})")
        return tuple(out)  # rho, ux, uy, uz, T

    def state(self):
        f = np.zeros((19,) + self.shape)
        g = np.zeros((7,) + self.shape)
        h = np.zeros((2,) + self.shape)
        lib().o3_get_state(self._h, _dp(f), _dp(g), _dp(h))
        return f, g, h

    def diagnostics(self):
        v = [ctypes.c_double() for _ in range(4)]
        lib().o3_diagnostics(self._h, *(ctypes.byref(x) for x in v))
        return tuple(x.value for x in v)

    def matrices(self):
        M, M7 = np.zeros((19, 19)), np.zeros((7, 7))
        lib().o3_matrices(self._h, _dp(M), _dp(M7))
        return M, M7
