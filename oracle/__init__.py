"""Plain FP64 CPU oracle of the thermal pseudopotential LBM (Wang, Huang & He, arXiv:2205.00686).

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code with the
GPU library in ``paper_2205_00686_amd``; the compute lives in ``lbm_oracle.c`` (plain C,
explicit matrices, FP64) and this module only marshals arguments through ctypes.

Parity status of each function (see the pins in ``tests/test_oracle_*.py``):
  * eos_p, eos_dpdT, Tc       -- pinned: critical-point conditions, ideal-gas limit,
                                 finite-difference derivative.
  * maxwell                   -- pinned: equal-area and equal-pressure conditions re-checked
                                 with scipy quadrature; flat-interface simulation.
  * feq, meq, force_moments   -- pinned: M f_eq = m_eq, Guo-forcing identity at sigma = 0.
  * Oracle.step               -- pinned by invariants and closed forms (mass, momentum,
                                 discrete energy identity, Gaussian pulse diffusion and
                                 advection, compression source, steady conduction,
                                 Poiseuille flow, Laplace law, D^2 law).
  * sigma (Eq. 8)             -- parity unpinned: not given in the paper; tuned against the
                                 Maxwell densities by ``oracle/tune_sigma.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

FREEZE_FLOW = 1
NO_S = 2
FREEZE_THERMAL = 4
BGK = 8  # D2Q5 with the BGK collision of Eq. (21) instead of the MRT one of Eq. (39)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, OpenMP over grid rows)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    from . import o3d  # the three-dimensional oracle is built alongside
    o3d.build(force)
    return _LIB


class _CParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("a", ctypes.c_double), ("b", ctypes.c_double), ("R", ctypes.c_double),
        ("acentric", ctypes.c_double), ("G", ctypes.c_double),
        ("nu", ctypes.c_double), ("s_e", ctypes.c_double), ("s_eps", ctypes.c_double),
        ("s_q", ctypes.c_double), ("sigma", ctypes.c_double),
        ("lambda_", ctypes.c_double), ("cv", ctypes.c_double), ("wdot", ctypes.c_double),
        ("vs3", ctypes.c_double), ("vs4", ctypes.c_double),
        ("gx", ctypes.c_double), ("gy", ctypes.c_double), ("rho_ave", ctypes.c_double),
        ("y_walls", ctypes.c_int32), ("thermal_box", ctypes.c_int32),
        ("T_box", ctypes.c_double), ("T_top", ctypes.c_double), ("T_bot", ctypes.c_double),
        ("hot_dT", ctypes.c_double), ("hot_x0", ctypes.c_double), ("hot_sigma", ctypes.c_double),
        ("theta_bot_deg", ctypes.c_double), ("theta_top_deg", ctypes.c_double),
        ("flags", ctypes.c_uint32), ("thermal_q", ctypes.c_int32), ("open_top", ctypes.c_int32),
    ]


def _params_struct(prm) -> _CParams:
    """Accepts any object with the physical parameter names (e.g. workloads.Params)."""
    c = _CParams()
    for name, _ in _CParams._fields_:
        src = "lambda_" if name == "lambda_" else name
        setattr(c, name, getattr(prm, src))
    return c


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(_CParams)
        d = ctypes.c_double
        dp = ctypes.POINTER(ctypes.c_double)
        vp = ctypes.c_void_p
        L.orc_eos_Tc.argtypes = [P]; L.orc_eos_Tc.restype = d
        L.orc_eos_p.argtypes = [P, d, d]; L.orc_eos_p.restype = d
        L.orc_eos_dpdT.argtypes = [P, d, d]; L.orc_eos_dpdT.restype = d
        L.orc_psi.argtypes = [P, d, d]; L.orc_psi.restype = d
        L.orc_maxwell.argtypes = [P, d, dp, dp, dp]; L.orc_maxwell.restype = ctypes.c_int
        L.orc_feq.argtypes = [d, d, d, dp]; L.orc_feq.restype = None
        L.orc_meq.argtypes = [d, d, d, dp]; L.orc_meq.restype = None
        L.orc_force_moments.argtypes = [d] * 10 + [dp]; L.orc_force_moments.restype = None
        L.orc_new.argtypes = [P]; L.orc_new.restype = vp
        L.orc_free.argtypes = [vp]; L.orc_free.restype = None
        L.orc_init.argtypes = [vp, dp, dp, dp, dp]; L.orc_init.restype = None
        L.orc_step.argtypes = [vp, ctypes.c_long]; L.orc_step.restype = ctypes.c_int
        L.orc_fields.argtypes = [vp, dp, dp, dp, dp]; L.orc_fields.restype = ctypes.c_int
        L.orc_get_state.argtypes = [vp, dp, dp, dp]; L.orc_get_state.restype = None
        L.orc_set_state.argtypes = [vp, dp, dp, dp]; L.orc_set_state.restype = None
        L.orc_diagnostics.argtypes = [vp, dp, dp, dp, dp]; L.orc_diagnostics.restype = None
        L.orc_rho_ave.argtypes = [vp]; L.orc_rho_ave.restype = d
        L.orc_get_post.argtypes = [vp, dp]; L.orc_get_post.restype = None
        L.orc_steps.argtypes = [vp]; L.orc_steps.restype = ctypes.c_long
        L.orc_num_threads.argtypes = []; L.orc_num_threads.restype = ctypes.c_int
        L.orc_set_threads.argtypes = [ctypes.c_int]; L.orc_set_threads.restype = None
        L.orc_matrices.argtypes = [vp, dp, dp, dp, dp]; L.orc_matrices.restype = None
        L.orc_relaxation.argtypes = [vp, dp, dp]; L.orc_relaxation.restype = None
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# ----------------------------------------------------------------------------- thermodynamics
def Tc(prm) -> float:
    """Critical temperature implied by a and b of the Peng-Robinson EOS (text after Eq. 10)."""
    c = _params_struct(prm)
    return lib().orc_eos_Tc(ctypes.byref(c))


def eos_p(prm, rho: float, T: float) -> float:
    """Peng-Robinson pressure, Eq. (10)."""
    c = _params_struct(prm)
    return lib().orc_eos_p(ctypes.byref(c), float(rho), float(T))


def eos_dpdT(prm, rho: float, T: float) -> float:
    """(d p_EOS / d T) at constant density, as needed by Q of Eq. (20)."""
    c = _params_struct(prm)
    return lib().orc_eos_dpdT(ctypes.byref(c), float(rho), float(T))


def psi(prm, rho: float, T: float) -> float:
    """Pseudopotential (text after Eq. 9); -1 where it is undefined."""
    c = _params_struct(prm)
    return lib().orc_psi(ctypes.byref(c), float(rho), float(T))


def maxwell(prm, T: float):
    """(rho_l, rho_g, p_sat) of the Maxwell equal-area construction at temperature T."""
    c = _params_struct(prm)
    rl, rg, ps = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    rc = lib().orc_maxwell(ctypes.byref(c), float(T), ctypes.byref(rl), ctypes.byref(rg), ctypes.byref(ps))
    if rc != 0:
        raise ValueError(f"no liquid-vapour coexistence at T={T}")
    return rl.value, rg.value, ps.value


# -------------------------------------------------------------------------- moment-space pieces
def feq(rho, ux, uy) -> np.ndarray:
    out = np.zeros(9)
    lib().orc_feq(float(rho), float(ux), float(uy), _dp(out))
    return out


def meq(rho, ux, uy) -> np.ndarray:
    out = np.zeros(9)
    lib().orc_meq(float(rho), float(ux), float(uy), _dp(out))
    return out


def force_moments(ux, uy, Fnx, Fny, Fmx, Fmy, psi_, sigma, s_e, s_eps) -> np.ndarray:
    out = np.zeros(9)
    lib().orc_force_moments(*(float(v) for v in (ux, uy, Fnx, Fny, Fmx, Fmy, psi_, sigma, s_e, s_eps)),
                            _dp(out))
    return out


# ----------------------------------------------------------------------------------- simulation
class OracleError(RuntimeError):
    pass


class Oracle:
    """One simulation on the CPU.  Fields are numpy arrays of shape (ny, nx), x fastest."""

    def __init__(self, prm):
        self.prm = prm
        self._c = _params_struct(prm)
        self.nx, self.ny = int(prm.nx), int(prm.ny)
        self._h = lib().orc_new(ctypes.byref(self._c))
        if not self._h:
            raise OracleError("invalid parameters")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_free(h)
            self._h = None

    def init(self, rho, ux, uy, T):
        arrs = [_c64(a).reshape(self.ny, self.nx) for a in (rho, ux, uy, T)]
        lib().orc_init(self._h, *(_dp(a) for a in arrs))
        return self

    def step(self, n: int = 1):
        rc = lib().orc_step(self._h, int(n))
        if rc != 0:
            raise OracleError(f"numerical failure (code {rc}) at step {self.steps}")
        return self

    @property
    def steps(self) -> int:
        return lib().orc_steps(self._h)

    @property
    def rho_ave(self) -> float:
        return lib().orc_rho_ave(self._h)

    def fields(self):
        out = [np.zeros((self.ny, self.nx)) for _ in range(4)]
        rc = lib().orc_fields(self._h, *(_dp(a) for a in out))
        if rc != 0:
            raise OracleError(f"numerical failure (code {rc})")
        return tuple(out)  # rho, ux, uy, T

    @property
    def q(self) -> int:
        """Velocities of the thermal lattice (5 or 9)."""
        return 9 if int(getattr(self.prm, "thermal_q", 5)) == 9 else 5

    def state(self):
        f = np.zeros((9, self.ny, self.nx))
        g = np.zeros((self.q, self.ny, self.nx))
        h = np.zeros((2, self.ny, self.nx))
        lib().orc_get_state(self._h, _dp(f), _dp(g), _dp(h))
        return f, g, h

    def post_collision(self):
        """f* of the last step, [9][ny][nx]."""
        fs = np.zeros((9, self.ny, self.nx))
        lib().orc_get_post(self._h, _dp(fs))
        return fs

    def set_state(self, f, g, h):
        f, g, h = _c64(f), _c64(g), _c64(h)
        lib().orc_set_state(self._h, _dp(f), _dp(g), _dp(h))

    def diagnostics(self):
        """(mass, energy, sum Q of last step, sum S of last step)."""
        v = [ctypes.c_double() for _ in range(4)]
        lib().orc_diagnostics(self._h, *(ctypes.byref(x) for x in v))
        return tuple(x.value for x in v)

    def matrices(self):
        M, Minv = np.zeros((9, 9)), np.zeros((9, 9))
        Mh, Mhinv = np.zeros((5, 5)), np.zeros((5, 5))
        lib().orc_matrices(self._h, _dp(M), _dp(Minv), _dp(Mh), _dp(Mhinv))
        return M, Minv, Mh, Mhinv

    def relaxation(self):
        S, L = np.zeros(9), np.zeros(5)
        lib().orc_relaxation(self._h, _dp(S), _dp(L))
        return S, L


def num_threads() -> int:
    """Number of threads the oracle's grid loops use (OpenMP)."""
    return int(lib().orc_num_threads())


def set_threads(n: int) -> None:
    """Threads for the oracle's following grid loops (for timing it on one core)."""
    lib().orc_set_threads(int(n))


def run(prm, rho, ux, uy, T, steps: int):
    """Convenience: initialise, run ``steps`` steps, return (rho, ux, uy, T)."""
    o = Oracle(prm).init(rho, ux, uy, T)
    o.step(steps)
    return o.fields()


__all__ = ["build", "num_threads", "set_threads", "Tc", "eos_p", "eos_dpdT", "psi", "maxwell", "feq", "meq", "force_moments",
           "Oracle", "OracleError", "run", "FREEZE_FLOW", "NO_S", "BGK"]
