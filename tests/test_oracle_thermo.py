"""Pins of the oracle's thermodynamics (Peng-Robinson EOS, Eq. 10; Maxwell coexistence).

The EOS is pinned by properties a typo cannot survive: the textbook Peng-Robinson critical
point (T_c, rho_c b, Z_c), the ideal-gas limit, and a finite-difference derivative.  The
Maxwell solver is re-checked by an independent 40-digit mpmath equal-area construction.
"""
import math

import mpmath
import numpy as np
import pytest



def _dpdrho(orc, p, r, T, h=1e-6):
    return (orc.eos_p(p, r + h, T) - orc.eos_p(p, r - h, T)) / (2 * h)


def test_critical_temperature_from_a_b(orc, base_params):
    # Text after Eq. (10): a = 0.45724 R^2 Tc^2/pc, b = 0.0778 R Tc/pc with a = 3/49, b = 2/21, R = 1.
    Tc = orc.Tc(base_params)
    assert Tc == pytest.approx(0.0778 * (3 / 49) / (0.45724 * (2 / 21)), rel=1e-15)
    assert Tc == pytest.approx(0.109383006111, rel=1e-11)


def test_critical_point_is_inflection_of_isotherm(orc, base_params):
    """Textbook PR critical point: dp/drho = d2p/drho2 = 0 at rho_c b = 0.25307, Z_c = 0.3074.
    The rounded constants 0.45724 / 0.0778 put the true critical temperature 2e-5 below the
    formula value, so the isotherm just above has no unstable branch and the one just below has."""
    p = base_params
    Tc = orc.Tc(p)
    rs = np.linspace(0.5, 6.0, 5501)
    d_above = np.array([_dpdrho(orc, p, r, Tc * 1.0001) for r in rs])
    d_below = np.array([_dpdrho(orc, p, r, Tc * 0.9999) for r in rs])
    assert d_above.min() > 0
    assert d_below.min() < 0
    d_at = np.array([_dpdrho(orc, p, r, Tc) for r in rs])
    k = int(np.argmin(d_at))
    rho_c = rs[k]
    assert abs(d_at[k]) < 1e-4 * (Tc * p.R)  # flat isotherm at the critical point
    assert rho_c * p.b == pytest.approx(0.25307, abs=2e-3)
    pc = orc.eos_p(p, rho_c, Tc)
    assert pc == pytest.approx(0.45724 * p.R ** 2 * Tc ** 2 / p.a, rel=1e-3)  # inverts the a(Tc, pc) relation
    assert pc / (rho_c * p.R * Tc) == pytest.approx(0.3074, abs=2e-3)        # Z_c of Peng-Robinson


def test_ideal_gas_limit(orc, base_params):
    Tc = orc.Tc(base_params)
    for T in (0.7 * Tc, Tc, 1.2 * Tc):
        r = 1e-7
        assert orc.eos_p(base_params, r, T) / r == pytest.approx(base_params.R * T, rel=1e-5)


def test_dpdT_is_temperature_derivative(orc, base_params):
    Tc = orc.Tc(base_params)
    for r in (0.2, 0.38, 2.6, 5.0, 6.5, 7.2):
        for T in (0.8 * Tc, 0.86 * Tc, 0.946 * Tc, 1.06 * Tc):
            h = 1e-6 * T
            fd = (orc.eos_p(base_params, r, T + h) - orc.eos_p(base_params, r, T - h)) / (2 * h)
            assert orc.eos_dpdT(base_params, r, T) == pytest.approx(fd, rel=1e-7, abs=1e-9)


def test_psi_vanishes_where_pressure_equals_ideal_part(orc, base_params):
    """psi^2 = 2 (p - rho c_s^2) / G is zero at the density where p_EOS = rho/3 and undefined above."""
    T = 0.86 * orc.Tc(base_params)
    f = lambda r: orc.eos_p(base_params, r, T) - r / 3.0
    lo, hi = 7.0, 10.0
    for _ in range(100):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if f(mid) < 0 else (lo, mid)
    assert orc.psi(base_params, lo * (1 - 1e-9), T) >= 0
    assert orc.psi(base_params, lo * (1 - 1e-9), T) < 1e-3
    assert orc.psi(base_params, hi * (1 + 1e-6), T) == -1.0
    assert lo == pytest.approx(8.974, abs=2e-3)


def _pr_mp(r, T, a, b, R, w, Tc):
    k = mpmath.mpf("0.37464") + mpmath.mpf("1.54226") * w - mpmath.mpf("0.26992") * w * w
    phi = (1 + k * (1 - mpmath.sqrt(T / Tc))) ** 2
    return r * R * T / (1 - b * r) - a * phi * r * r / (1 + 2 * b * r - b * b * r * r)


@pytest.mark.parametrize("T_rel", [0.80, 0.86, 0.90, 0.946])
def test_maxwell_equal_area_independent(orc, base_params, T_rel):
    """The oracle's Maxwell densities satisfy equal pressure and equal area to high accuracy when
    checked with a 40-digit mpmath construction (independent quadrature and root finding)."""
    mpmath.mp.dps = 40
    a, b, R, w = mpmath.mpf(3) / 49, mpmath.mpf(2) / 21, mpmath.mpf(1), mpmath.mpf("0.344")
    Tc = mpmath.mpf("0.0778") * a / (mpmath.mpf("0.45724") * b * R)
    T = mpmath.mpf(T_rel) * Tc
    rl, rg, ps = orc.maxwell(base_params, float(T))
    # independent solve: unknowns (rho_g, rho_l) of p(rg) = p(rl) and the equal-area integral
    p = lambda r: _pr_mp(r, T, a, b, R, w, Tc)
    area = lambda g_, l_: mpmath.quad(lambda r: (p(r) - p(g_)) / r ** 2, [g_, l_])
    sol = mpmath.findroot(lambda g_, l_: [p(g_) - p(l_), area(g_, l_)], (mpmath.mpf(rg), mpmath.mpf(rl)))
    g_mp, l_mp = float(sol[0]), float(sol[1])
    assert rl == pytest.approx(l_mp, rel=1e-9)
    assert rg == pytest.approx(g_mp, rel=1e-8)
    assert ps == pytest.approx(float(p(sol[0])), rel=1e-8)


def test_maxwell_absent_above_critical(orc, base_params):
    with pytest.raises(ValueError):
        orc.maxwell(base_params, 1.01 * orc.Tc(base_params))
