"""Pins of the oracle's moment-space pieces (Eqs. 3-8, 22, 26, 40, 47).

Each check is an identity that holds for the correct tables and fails for a plausible typo:
M f_eq = m_eq (catches the misprinted row 3 of Eq. 4 and any sign slip in Eq. 3 or 7), the
orthogonality of the Lallemand-Luo rows, Li's forcing at sigma = 0 equal to the moments of
Guo's forcing (catches a wrong factor or sign in Eq. 8), and the D2Q5 moment relations.
"""
import numpy as np
import pytest

CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


@pytest.fixture(scope="module")
def mats(orc, base_params):
    o = orc.Oracle(base_params.replace(nx=4, ny=4))
    return o.matrices()


def test_M_rows_are_orthogonal_and_inverse_exact(mats):
    M, Minv, Mh, Mhinv = mats
    G = M @ M.T
    assert np.allclose(G - np.diag(np.diag(G)), 0.0, atol=0)
    assert np.allclose(np.diag(G), [9, 36, 36, 6, 12, 6, 12, 4, 4])
    assert np.allclose(M @ Minv, np.eye(9), atol=1e-14)
    assert np.allclose(Mh @ Mhinv, np.eye(5), atol=1e-14)


def test_M_row1_to_row4_are_velocity_moments(mats):
    M = mats[0]
    assert np.array_equal(M[3], CX) and np.array_equal(M[5], CY)
    assert np.array_equal(M[7], CX ** 2 - CY ** 2) and np.array_equal(M[8], CX * CY)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_M_feq_equals_meq(orc, mats, seed):
    rng = np.random.default_rng(seed)
    M = mats[0]
    for _ in range(20):
        rho = rng.uniform(0.1, 7.0)
        ux, uy = rng.uniform(-0.2, 0.2, 2)
        assert np.allclose(M @ orc.feq(rho, ux, uy), orc.meq(rho, ux, uy), atol=1e-13)


def test_printed_row3_breaks_the_equilibrium_identity(orc, mats):
    """Documents the reading of Eq. (4): with the row as printed, M f_eq != m_eq."""
    M = mats[0].copy()
    M[2] = [4, -2, -2, -2, 1, 1, 1, 1, 1]
    err = np.abs(M @ orc.feq(1.0, 0.05, -0.03) - orc.meq(1.0, 0.05, -0.03)).max()
    assert err > 0.1


def test_feq_moments(orc):
    """Eq. (3): zeroth, first and second moments of f_eq are rho, rho u, rho(c_s^2 I + u u)."""
    rho, ux, uy = 2.3, 0.07, -0.04
    f = orc.feq(rho, ux, uy)
    assert f.sum() == pytest.approx(rho, rel=1e-15)
    assert (CX * f).sum() == pytest.approx(rho * ux, rel=1e-14)
    assert (CY * f).sum() == pytest.approx(rho * uy, rel=1e-14)
    assert (CX * CX * f).sum() == pytest.approx(rho * (1 / 3 + ux * ux), rel=1e-14)
    assert (CX * CY * f).sum() == pytest.approx(rho * ux * uy, rel=1e-13)


@pytest.mark.parametrize("seed", [3, 4])
def test_li_forcing_at_sigma0_is_guo_forcing(orc, mats, seed):
    """At sigma = 0, Eq. (8) is M applied to Guo's forcing w_i[(c_i-u)/c_s^2 + (c_i.u)c_i/c_s^4].F."""
    M = mats[0]
    rng = np.random.default_rng(seed)
    for _ in range(10):
        ux, uy, Fx, Fy = rng.uniform(-0.1, 0.1, 4)
        cu = CX * ux + CY * uy
        guo = W * (((CX - ux) * Fx + (CY - uy) * Fy) * 3.0 + cu * (CX * Fx + CY * Fy) * 9.0)
        F = orc.force_moments(ux, uy, Fx, Fy, 0.3, -0.2, 1.7, 0.0, 1.0, 1.0)
        assert np.allclose(F, M @ guo, atol=1e-14)


def test_li_sigma_term_enters_e_and_epsilon_rows_only(orc):
    base = orc.force_moments(0.01, 0.02, 0.003, -0.004, 0.002, 0.001, 1.5, 0.0, 1.0, 1.0)
    corr = orc.force_moments(0.01, 0.02, 0.003, -0.004, 0.002, 0.001, 1.5, 1.25, 1.0, 0.8)
    d = corr - base
    fm2 = 0.002 ** 2 + 0.001 ** 2
    assert d[1] == pytest.approx(1.25 * fm2 / (1.5 ** 2 * (1 / 1.0 - 0.5)), rel=1e-14)
    assert d[2] == pytest.approx(-1.25 * fm2 / (1.5 ** 2 * (1 / 0.8 - 0.5)), rel=1e-14)
    assert np.all(d[[0, 3, 4, 5, 6, 7, 8]] == 0)


def test_d2q5_weights_and_equilibrium_moments(orc, base_params, mats):
    """Eqs. (26), (33), (47): sum what_i = 1, sum what_i c_i c_i = chat_s^2 I, Mh g_eq = [T,0,0,wdot T,0]."""
    Mh = mats[2]
    p = base_params.replace(nx=3, ny=3)
    o = orc.Oracle(p).init(np.ones((3, 3)), np.zeros((3, 3)), np.zeros((3, 3)), np.full((3, 3), 0.7))
    g = o.state()[1][:, 0, 0]
    hx = np.array([0, 1, 0, -1, 0])
    hy = np.array([0, 0, 1, 0, -1])
    assert g.sum() == pytest.approx(0.7, rel=1e-15)
    assert (hx * hx * g).sum() == pytest.approx(0.7 * p.wdot / 2, rel=1e-15)
    assert (hx * hy * g).sum() == 0 and (hx * g).sum() == 0
    assert np.allclose(Mh @ g, [0.7, 0, 0, p.wdot * 0.7, 0], atol=1e-15)


def test_relaxation_rates_follow_nu_and_lambda(orc, base_params):
    """nu = c_s^2 (1/s_p - 1/2) and lambda = chat_s^2 (1/varsigma_1 - 1/2) (Eq. 53)."""
    for nu, lam in ((0.1, 1 / 3), (0.05, 2 / 3)):
        p = base_params.replace(nx=4, ny=4, nu=nu, lambda_=lam)
        S, L = orc.Oracle(p).relaxation()
        assert (1 / S[7] - 0.5) / 3 == pytest.approx(nu, rel=1e-14)
        assert S[7] == S[8]
        assert (1 / L[1] - 0.5) * p.wdot / 2 == pytest.approx(lam, rel=1e-14)
        assert L[1] == L[2]
