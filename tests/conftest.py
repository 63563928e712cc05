"""Shared test set-up: markers, import path, and the FP64 CPU oracle (test infrastructure)."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI library)")
    config.addinivalue_line("markers", "slow: long CPU run of the oracle (tens of seconds)")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.build(force=False)
    return oracle


@pytest.fixture(scope="session")
def base_params():
    from workloads import Params
    return Params()


@pytest.fixture(scope="session")
def sat(orc, base_params):
    """(Tc, T_sat, rho_l, rho_g, p_sat) at T_sat = 0.86 Tc from the oracle's EOS."""
    Tc = orc.Tc(base_params)
    T = 0.86 * Tc
    rl, rg, ps = orc.maxwell(base_params, T)
    return Tc, T, rl, rg, ps
