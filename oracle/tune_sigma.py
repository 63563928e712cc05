"""Tune sigma of Li et al.'s forcing (Eq. 8) against the Maxwell coexistence densities.

The paper leaves sigma unstated.  Its Eq. (8) writes the correction as
sigma |F_m|^2 / (psi^2 dt (1/s_e - 1/2)), i.e. without the factor 12 of Li et al.'s own
formulation, so the value here is about twelve times the one usually quoted for that model.

Procedure (oracle only, FP64): a flat liquid slab in a periodic 4 x 256 box at T = 0.86 Tc,
temperature frozen, run to equilibrium; the bulk vapour density (mean over the vapour core,
averaged over the last steps) is driven to the Maxwell value by bisection on sigma.

Usage:  python oracle/tune_sigma.py      (prints sigma and the resulting densities)
"""
from __future__ import annotations

import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import oracle  # noqa: E402
from workloads import Params  # noqa: E402


def flat_interface(sigma: float, T_rel: float = 0.86, ny: int = 256, steps: int = 30000, avg: int = 5000):
    p = Params(nx=4, ny=ny, sigma=sigma, flags=oracle.FREEZE_THERMAL)
    Tc = oracle.Tc(p)
    T = T_rel * Tc
    rl, rg, _ = oracle.maxwell(p, T)
    y = np.arange(ny, dtype=np.float64)[:, None] * np.ones((1, 4))
    half = ny / 4.0
    rho = 0.5 * (rl + rg) - 0.5 * (rl - rg) * np.tanh((np.abs(y - (ny - 1) / 2.0) - half) / 2.5)
    o = oracle.Oracle(p).init(rho, 0 * rho, 0 * rho, np.full_like(rho, T))
    o.step(steps - avg)
    liq, vap = [], []
    c = ny // 2
    for _ in range(avg // 100):
        o.step(100)
        r = o.fields()[0][:, 0]
        liq.append(r[c - ny // 16: c + ny // 16].mean())
        vap.append(np.concatenate([r[: ny // 16], r[-ny // 16:]]).mean())
    return float(np.mean(liq)), float(np.mean(vap)), rl, rg


def tune(lo: float = 1.0, hi: float = 1.5, iters: int = 8):
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        _, rg_sim, _, rg = flat_interface(mid)
        if rg_sim < rg:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


if __name__ == "__main__":
    oracle.build(force=False)
    s = tune()
    rl_sim, rg_sim, rl, rg = flat_interface(s)
    print(f"sigma = {s:.4f}: rho_l = {rl_sim:.6f} (Maxwell {rl:.6f}, {rl_sim / rl - 1:+.2e}), "
          f"rho_g = {rg_sim:.6f} (Maxwell {rg:.6f}, {rg_sim / rg - 1:+.2e})")
