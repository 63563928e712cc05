"""Tune sigma of Li et al.'s forcing for the three-dimensional extension (D3Q19, the reading of
the sigma term in ``lbm3d_oracle.c``) against the Maxwell coexistence densities, as
``tune_sigma.py`` does for D2Q9: a flat liquid slab across a periodic 4 x 4 x 256 box at
T = 0.86 Tc, temperature frozen, run to equilibrium, bulk vapour density averaged over the last
steps, bisection on sigma.

Usage:  python oracle/tune_sigma3d.py
"""
from __future__ import annotations

import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import oracle  # noqa: E402
from oracle import o3d  # noqa: E402
from workloads import Params, Params3D  # noqa: E402


def flat_interface(sigma: float, T_rel: float = 0.86, nz: int = 256, steps: int = 30000, avg: int = 5000):
    p = Params3D(nx=4, ny=4, nz=nz, sigma=sigma, flags=o3d.FREEZE_THERMAL)
    p2 = Params()
    T = T_rel * oracle.Tc(p2)
    rl, rg, _ = oracle.maxwell(p2, T)
    z = np.arange(nz, dtype=np.float64)[:, None, None] * np.ones((1, 4, 4))
    rho = 0.5 * (rl + rg) - 0.5 * (rl - rg) * np.tanh((np.abs(z - (nz - 1) / 2.0) - nz / 4.0) / 2.5)
    zero = 0 * rho
    o = o3d.Oracle3D(p).init(rho, zero, zero, zero, np.full_like(rho, T))
    o.step(steps - avg)
    liq, vap = [], []
    c = nz // 2
    for _ in range(avg // 100):
        o.step(100)
        r = o.fields()[0][:, 0, 0]
        liq.append(r[c - nz // 16: c + nz // 16].mean())
        vap.append(np.concatenate([r[: nz // 16], r[-nz // 16:]]).mean())
    return float(np.mean(liq)), float(np.mean(vap)), rl, rg


def tune(lo: float = 0.8, hi: float = 1.6, iters: int = 7):
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
    if len(sys.argv) > 1:
        for s in map(float, sys.argv[1:]):
            rl_sim, rg_sim, rl, rg = flat_interface(s)
            print(f"sigma = {s}: rho_l {rl_sim / rl - 1:+.2e}, rho_g {rg_sim / rg - 1:+.2e}", flush=True)
        sys.exit(0)
    s = tune()
    rl_sim, rg_sim, rl, rg = flat_interface(s)
    print(f"sigma = {s:.4f}: rho_l = {rl_sim:.6f} (Maxwell {rl:.6f}, {rl_sim / rl - 1:+.2e}), "
          f"rho_g = {rg_sim:.6f} (Maxwell {rg:.6f}, {rg_sim / rg - 1:+.2e})")
