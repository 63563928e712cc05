"""Seeded synthetic workloads shared by the GPU library's callers and the oracle's tests.

This module holds only problem parameters and initial-field recipes (the initial density
profile of Eq. 56, uniform temperatures, seeded noise).  It holds none of the method's
arithmetic: thermodynamic quantities (critical temperature, coexistence densities) are
computed by the caller -- the oracle in tests, the GPU library in the benchmark -- and passed
in.  Random numbers come from numpy's PCG64 with an explicit seed.

Workloads (sizes and values follow the paper's test problems, Section 4):
  droplet      static droplet, periodic box (Laplace-law family)
  evaporation  droplet in saturated vapour, Dirichlet temperature on the box edges (D^2 law)
  boiling      liquid pool on a heated wall with a Gaussian hot spot, gravity (nucleate boiling)
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field

import numpy as np

FREEZE_FLOW = 1
NO_S = 2
FREEZE_THERMAL = 4
BGK = 8


@dataclass
class Params:
    """Physical and numerical parameters of one simulation (lattice units, dx = dt = 1)."""
    nx: int = 64
    ny: int = 64
    # Peng-Robinson EOS, Eq. (10): a = 3/49, b = 2/21, R = 1, acentric factor 0.344; G = -1 (Eq. 9)
    a: float = 3.0 / 49.0
    b: float = 2.0 / 21.0
    R: float = 1.0
    acentric: float = 0.344
    G: float = -1.0
    # D2Q9 MRT: kinematic viscosity nu (s_p = 1/(3 nu + 1/2)); other rates 1 (Section 4)
    nu: float = 0.1
    s_e: float = 1.0
    s_eps: float = 1.0
    s_q: float = 1.0
    # sigma of Li et al.'s forcing (Eq. 8) is not given in the paper; 1.25 puts the flat-interface
    # coexistence densities at T = 0.86 Tc on the Maxwell values (oracle/tune_sigma.py: 1.2529)
    sigma: float = 1.25
    # D2Q5 thermal model: conductivity, heat capacity, weight parameter wdot in (0, 1)
    lambda_: float = 1.0 / 3.0
    cv: float = 5.0
    wdot: float = 2.0 / 3.0
    vs3: float = 1.0
    vs4: float = 1.0
    # buoyancy F_b = (rho - rho_ave) g ; rho_ave = NaN -> mean of the initial density
    gx: float = 0.0
    gy: float = 0.0
    rho_ave: float = float("nan")
    # boundaries
    y_walls: int = 0
    thermal_box: int = 0
    T_box: float = 0.0
    T_top: float = 0.0
    T_bot: float = 0.0
    hot_dT: float = 0.0
    hot_x0: float = 0.0
    hot_sigma: float = 0.0
    theta_bot_deg: float = 90.0
    theta_top_deg: float = 90.0
    flags: int = 0
    # thermal lattice: 5 (D2Q5, the paper's model) or 9 (D2Q9 with the BGK collision of Eq. 21)
    thermal_q: int = 5
    # with y_walls: the top is an open (outflow) boundary instead of a wall
    open_top: int = 0

    def replace(self, **kw) -> "Params":
        return dataclasses.replace(self, **kw)



# ------------------------------------------------------------------------------ field recipes
def tanh_disk(nx, ny, x0, y0, R0, rho_l, rho_g, width=5.0) -> np.ndarray:
    """Eq. (56): rho = (rho_l+rho_g)/2 - (rho_l-rho_g)/2 tanh((|x - x0| - R0)/(0.5 w))."""
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    r = np.sqrt((x - x0) ** 2 + (y - y0) ** 2)
    return 0.5 * (rho_l + rho_g) - 0.5 * (rho_l - rho_g) * np.tanh((r - R0) / (0.5 * width))


def tanh_slab(nx, ny, y_interface, rho_l, rho_g, width=5.0) -> np.ndarray:
    """Liquid below y_interface, vapour above, with the interface profile of Eq. (56)."""
    y = np.arange(ny, dtype=np.float64)[:, None] * np.ones((1, nx))
    return 0.5 * (rho_l + rho_g) - 0.5 * (rho_l - rho_g) * np.tanh((y - y_interface) / (0.5 * width))


def uniform_noise(shape, amplitude, seed) -> np.ndarray:
    """Additive U[-amplitude, amplitude] noise from PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-amplitude, amplitude, size=shape)


@dataclass
class Workload:
    name: str
    params: Params
    rho: np.ndarray
    ux: np.ndarray
    uy: np.ndarray
    T: np.ndarray
    steps: int
    meta: dict = field(default_factory=dict)

    @property
    def nodes(self) -> int:
        return self.params.nx * self.params.ny


def _zeros(ny, nx):
    return np.zeros((ny, nx), dtype=np.float64)


def droplet(Tc, rho_l, rho_g, nx=64, ny=64, R=16.0, T_rel=0.86, steps=2000, **kw) -> Workload:
    """Static droplet in a periodic box at uniform saturation temperature."""
    T_sat = T_rel * Tc
    p = Params(nx=nx, ny=ny, **kw)
    rho = tanh_disk(nx, ny, nx / 2.0, ny / 2.0, R, rho_l, rho_g)
    return Workload("droplet", p, rho, _zeros(ny, nx), _zeros(ny, nx), np.full((ny, nx), T_sat), steps,
                    {"R": R, "T_sat": T_sat})


def evaporation(Tc, rho_l, rho_g, nx=512, ny=512, R=64.0, T_rel=0.86, superheat=1.10, steps=20000,
                hot_vapour=False, **kw) -> Workload:
    """Droplet in saturated vapour; box edges held at T_box = superheat * T_sat; flow periodic.
    Initial temperature is T_sat everywhere, or (hot_vapour=True, the set-up of the paper's
    D^2-law test) T_sat in the liquid and T_box in the vapour, split at rho = (rho_l+rho_g)/2."""
    T_sat = T_rel * Tc
    T_box = superheat * T_sat
    p = Params(nx=nx, ny=ny, thermal_box=1, T_box=T_box, **kw)
    rho = tanh_disk(nx, ny, nx / 2.0, ny / 2.0, R, rho_l, rho_g)
    T = np.full((ny, nx), T_sat)
    if hot_vapour:
        T = np.where(rho > 0.5 * (rho_l + rho_g), T_sat, T_box)
    return Workload("evaporation", p, rho, _zeros(ny, nx), _zeros(ny, nx), T, steps,
                    {"R": R, "T_sat": T_sat})


def heated_droplet(Tc, rho_l, rho_g, nx=200, ny=100, R=35.0, T_rel=0.86, T_h_rel=0.95, T_s_rel=None,
                   lambda_=0.08, theta=90.0, steps=20000, **kw) -> Workload:
    """Droplet on a heated wall under an open top (Section 4.2): a half disk of radius R centred on
    the bottom wall at x = nx/2 (Eq. 56, width 5), contact angle theta, wall at T_h, open top
    held at T_s (T_sat unless given), periodic in x, initial T = T_sat everywhere.  The paper
    gives neither T_h nor T_s: T_h = 0.95 Tc (about 10 % above T_sat) and T_s = T_sat are proposed
    here.  Its 'thermal diffusivity 0.08' is taken as the conductivity lambda.  The paper first
    runs the droplet without evaporation until its contact angle settles: T_h_rel = T_rel gives
    that unheated stage."""
    T_sat = T_rel * Tc
    T_s = (T_s_rel * Tc) if T_s_rel is not None else T_sat
    p = Params(nx=nx, ny=ny, y_walls=1, open_top=1, T_bot=T_h_rel * Tc, T_top=T_s, theta_bot_deg=theta,
               theta_top_deg=90.0, lambda_=lambda_, **kw)
    rho = tanh_disk(nx, ny, nx / 2.0, 0.0, R, rho_l, rho_g)
    return Workload("heated_droplet", p, rho, _zeros(ny, nx), _zeros(ny, nx), np.full((ny, nx), T_sat), steps,
                    {"R": R, "T_sat": T_sat, "T_h": T_h_rel * Tc, "T_s": T_s})


def boiling(Tc, rho_l, rho_g, nx=1024, ny=2048, T_rel=0.86, dT_rel=0.2, gravity=2e-5, hot_width=32.0,
            fill=0.5, noise=1e-3, seed=1, theta_bot=75.0, theta_top=90.0, steps=50000, lambda_=2.0 / 3.0,
            **kw) -> Workload:
    """Liquid pool on a bottom wall with a Gaussian hot spot, gravity along -y, walls at y."""
    T_sat = T_rel * Tc
    p = Params(nx=nx, ny=ny, y_walls=1, gy=-gravity, T_bot=T_sat, T_top=T_sat, hot_dT=dT_rel * Tc,
               hot_x0=nx / 2.0, hot_sigma=hot_width, theta_bot_deg=theta_bot, theta_top_deg=theta_top,
               lambda_=lambda_, **kw)
    rho = tanh_slab(nx, ny, fill * ny, rho_l, rho_g) + uniform_noise((ny, nx), noise, seed)
    return Workload("boiling", p, rho, _zeros(ny, nx), _zeros(ny, nx), np.full((ny, nx), T_sat), steps,
                    {"T_sat": T_sat, "seed": seed, "fill": fill})


def head_limited_fill(rho_l, rho_g, p_sat, gravity, ny, fill=0.5, head_frac=0.5) -> float:
    """Liquid fill fraction of a boiling pool whose vapour head stays within head_frac * p_sat.

    With buoyancy (rho - rho_ave) g in a box closed at the top, the hydrostatic pressure rise
    across the vapour column is fill (1 - fill) (rho_l - rho_g) g ny (rho_ave = fill rho_l +
    (1 - fill) rho_g).  When it approaches the gap between p_sat and the vapour spinodal, the top
    vapour cannot stay vapour and the column collapses (density reaches zero within ~1500 steps).
    Returns `fill` if its head is within the limit, otherwise the larger fill (a fuller pool with
    a shallower vapour headspace) whose head equals the limit."""
    span = (rho_l - rho_g) * abs(gravity) * ny
    cap = head_frac * p_sat
    if span <= 0.0 or fill * (1.0 - fill) * span <= cap:
        return fill
    q = cap / span  # fill (1 - fill) = q, q < 1/4 here
    return 0.5 + math.sqrt(max(0.0, 0.25 - q))


# ------------------------------------------------------------------------- batched / served mixes
GRID_CLASSES = ((256, 512), (384, 768), (512, 1024))


def gravity_sweep(n=64, seed=2, steps=10000):
    """Per-instance (nx, ny, g, dT_rel) of the batched gravity sweep: grids uniform over three
    classes, g log-uniform in [5e-6, 5e-5], hot-spot dT uniform in [0.1, 0.3] Tc."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for k in range(n):
        nx, ny = GRID_CLASSES[int(rng.integers(0, len(GRID_CLASSES)))]
        g = float(math.exp(rng.uniform(math.log(5e-6), math.log(5e-5))))
        dT = float(rng.uniform(0.1, 0.3))
        out.append({"nx": nx, "ny": ny, "gravity": g, "dT_rel": dT, "steps": steps, "seed": 1000 + k})
    return out


def request_stream(n=256, rate=20.0, seed=3, nx_range=(128, 1024), ny_range=(128, 2048),
                   steps_range=(1000, 20000)):
    """Poisson arrivals of mixed solve requests: kind uniform over {droplet, evaporation, boiling},
    nx and ny log-uniform (independent), step counts uniform."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    kinds = ("droplet", "evaporation", "boiling")
    for k in range(n):
        t += float(rng.exponential(1.0 / rate))
        kind = kinds[int(rng.integers(0, 3))]
        nx = int(round(math.exp(rng.uniform(math.log(nx_range[0]), math.log(nx_range[1])))))
        ny = int(round(math.exp(rng.uniform(math.log(ny_range[0]), math.log(ny_range[1])))))
        steps = int(rng.integers(steps_range[0], steps_range[1] + 1))
        out.append({"id": k, "arrival": t, "kind": kind, "nx": nx, "ny": ny, "steps": steps, "seed": 5000 + k})
    return out


# ----------------------------------------------------------------------------- three dimensions
@dataclass
class Params3D:
    """Parameters of a three-dimensional simulation (D3Q19 flow, D3Q7 temperature; lattice units).
    Defaults follow the two-dimensional ones; the D3Q7 weight parameter wdot gives chat_s^2 = wdot/3."""
    nx: int = 32
    ny: int = 32
    nz: int = 32
    a: float = 3.0 / 49.0
    b: float = 2.0 / 21.0
    R: float = 1.0
    acentric: float = 0.344
    G: float = -1.0
    nu: float = 0.1
    s_e: float = 1.0
    s_eps: float = 1.0
    sigma: float = 1.25
    lambda_: float = 1.0 / 3.0
    cv: float = 5.0
    wdot: float = 2.0 / 3.0
    vs3: float = 1.0
    thermal_box: int = 0
    T_box: float = 0.0
    flags: int = 0
    z_chunk: int = 0  # GPU fused path: z planes per workgroup (0: automatic)
    path: int = 0     # GPU step path: 0 fused, 1 per-node kernels

    def replace(self, **kw) -> "Params3D":
        return dataclasses.replace(self, **kw)


@dataclass
class Workload3D:
    name: str
    params: Params3D
    rho: np.ndarray
    ux: np.ndarray
    uy: np.ndarray
    uz: np.ndarray
    T: np.ndarray
    steps: int
    meta: dict = field(default_factory=dict)

    @property
    def nodes(self) -> int:
        return int(self.params.nx) * int(self.params.ny) * int(self.params.nz)


def tanh_sphere(nx, ny, nz, R0, rho_l, rho_g, width=5.0) -> np.ndarray:
    """Eq. (56) in three dimensions, centred in the box: arrays of shape (nz, ny, nx)."""
    z, y, x = np.mgrid[0:nz, 0:ny, 0:nx].astype(np.float64)
    r = np.sqrt((x - nx / 2.0) ** 2 + (y - ny / 2.0) ** 2 + (z - nz / 2.0) ** 2)
    return 0.5 * (rho_l + rho_g) - 0.5 * (rho_l - rho_g) * np.tanh((r - R0) / (0.5 * width))


def droplet3d(Tc, rho_l, rho_g, n=48, R=12.0, T_rel=0.86, steps=2000, **kw) -> Workload3D:
    """Static droplet in a periodic cube at uniform saturation temperature."""
    p = Params3D(nx=n, ny=n, nz=n, **kw)
    rho = tanh_sphere(n, n, n, R, rho_l, rho_g)
    z = np.zeros_like(rho)
    return Workload3D("droplet3d", p, rho, z, z.copy(), z.copy(), np.full_like(rho, T_rel * Tc), steps, {"R": R})


def evaporation3d(Tc, rho_l, rho_g, n=128, R=16.0, T_rel=0.86, superheat=1.10, steps=20000, **kw) -> Workload3D:
    """Droplet in saturated vapour in a cube whose faces are held at superheat * T_sat; flow periodic."""
    T_sat = T_rel * Tc
    p = Params3D(nx=n, ny=n, nz=n, thermal_box=1, T_box=superheat * T_sat, **kw)
    rho = tanh_sphere(n, n, n, R, rho_l, rho_g)
    z = np.zeros_like(rho)
    return Workload3D("evaporation3d", p, rho, z, z.copy(), z.copy(), np.full_like(rho, T_sat), steps,
                      {"R": R, "T_sat": T_sat})
