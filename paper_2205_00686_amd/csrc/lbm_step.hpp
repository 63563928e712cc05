// The fused time step: one workgroup per TX x TY tile of one simulation.
//
// One step (phases separated by workgroup barriers; the arithmetic of a node never depends on
// where its tile lies or on the tile shape, so a node's result is the same in a single run, in a
// batch and with any shape):
//   1  load f and g of the tile plus a halo (HXW columns, HYW rows); per node rho, j, T
//      (Eqs. 11, 25), 1/(rho c_v) and psi (Eq. 10 and the text after Eq. 9) into LDS; own nodes
//      keep f, g and (dp/dT)_rho in registers.  Wall tiles then fill the ghost rows with the
//      wetting density of Eq. (54) at the wall temperature.
//   2  on the tile plus one halo node: interaction force (Eq. 9), buoyancy, velocity (Eq. 11).
//   3  own nodes: div u (isotropic stencil, mirrored ghost velocity at walls), grad T from the
//      D2Q5 non-equilibrium moments (Eqs. 49-50), Q (Eq. 20), S (Eq. 24, backward second
//      difference of T), MRT collision of f with Li's forcing (Eqs. 5, 7, 8), MRT collision of
//      g (Eq. 39), push-streaming of f (Eq. 6, halfway bounce-back at walls) and of g with the
//      rho c_v-weighted blend at the destination (Eq. 39; anti-bounce-back at Dirichlet edges).
//
// Two steps per launch (shapes with DEPTH 2, FP32): the workgroup loads a wider halo (MXH
// columns, MYH rows), runs the first step on the tile plus the ring the second step reads, and
// streams its result into LDS instead of HBM; the second step is the one-step body reading that
// LDS state.  HBM traffic and the fixed cost of a launch are paid once per two steps.
//
// A workgroup has S::WAVES wavefronts of 64 lanes along x; each thread owns S::RPT rows of its
// column (rows ty, ty + WAVES, ...).
#pragma once
#include <type_traits>

#include "lbm_device.hpp"

namespace lbm {

// Per-node fields a step keeps in LDS, over a MY x MX region (QG: velocities of the thermal
// lattice, 5 or 9).
template <typename real, int MY, int MX, int QG = 5>
struct MacroLds {
  real rho[MY][MX];
  real irc[MY][MX];  // 1 / (rho c_v), needed at the streaming destination
  real psi[MY][MX];
  real ux[MY][MX];   // holds j_x after phase 1, u_x after phase 2
  real uy[MY][MX];
  real g[QG - 1][MY][MX];  // pre-collision g_1..g_{QG-1} (needed at the streaming destination)
};

template <typename real, int EYW, int QG = 5>
using StepLds = MacroLds<real, EYW, EXW, QG>;

// LDS of a two-step launch: the first step's fields over the wide region, aliased by the second
// step's fields once the first step has streamed; the state between the two steps (f and g
// after the first step) over the second step's load region.
template <typename real, class S>
struct Step2Lds {
  union {
    MacroLds<real, S::MY, S::MX> m1;
    StepLds<real, S::EYW> m2;
  };
  real sf[9][S::EYW][EXW];
  real sg[5][S::EYW][EXW];
};

// Cells of the rectangular annulus between "tile plus (ai, bi)" and "tile plus (ao, bo)"
// (columns, rows on each side of the TX x TY_ tile).
template <int TY_, int ai, int bi, int ao, int bo>
constexpr int annulus_cells() {
  return (TX + 2 * ao) * (TY_ + 2 * bo) - (TX + 2 * ai) * (TY_ + 2 * bi);
}

// Position of cell r of that annulus, relative to the outer rectangle's corner: the top rows,
// the bottom rows, then the side columns of the rows in between.
template <int TY_, int ai, int bi, int ao, int bo>
__device__ __forceinline__ void annulus_cell(int r, int& ex, int& ey) {
  constexpr int W = TX + 2 * ao, H = TY_ + 2 * bo, tx = ao - ai, ty = bo - bi;
  if (r < ty * W) {
    ey = r / W;
    ex = r - ey * W;
  } else if (r < 2 * ty * W) {
    const int q = r - ty * W;
    ey = H - ty + q / W;
    ex = q % W;
  } else {
    const int q = r - 2 * ty * W;
    ey = ty + q / (2 * tx);
    const int c = q % (2 * tx);
    ex = c < tx ? c : W - tx + (c - tx);
  }
}

// Ring cell r of the region "tile plus hx columns and hy rows on each side"
template <int TY_, int hx, int hy>
__device__ __forceinline__ void ring_cell(int r, int& ex, int& ey) {
  annulus_cell<TY_, 0, 0, hx, hy>(r, ex, ey);
}

// position of halo cell r of the velocity region (one node around the interior)
template <class S>
__device__ __forceinline__ void uring_cell(int r, int& ex, int& ey) {
  if (r < 2 * (TX + 2)) {
    const int side = r / (TX + 2);
    ey = side ? S::EYW - HYW : HYW - 1;
    ex = HXW - 1 + (r - side * (TX + 2));
  } else {
    const int q = r - 2 * (TX + 2);
    ey = HYW + q / 2;
    ex = (q & 1) ? HXW + TX : HXW - 1;
  }
}

// Code variant of a tile.  Variant 0: interior tile (load region inside the grid, away from
// walls and Dirichlet edges): no index wrapping and no boundary tests.  Variants 1-4: any tile,
// compiled for the simulation's boundary kinds, so that a tile pays only for the boundary code
// its simulation can need: 1 + (Dirichlet temperature box) + 2 (walls at y = 0, ny - 1).
template <int V>
struct Variant {
  static constexpr bool INTERIOR = V == 0;
  static constexpr bool TB = V != 0 && ((V - 1) & 1) != 0;
  static constexpr bool WALLS = V != 0 && ((V - 1) & 2) != 0;
};
__device__ __forceinline__ int general_variant(int thermal_box, int y_walls) {
  return 1 + (thermal_box != 0 ? 1 : 0) + (y_walls != 0 ? 2 : 0);
}
// Calls fn(std::integral_constant<int, v>) for the general variant v (1-4).
template <class Fn>
__device__ __forceinline__ void with_general_variant(int v, Fn&& fn) {
  switch (v) {
    case 1: fn(std::integral_constant<int, 1>{}); break;
    case 2: fn(std::integral_constant<int, 2>{}); break;
    case 3: fn(std::integral_constant<int, 3>{}); break;
    default: fn(std::integral_constant<int, 4>{}); break;
  }
}

// Row classification in a walled domain: 0 fluid row, 1 bottom ghost (y=-1), 2 top ghost
// (y=ny), 3 unused.  Periodic domains have fluid rows only (wrapped).
__device__ __forceinline__ int row_kind(int y, int ny, int walls) {
  if (!walls || (y >= 0 && y < ny)) return 0;
  if (y == -1) return 1;
  if (y == ny) return 2;
  return 3;
}

// ------------------------------------------------------------------------- per-node arithmetic

// rho, j, T of a node and its LDS entries (Eqs. 11 and 25), psi with error checks; returns
// (dp/dT)_rho for the node's own collision
// T - T_ref = sum of the thermal populations (Eq. 25), in a fixed order per lattice
template <typename real, int QG>
__device__ __forceinline__ real thermal_sum(const real (&g)[QG]) {
  if constexpr (QG == 9) return ((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + g[7])) + g[8];
  else return ((g[0] + g[1]) + (g[2] + g[3])) + g[4];
}

template <typename real, int QG, class LDS>
__device__ __forceinline__ real node_macro_to_lds(LDS& L, int ex, int ey, const DevParams<real>& p,
                                                  const real (&f)[9], const real (&g)[QG], unsigned& err) {
  const real rho = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
  const real jx = (f[1] - f[3]) + ((f[5] - f[6]) + (f[8] - f[7]));
  const real jy = (f[2] - f[4]) + ((f[5] + f[6]) - (f[7] + f[8]));
  const real T = p.T_ref + thermal_sum<real, QG>(g);
  real psi = real(0), dpdT = real(0);
  if (!(rho > real(0)) || !isfinite(rho)) {
    err |= ERR_RHO;
  } else if (!(T > real(0)) || !isfinite(T)) {
    err |= ERR_T;
  } else {
    real press;
    pr_eos(p, rho, T, press, dpdT);
    psi = psi_from_pressure(p, rho, press, err);
  }
  L.rho[ey][ex] = rho;
  L.irc[ey][ex] = rcp(rho * p.cv);
  L.psi[ey][ex] = psi;
  L.ux[ey][ex] = jx;
  L.uy[ey][ex] = jy;
#pragma unroll
  for (int k = 0; k < QG - 1; ++k) L.g[k][ey][ex] = g[k + 1];
  return dpdT;
}

template <typename real, class LDS>
__device__ __forceinline__ void zero_lds_cell(LDS& L, int ex, int ey) {
  L.rho[ey][ex] = real(0);
  L.irc[ey][ex] = real(0);
  L.psi[ey][ex] = real(0);
  L.ux[ey][ex] = real(0);
  L.uy[ey][ex] = real(0);
  constexpr int NG = (int)(sizeof(L.g) / sizeof(L.g[0]));
#pragma unroll
  for (int k = 0; k < NG; ++k) L.g[k][ey][ex] = real(0);
}

// Stencil of the interaction force: F_m = -G psi(x) (sx, sy) with (sx, sy) =
// sum_i varpi_i psi(x + c_i) c_i (Eq. 9), varpi = 1/3 (axes), 1/12 (diagonals)
template <typename real, class LDS>
__device__ __forceinline__ void psi_stencil(const LDS& L, int ex, int ey, real& sx, real& sy) {
  const real pE = L.psi[ey][ex + 1], pN = L.psi[ey + 1][ex], pW = L.psi[ey][ex - 1], pS = L.psi[ey - 1][ex];
  const real pNE = L.psi[ey + 1][ex + 1], pNW = L.psi[ey + 1][ex - 1], pSW = L.psi[ey - 1][ex - 1],
             pSE = L.psi[ey - 1][ex + 1];
  sx = real(1.0 / 3.0) * (pE - pW) + real(1.0 / 12.0) * ((pNE - pNW) + (pSE - pSW));
  sy = real(1.0 / 3.0) * (pN - pS) + real(1.0 / 12.0) * ((pNE + pNW) - (pSE + pSW));
}

// Interaction force (Eq. 9), buoyancy, and velocity u = (j + F/2) / rho (Eq. 11) of the node at
// (ex, ey); u replaces j in LDS.  S2 = |F_m|^2 / psi^2 of Li's correction (Eq. 8).
template <typename real, class LDS>
__device__ __forceinline__ void node_force_velocity(LDS& L, int ex, int ey, const DevParams<real>& p, bool freeze,
                                                    real& Fx, real& Fy, real& S2) {
  const real rho = L.rho[ey][ex];
  real fx = real(0), fy = real(0), s2 = real(0);
  if (!freeze) {
    real sx, sy;
    psi_stencil<real>(L, ex, ey, sx, sy);
    const real c = -p.G * L.psi[ey][ex];
    fx = c * sx + (rho - p.rho_ave) * p.gx;
    fy = c * sy + (rho - p.rho_ave) * p.gy;
    s2 = p.GG * (sx * sx + sy * sy);
  }
  Fx = fx;
  Fy = fy;
  S2 = s2;
  const real ir = L.irc[ey][ex] * p.cv;  // 1/rho
  L.ux[ey][ex] = (L.ux[ey][ex] + real(0.5) * fx) * ir;
  L.uy[ey][ex] = (L.uy[ey][ex] + real(0.5) * fy) * ir;
}

// div u = 3 sum_i w_i c_i . u(x + c_i); a ghost row carries -u of the fluid row next to it
// (gs_: the node is on the bottom fluid row of a walled domain, gn_: on the top one), or +u
// above an open top (sn = +1 instead of -1: zero gradient)
template <typename real, class LDS>
__device__ __forceinline__ real node_divu(const LDS& L, int ex, int ey, bool gs_, bool gn_, real sn = real(-1)) {
  const real uy = L.uy[ey][ex];
  const real uxE = L.ux[ey][ex + 1], uxW = L.ux[ey][ex - 1];
  const real uyN = gn_ ? sn * uy : L.uy[ey + 1][ex];
  const real uyS = gs_ ? -uy : L.uy[ey - 1][ex];
  const real uxNE = gn_ ? sn * uxE : L.ux[ey + 1][ex + 1], uyNE = gn_ ? sn * L.uy[ey][ex + 1] : L.uy[ey + 1][ex + 1];
  const real uxNW = gn_ ? sn * uxW : L.ux[ey + 1][ex - 1], uyNW = gn_ ? sn * L.uy[ey][ex - 1] : L.uy[ey + 1][ex - 1];
  const real uxSW = gs_ ? -uxW : L.ux[ey - 1][ex - 1], uySW = gs_ ? -L.uy[ey][ex - 1] : L.uy[ey - 1][ex - 1];
  const real uxSE = gs_ ? -uxE : L.ux[ey - 1][ex + 1], uySE = gs_ ? -L.uy[ey][ex + 1] : L.uy[ey - 1][ex + 1];
  return real(1.0 / 3.0) * ((uxE - uxW) + (uyN - uyS)) +
         real(1.0 / 12.0) * (((uxNE - uxSW) + (uxSE - uxNW)) + ((uyNE - uySW) + (uyNW - uySE)));
}

// Collision of one node: grad T from the relaxed non-equilibrium first moments of the thermal
// populations (Eqs. 49-50), Q (Eq. 20), S (Eq. 24), the D2Q9 MRT collision with Li's forcing,
// and the thermal collision: D2Q5 MRT (Eq. 39), or BGK (Eq. 21) on the D2Q9 thermal lattice.
// Tr = T - T_ref of the node; T1, T2 are T(t-1) - T_ref and T(t-2) - T_ref.
template <typename real, int QG>
__device__ __forceinline__ void node_collide(const DevParams<real>& p, bool freeze, const real (&f)[9],
                                             const real (&g)[QG], real rho, real ux, real uy, real fx, real fy,
                                             real S2, real dpdT, real divu, real T1, real T2, real (&fs_)[9],
                                             real (&gs_)[QG], real& Tr) {
  Tr = thermal_sum<real, QG>(g);  // T - T_ref
  const real T = p.T_ref + Tr;
  // first moments sum_i c_i g_i (their equilibrium parts vanish), relaxed by 1/tau_g
  real dm1, dm2;
  if constexpr (QG == 9) {
    dm1 = p.vs1 * ((g[1] - g[3]) + ((g[5] - g[6]) + (g[8] - g[7])));
    dm2 = p.vs1 * ((g[2] - g[4]) + ((g[5] + g[6]) - (g[7] + g[8])));
  } else {
    dm1 = p.vs1 * (g[1] - g[3]);
    dm2 = p.vs1 * (g[2] - g[4]);
  }
  const real dTx = -dm1 * p.inv_cs2h;
  const real dTy = -dm2 * p.inv_cs2h;
  const real rcv = rho * p.cv;
  const real Q = -(rcv * (ux * dTx + uy * dTy) + T * dpdT * divu);
  const real Ssum = (p.flags & FL_NO_S) ? real(0) : rcv * real(0.5) * ((Tr - T1) - (T1 - T2));

  // ---- D2Q9 MRT collision with Li's forcing, moments of the orthogonal basis of Eq. (4).
  // Applied as a correction f* = f + M^-1 dm with dm = -S (m - m_eq) + (1 - S/2) F (Eq. 5):
  // dm_0 = 0, so mass is conserved to rounding (no product of rho with a rounded 1/9).
  if (freeze) {
#pragma unroll
    for (int i = 0; i < 9; ++i) fs_[i] = f[i];
  } else {
    const real* fi = f;
    const real sa = (fi[1] + fi[2]) + (fi[3] + fi[4]);
    const real sd = (fi[5] + fi[6]) + (fi[7] + fi[8]);
    const real m1 = -real(4) * fi[0] - sa + real(2) * sd;
    const real m2 = real(4) * fi[0] - real(2) * sa + sd;
    const real m4 = real(-2) * (fi[1] - fi[3]) + ((fi[5] - fi[6]) + (fi[8] - fi[7]));
    const real m6 = real(-2) * (fi[2] - fi[4]) + ((fi[5] + fi[6]) - (fi[7] + fi[8]));
    const real m7 = (fi[1] - fi[2]) + (fi[3] - fi[4]);
    const real m8 = (fi[5] - fi[6]) + (fi[7] - fi[8]);
    const real uu = ux * ux + uy * uy;
    const real uF = ux * fx + uy * fy;
    const real F1 = real(6) * uF + p.corr_e * S2;
    const real F2 = -real(6) * uF - p.corr_eps * S2;
    const real F7 = real(2) * (ux * fx - uy * fy);
    const real F8 = ux * fy + uy * fx;
    // m_eq of Eq. (7); the conserved moments j change by exactly F (s_j drops out)
    const real d1 = -p.s_e * (m1 - rho * (real(-2) + real(3) * uu)) + p.om_e * F1;
    const real d2 = -p.s_eps * (m2 - rho * (real(1) - real(3) * uu)) + p.om_eps * F2;
    const real d4 = -p.s_q * (m4 + rho * ux) - p.om_q * fx;
    const real d6 = -p.s_q * (m6 + rho * uy) - p.om_q * fy;
    const real d7 = -p.s_p * (m7 - rho * (ux * ux - uy * uy)) + p.om_p * F7;
    const real d8 = -p.s_p * (m8 - rho * ux * uy) + p.om_p * F8;
    // M^-1 = M^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4)
    const real b1 = d1 * real(1.0 / 36.0), b2 = d2 * real(1.0 / 36.0);
    const real c3 = fx * real(1.0 / 6.0), c4 = d4 * real(1.0 / 12.0);
    const real c5 = fy * real(1.0 / 6.0), c6 = d6 * real(1.0 / 12.0);
    const real e7 = d7 * real(0.25), e8 = d8 * real(0.25);
    const real axis = -b1 - real(2) * b2;
    const real diag = real(2) * b1 + b2;
    const real cx_ = c3 - real(2) * c4, cy_ = c5 - real(2) * c6;
    const real dx_ = c3 + c4, dy_ = c5 + c6;
    fs_[0] = fi[0] + (real(4) * (b2 - b1));
    fs_[1] = fi[1] + ((axis + cx_) + e7);
    fs_[2] = fi[2] + ((axis + cy_) - e7);
    fs_[3] = fi[3] + ((axis - cx_) + e7);
    fs_[4] = fi[4] + ((axis - cy_) - e7);
    fs_[5] = fi[5] + ((diag + (dx_ + dy_)) + e8);
    fs_[6] = fi[6] + ((diag - (dx_ - dy_)) - e8);
    fs_[7] = fi[7] + ((diag - (dx_ + dy_)) + e8);
    fs_[8] = fi[8] + ((diag + (dx_ - dy_)) - e8);
  }

  if constexpr (QG == 9) {
    // ---- BGK collision (Eq. 21) with the linear equilibrium w_i T (Eq. 22); the stored g and
    // Tr are shifted by w_i T_ref and T_ref alike, so g - g_eq is unchanged by the shift
    const real src = Q + Ssum;
    const real e0 = p.w0h * Tr, e1 = p.w1h * Tr, e2 = p.w2h * Tr;
    const real s0 = p.w0h * src, s1 = p.w1h * src, s2 = p.w2h * src;
    gs_[0] = g[0] + (p.vs1 * (e0 - g[0]) + s0);
#pragma unroll
    for (int i = 1; i < 5; ++i) gs_[i] = g[i] + (p.vs1 * (e1 - g[i]) + s1);
#pragma unroll
    for (int i = 5; i < 9; ++i) gs_[i] = g[i] + (p.vs1 * (e2 - g[i]) + s2);
  } else {
    // ---- D2Q5 MRT collision (Eq. 39) with the non-orthogonal basis of Eq. (40)
    const real* gi = g;
    const real dm3 = p.vs3 * (((gi[1] + gi[2]) + (gi[3] + gi[4])) - p.wdot * Tr);
    const real dm4 = p.vs4 * ((gi[1] - gi[2]) + (gi[3] - gi[4]));
    const real src = Q + Ssum;
    const real q34p = real(0.25) * (dm3 + dm4), q34m = real(0.25) * (dm3 - dm4);
    gs_[0] = gi[0] + dm3 + p.w0h * src;
    gs_[1] = gi[1] - (q34p + real(0.5) * dm1) + p.w1h * src;
    gs_[3] = gi[3] - (q34p - real(0.5) * dm1) + p.w1h * src;
    gs_[2] = gi[2] - (q34m + real(0.5) * dm2) + p.w1h * src;
    gs_[4] = gi[4] - (q34m - real(0.5) * dm2) + p.w1h * src;
  }
}

// Wetting ghost rows of an LDS region whose cell (0, 0) is the grid node (ox, oy):
// psi at the ghost node from rho_0 = rho_2 + tan(pi/2 - theta) |rho_{x+1,1} - rho_{x-1,1}|
// (Eq. 54) at the wall temperature.  Returns true if the region holds a ghost row (the caller
// then needs a barrier).
template <typename real, int W, int H, class LDS, class WX>
__device__ __forceinline__ bool ghost_rows(LDS& L, const DevParams<real>& p, int ox, int oy, int ny, int tid, int nt,
                                           WX wx, unsigned& err) {
  const int eyb = -1 - oy;  // LDS row of y = -1
  const int eyt = ny - oy;  // LDS row of y = ny
  const bool hasb = eyb >= 0 && eyb < H, hast = eyt >= 0 && eyt < H;
  if (!(hasb || hast)) return false;
  for (int c = tid; c < 2 * W; c += nt) {
    const int top = c >= W;
    const int ex = c - top * W;
    const int ey = top ? eyt : eyb;
    if (top && hast && p.open_top) {
      L.psi[ey][ex] = L.psi[ey - 1][ex];  // above an open top: zero gradient
    } else if ((top ? hast : hasb) && ex >= 1 && ex <= W - 2) {
      const int d = top ? -1 : 1;  // towards the fluid
      const real tanv = top ? p.tan_top : p.tan_bot;
      const real rg = L.rho[ey + 2 * d][ex] + tanv * fabs(L.rho[ey + d][ex + 1] - L.rho[ey + d][ex - 1]);
      const real Tw = wall_temperature(p, top, wx(ox + ex));
      L.psi[ey][ex] = pseudo(p, rg, Tw, err);
    }
  }
  return true;
}

// ------------------------------------------------------------------------- one step

// Where the one-step body takes f and g from: the global A/B buffers, or the LDS state left by
// the first step of a two-step launch (with the temperature history handed over in registers).
template <typename real, class S>
struct LdsState {
  const real (*sf)[S::EYW][EXW];
  const real (*sg)[S::EYW][EXW];
  const real* T1;  // per own row: T(t-1) - T_ref, T(t-2) - T_ref after the first step
  const real* T2;
};

// One step of one tile (code variant V, see Variant).  Interior tiles (load region entirely inside the grid, away from walls
// and Dirichlet edges) need no index wrapping and no boundary tests; the general variant
// handles periodic wrap, wall ghost rows, bounce-back and anti-bounce-back.  Both variants
// perform the same arithmetic on every node.  FROM_LDS: f and g come from `st` (second step of
// a two-step launch) instead of the global source buffers.
template <typename real, class S, int V, bool FROM_LDS, int QG = 5>
__device__ __forceinline__ void step_body(const InstDesc<real>& D, StepLds<real, S::EYW, QG>& L, bool odd, bool hodd,
                                          int x0, int y0, const LdsState<real, S>& st, unsigned& err, int tid) {
  static_assert(!FROM_LDS || QG == 5, "the two-step state in LDS holds D2Q5 thermal populations");
  constexpr int NT = S::NT, RPT = S::RPT, WAVES = S::WAVES, RING = S::RING, URING = S::URING, EYW = S::EYW;
  const int nx = D.nx, ny = D.ny;
  constexpr ptrdiff_t SZ = sizeof(real);
  const ptrdiff_t PB = (ptrdiff_t)nx * (ptrdiff_t)ny * SZ;  // bytes per plane
  const gptr<const char> fs = (gptr<const char>)to_global<const real>(odd ? D.fB : D.fA);
  const gptr<const char> gs = (gptr<const char>)to_global<const real>(odd ? D.gB : D.gA);
  const gptr<char> fd = (gptr<char>)to_global<real>(odd ? D.fA : D.fB);
  const gptr<char> gd = (gptr<char>)to_global<real>(odd ? D.gA : D.gB);
  // temperature history: a step that reads only its own nodes' history (every step but the second
  // of a two-step launch, whose first step read the ring's) updates it in place; the second step
  // of a two-step launch writes the other copy
  const gptr<const char> Ths = (gptr<const char>)to_global<const real>(hodd ? D.ThB : D.ThA);
  const gptr<char> Thd = (gptr<char>)to_global<real>((hodd != FROM_LDS) ? D.ThB : D.ThA);
  DevParams<real> p = D.p;
  // rho_ave of the buoyancy: the current mean density where mass crosses an open top
  if (p.live_rho_ave) p.rho_ave = (real)D.live->rho_ave;
  constexpr bool INTERIOR = Variant<V>::INTERIOR;
  constexpr int walls = Variant<V>::WALLS ? 1 : 0;
  constexpr bool tb = Variant<V>::TB;
  const bool freeze = (p.flags & FL_FREEZE_FLOW) != 0;
  const bool tiny = nx < EXW + 1 || ny < EYW + 1;  // periodic images closer than one halo

  const int tx = tid & (TX - 1);
  const int ty = tid >> 6;

  auto wx = [&](int v) { return INTERIOR ? v : wrapi(v, nx, tiny); };
  auto wy = [&](int v) { return (INTERIOR || walls) ? v : wrapi(v, ny, tiny); };
  auto fluid_row = [&](int y) { return INTERIOR || row_kind(y, ny, walls) == 0; };
  auto gdp = [&](int i) { return sbase(gd + i * opaque(PB)); };  // D2Q9 thermal stores

  // ---- phase 1: every global load of the tile is issued first (own nodes with their T
  // history, then the halo ring), so that the workgroup waits for memory once.  Own nodes keep
  // f, g and the history in registers.
  constexpr int RPN = (RING + NT - 1) / NT;  // halo ring nodes per thread
  const int xg = x0 + tx;
  const int xw = wx(xg);
  real f[RPT][9], g[RPT][QG], T1[RPT], T2[RPT], dpdT[RPT];
  unsigned ob[RPT];  // byte offset of the own node in a plane
  bool own[RPT];
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int yg = y0 + ty + WAVES * r;
    const int ey = HYW + ty + WAVES * r;
    own[r] = fluid_row(yg);
    ob[r] = (unsigned)(wy(yg) * nx + xw) * (unsigned)SZ;
    if (own[r]) {
      if constexpr (FROM_LDS) {
#pragma unroll
        for (int i = 0; i < 9; ++i) f[r][i] = st.sf[i][ey][HXW + tx];
#pragma unroll
        for (int i = 0; i < QG; ++i) g[r][i] = st.sg[i][ey][HXW + tx];
        T1[r] = st.T1[r];
        T2[r] = st.T2[r];
      } else {
        PlaneWalk<const char> wf{fs, PB}, wg{gs, PB};
#pragma unroll
        for (int i = 0; i < 9; ++i) f[r][i] = ldb<real>(wf.next(), ob[r]);
#pragma unroll
        for (int i = 0; i < QG; ++i) g[r][i] = ldb<real>(wg.next(), ob[r]);
        T1[r] = ldb<real>(Ths, ob[r]);
        T2[r] = ldb<real>(sbase(Ths + opaque(PB)), ob[r]);
      }
    } else {
#pragma unroll
      for (int i = 0; i < 9; ++i) f[r][i] = real(0);
#pragma unroll
      for (int i = 0; i < QG; ++i) g[r][i] = real(0);
      T1[r] = T2[r] = real(0);
    }
  }
  real fr[RPN][9], gr[RPN][QG];
  int rex[RPN], rey[RPN];
  bool rin[RPN], rfl[RPN];
#pragma unroll
  for (int q = 0; q < RPN; ++q) {
    const int r = tid + q * NT;
    rin[q] = r < RING;
    ring_cell<S::TY, HXW, HYW>(rin[q] ? r : 0, rex[q], rey[q]);
    const int yg = y0 - HYW + rey[q];
    rfl[q] = rin[q] && fluid_row(yg);
    if (rfl[q]) {
      if constexpr (FROM_LDS) {
#pragma unroll
        for (int i = 0; i < 9; ++i) fr[q][i] = st.sf[i][rey[q]][rex[q]];
#pragma unroll
        for (int i = 0; i < QG; ++i) gr[q][i] = st.sg[i][rey[q]][rex[q]];
      } else {
        const unsigned o = (unsigned)(wy(yg) * nx + wx(x0 - HXW + rex[q])) * (unsigned)SZ;
        PlaneWalk<const char> wf{fs, PB}, wg{gs, PB};
#pragma unroll
        for (int i = 0; i < 9; ++i) fr[q][i] = ldb<real>(wf.next(), o);
#pragma unroll
        for (int i = 0; i < QG; ++i) gr[q][i] = ldb<real>(wg.next(), o);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int ey = HYW + ty + WAVES * r;
    dpdT[r] = real(0);
    if (own[r]) dpdT[r] = node_macro_to_lds<real, QG>(L, HXW + tx, ey, p, f[r], g[r], err);
    else zero_lds_cell<real>(L, HXW + tx, ey);
  }
#pragma unroll
  for (int q = 0; q < RPN; ++q) {
    if (rfl[q]) (void)node_macro_to_lds<real, QG>(L, rex[q], rey[q], p, fr[q], gr[q], err);
    else if (rin[q]) zero_lds_cell<real>(L, rex[q], rey[q]);
  }
  __syncthreads();

  // ---- phase 1b: wetting ghost rows
  if constexpr (walls != 0) {
    if (ghost_rows<real, EXW, EYW>(L, p, x0 - HXW, y0 - HYW, ny, tid, NT, wx, err)) __syncthreads();
  }

  // ---- phase 2: forces and velocity on the tile plus one node
  real Fx[RPT], Fy[RPT], S2[RPT];
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int ex = HXW + tx, ey = HYW + ty + WAVES * r;
    Fx[r] = Fy[r] = S2[r] = real(0);
    if (own[r]) node_force_velocity<real>(L, ex, ey, p, freeze, Fx[r], Fy[r], S2[r]);
  }
  for (int r = tid; r < URING; r += NT) {
    int ex, ey;
    uring_cell<S>(r, ex, ey);
    const int yg = y0 - HYW + ey;
    if (fluid_row(yg)) {
      real fx, fy, s2;
      node_force_velocity<real>(L, ex, ey, p, freeze, fx, fy, s2);
    }
  }
  __syncthreads();

  // ---- phase 3: collision and streaming of the own nodes
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int ex = HXW + tx, ey = HYW + ty + WAVES * r;
    const int yg = y0 + ty + WAVES * r;
    if (!INTERIOR && (xg >= nx || yg >= ny)) continue;
    const real rho = L.rho[ey][ex];
    const real ux = L.ux[ey][ex], uy = L.uy[ey][ex];
    const unsigned o = ob[r];
    const real divu = node_divu<real>(L, ex, ey, walls && yg == 0, walls && yg == ny - 1,
                                      walls && p.open_top ? real(1) : real(-1));
    real fs_[9], gs_[QG], Tr;
    node_collide<real, QG>(p, freeze, f[r], g[r], rho, ux, uy, Fx[r], Fy[r], S2[r], dpdT[r], divu, T1[r], T2[r],
                           fs_, gs_, Tr);
    stb(Thd, o, Tr);
    stb(sbase(Thd + opaque(PB)), o, T1[r]);

    // ---- streaming.  Interior tiles: a neighbour's byte offset differs from the node's by a
    // uniform amount, folded into the plane base.  Other tiles: wrapped offsets of the eight
    // neighbours (a wall row is never written).
    const ptrdiff_t RB = (ptrdiff_t)nx * SZ;
    const bool wall_n = walls && yg == ny - 1, wall_s = walls && yg == 0;
    const unsigned cE = (unsigned)wx(xg + 1), cW = (unsigned)wx(xg - 1);
    const unsigned rowc = (unsigned)(yg * nx);
    const unsigned rown = wall_n ? 0u : (unsigned)(wy(yg + 1) * nx);
    const unsigned rows = wall_s ? 0u : (unsigned)(wy(yg - 1) * nx);
    const unsigned xwu = (unsigned)xw;
    // destination of a population moving by (dx, dy): plane base and byte offset
    auto dst = [&](gptr<char> plane, int dx, int dy, unsigned& off) -> gptr<char> {
      if (INTERIOR) {
        off = o;
        return sbase(plane + (dy * RB + dx * SZ));
      }
      const unsigned row = dy > 0 ? rown : dy < 0 ? rows : rowc;
      const unsigned col = dx > 0 ? cE : dx < 0 ? cW : xwu;
      off = (row + col) * (unsigned)SZ;
      return plane;
    };
    unsigned off;

    // f: push to x + c_i, halfway bounce-back through the walls (Eq. 6).  The destination planes
    // are written in order, each receiving the push of its own population and, at a wall, the
    // bounce-back of the opposite one.  At the top wall the upward populations bounce back; under
    // an open top they leave instead: the boundary pass after the step reads them from these slots
    // as the outflow of the top row, then replaces them by the populations that enter from outside.
    PlaneWalk<char> wd{fd, PB};
    if (freeze) {
#pragma unroll
      for (int i = 0; i < 9; ++i) stb(wd.next(), o, fs_[i]);
    } else {
      stb(wd.next(), o, fs_[0]);
      { const auto pl = wd.next(); const auto b = dst(pl, 1, 0, off); stb(b, off, fs_[1]); }
      {
        const auto pl = wd.next();
        if (!wall_n) { const auto b = dst(pl, 0, 1, off); stb(b, off, fs_[2]); }
        if (wall_s) stb(pl, o, fs_[4]);
      }
      { const auto pl = wd.next(); const auto b = dst(pl, -1, 0, off); stb(b, off, fs_[3]); }
      {
        const auto pl = wd.next();
        if (!wall_s) { const auto b = dst(pl, 0, -1, off); stb(b, off, fs_[4]); }
        if (wall_n) stb(pl, o, fs_[2]);
      }
      {
        const auto pl = wd.next();
        if (!wall_n) { const auto b = dst(pl, 1, 1, off); stb(b, off, fs_[5]); }
        if (wall_s) stb(pl, o, fs_[7]);
      }
      {
        const auto pl = wd.next();
        if (!wall_n) { const auto b = dst(pl, -1, 1, off); stb(b, off, fs_[6]); }
        if (wall_s) stb(pl, o, fs_[8]);
      }
      {
        const auto pl = wd.next();
        if (!wall_s) { const auto b = dst(pl, -1, -1, off); stb(b, off, fs_[7]); }
        if (wall_n) stb(pl, o, fs_[5]);
      }
      {
        const auto pl = wd.next();
        if (!wall_s) { const auto b = dst(pl, 1, -1, off); stb(b, off, fs_[8]); }
        if (wall_n) stb(pl, o, fs_[6]);
      }
    }

    // g with the modified collision of Eq. (39):
    //   g_i(y, t+1) = g_i(y, t) + [g*_i(y - c_i) - g_i(y, t)] / (rho(y, t) c_v)
    // An edge with a Dirichlet temperature replaces the upstream term by anti-bounce-back,
    // -g*_i(y) + 2 what_i T_w, for the population entering y in the opposite direction.
    if constexpr (QG == 9) {
      // D2Q9 thermal lattice: a population whose destination lies beyond a Dirichlet edge
      // (x edges of the temperature box; y edges of the box or the walls, corners included)
      // returns to the node in the opposite direction by anti-bounce-back at the temperature of
      // that edge; every other one is pushed and blended at its destination.
      const real ircv = L.irc[ey][ex];
      stb(gdp(0), o, g[r][0] + (gs_[0] - g[r][0]) * ircv);
      constexpr int CXg[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
      constexpr int CYg[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
      constexpr int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
#pragma unroll
      for (int i = 1; i < 9; ++i) {
        const int dx = CXg[i], dy = CYg[i];
        const bool out_x = tb && ((dx > 0 && xg == nx - 1) || (dx < 0 && xg == 0));
        const bool out_y = (walls || tb) && ((dy > 0 && yg == ny - 1) || (dy < 0 && yg == 0));
        if (out_x || out_y) {
          const real Tw = tb ? p.T_box : dy < 0 ? wall_temperature(p, 0, xw) : p.T_top;
          const real two_w = i < 5 ? p.two_w1h : p.two_w2h;
          const int b = OPP[i];
          const real up = -gs_[i] + two_w * (Tw - p.T_ref);
          stb(gdp(b), o, g[r][b] + (up - g[r][b]) * ircv);
        } else {
          const real gold = L.g[i - 1][ey + dy][ex + dx];
          auto bp = dst(gdp(i), dx, dy, off);
          stb(bp, off, gold + (gs_[i] - gold) * L.irc[ey + dy][ex + dx]);
        }
      }
    } else {
      // D2Q5: the destination planes in order, each receiving the push of its own population and,
      // at a Dirichlet edge, the anti-bounce-back of the opposite one
      const real ircv = L.irc[ey][ex];
      const bool out_e = tb && xg == nx - 1, out_w = tb && xg == 0;
      const bool out_n = (walls || tb) && yg == ny - 1, out_s = (walls || tb) && yg == 0;
      const real two_w = p.two_w1h;
      PlaneWalk<char> wg{gd, PB};
      stb(wg.next(), o, g[r][0] + (gs_[0] - g[r][0]) * ircv);
      {
        const auto pl = wg.next();
        if (!out_e) {
          const real gold = L.g[0][ey][ex + 1];
          const auto b = dst(pl, 1, 0, off);
          stb(b, off, gold + (gs_[1] - gold) * L.irc[ey][ex + 1]);
        }
        if (out_w) {
          const real up = -gs_[3] + two_w * (p.T_box - p.T_ref);
          stb(pl, o, g[r][1] + (up - g[r][1]) * ircv);
        }
      }
      {
        const auto pl = wg.next();
        if (!out_n) {
          const real gold = L.g[1][ey + 1][ex];
          const auto b = dst(pl, 0, 1, off);
          stb(b, off, gold + (gs_[2] - gold) * L.irc[ey + 1][ex]);
        }
        if (out_s) {
          const real Ts = tb ? p.T_box : wall_temperature(p, 0, xw);
          const real up = -gs_[4] + two_w * (Ts - p.T_ref);
          stb(pl, o, g[r][2] + (up - g[r][2]) * ircv);
        }
      }
      {
        const auto pl = wg.next();
        if (!out_w) {
          const real gold = L.g[2][ey][ex - 1];
          const auto b = dst(pl, -1, 0, off);
          stb(b, off, gold + (gs_[3] - gold) * L.irc[ey][ex - 1]);
        }
        if (out_e) {
          const real up = -gs_[1] + two_w * (p.T_box - p.T_ref);
          stb(pl, o, g[r][3] + (up - g[r][3]) * ircv);
        }
      }
      {
        const auto pl = wg.next();
        if (!out_s) {
          const real gold = L.g[3][ey - 1][ex];
          const auto b = dst(pl, 0, -1, off);
          stb(b, off, gold + (gs_[4] - gold) * L.irc[ey - 1][ex]);
        }
        if (out_n) {
          const real Tn = tb ? p.T_box : p.T_top;
          const real up = -gs_[2] + two_w * (Tn - p.T_ref);
          stb(pl, o, g[r][4] + (up - g[r][4]) * ircv);
        }
      }
    }
  }
}

// ------------------------------------------------------------------------- two steps

// First step of a two-step launch on the region the second step reads.  Region names, as
// offsets around the tile (columns, rows): the first step loads M (MXH, MYH) = (HXW + 4, HYW + 3),
// computes forces and velocities on C+1 = (HXW + 2, HYW + 2), collides C = (HXW + 1, HYW + 1),
// and streams into the state arrays over the second step's load region (HXW, HYW).  Pushes that
// leave that region are dropped; every kept slot is written exactly once.
template <typename real, class S, int V>
__device__ __forceinline__ void first_step(const InstDesc<real>& D, Step2Lds<real, S>& L, bool odd, bool hodd, int x0,
                                           int y0, real (&Tn1)[S::RPT], real (&Tn2)[S::RPT], unsigned& err, int tid) {
  constexpr int NT = S::NT, RPT = S::RPT, WAVES = S::WAVES, MX = S::MX, MY = S::MY, MXH = S::MXH, MYH = S::MYH;
  constexpr int MRING = MX * MY - TX * S::TY;
  constexpr int RPN = (MRING + NT - 1) / NT;
  constexpr int DX = MXH - HXW, DY = MYH - HYW;  // state cell (sx, sy) = M cell (sx + DX, sy + DY)
  const int nx = D.nx, ny = D.ny;
  constexpr ptrdiff_t SZ = sizeof(real);
  const ptrdiff_t PB = (ptrdiff_t)nx * (ptrdiff_t)ny * SZ;
  const gptr<const char> fs = (gptr<const char>)to_global<const real>(odd ? D.fB : D.fA);
  const gptr<const char> gs = (gptr<const char>)to_global<const real>(odd ? D.gB : D.gA);
  const gptr<const char> Th = (gptr<const char>)to_global<const real>(hodd ? D.ThB : D.ThA);
  const DevParams<real> p = D.p;
  constexpr bool INTERIOR = Variant<V>::INTERIOR;
  constexpr int walls = Variant<V>::WALLS ? 1 : 0;
  constexpr bool tb = Variant<V>::TB;
  const bool freeze = (p.flags & FL_FREEZE_FLOW) != 0;
  const bool tiny = nx < MX + 1 || ny < MY + 1;

  const int tx = tid & (TX - 1);
  const int ty = tid >> 6;

  auto wx = [&](int v) { return INTERIOR ? v : wrapi(v, nx, tiny); };
  auto wy = [&](int v) { return (INTERIOR || walls) ? v : wrapi(v, ny, tiny); };
  auto fluid_row = [&](int y) { return INTERIOR || row_kind(y, ny, walls) == 0; };
  auto in_c = [](int mx, int my) { return mx >= MXH - HXW - 1 && mx < MX - (MXH - HXW - 1) && my >= MYH - HYW - 1 &&
                                          my < MY - (MYH - HYW - 1); };
  auto in_u = [](int mx, int my) { return mx >= MXH - HXW - 2 && mx < MX - (MXH - HXW - 2) && my >= MYH - HYW - 2 &&
                                          my < MY - (MYH - HYW - 2); };

  // nodes of this thread: RPT own rows, then RPN cells of the ring of M
  constexpr int NN = RPT + RPN;
  real f[NN][9], g[NN][5], T1[NN], T2[NN], dpdT[NN];
  int mx_[NN], my_[NN];
  bool valid[NN], fl[NN];
#pragma unroll
  for (int n = 0; n < NN; ++n) {
    if (n < RPT) {
      mx_[n] = MXH + tx;
      my_[n] = MYH + ty + WAVES * n;
      valid[n] = true;
    } else {
      const int r = tid + (n - RPT) * NT;
      valid[n] = r < MRING;
      ring_cell<S::TY, MXH, MYH>(valid[n] ? r : 0, mx_[n], my_[n]);
    }
    const int xgl = x0 - MXH + mx_[n], ygl = y0 - MYH + my_[n];
    fl[n] = valid[n] && fluid_row(ygl);
    T1[n] = T2[n] = real(0);
    if (fl[n]) {
      const unsigned o = (unsigned)(wy(ygl) * nx + wx(xgl)) * (unsigned)SZ;
      PlaneWalk<const char> wf{fs, PB}, wg{gs, PB};
#pragma unroll
      for (int i = 0; i < 9; ++i) f[n][i] = ldb<real>(wf.next(), o);
#pragma unroll
      for (int i = 0; i < 5; ++i) g[n][i] = ldb<real>(wg.next(), o);
      if (in_c(mx_[n], my_[n])) {
        T1[n] = ldb<real>(Th, o);
        T2[n] = ldb<real>(sbase(Th + opaque(PB)), o);
      }
    }
  }
#pragma unroll
  for (int n = 0; n < NN; ++n) {
    dpdT[n] = real(0);
    if (fl[n]) dpdT[n] = node_macro_to_lds<real, 5>(L.m1, mx_[n], my_[n], p, f[n], g[n], err);
    else if (valid[n]) zero_lds_cell<real>(L.m1, mx_[n], my_[n]);
  }
  __syncthreads();

  if constexpr (walls != 0) {
    if (ghost_rows<real, MX, MY>(L.m1, p, x0 - MXH, y0 - MYH, ny, tid, NT, wx, err)) __syncthreads();
  }

  real Fx[NN], Fy[NN], S2[NN];
#pragma unroll
  for (int n = 0; n < NN; ++n) {
    Fx[n] = Fy[n] = S2[n] = real(0);
    if (fl[n] && in_u(mx_[n], my_[n])) node_force_velocity<real>(L.m1, mx_[n], my_[n], p, freeze, Fx[n], Fy[n], S2[n]);
  }
  __syncthreads();

  // collision of C and streaming into the state arrays
  auto in_s = [](int sx, int sy) { return sx >= 0 && sx < EXW && sy >= 0 && sy < S::EYW; };
#pragma unroll
  for (int n = 0; n < NN; ++n) {
    const int mx = mx_[n], my = my_[n];
    if (!fl[n] || !in_c(mx, my)) continue;
    const int xw = wx(x0 - MXH + mx), yw = wy(y0 - MYH + my);  // node of the grid (wrapped image)
    const real rho = L.m1.rho[my][mx];
    const real ux = L.m1.ux[my][mx], uy = L.m1.uy[my][mx];
    const real divu = node_divu<real>(L.m1, mx, my, walls && yw == 0, walls && yw == ny - 1);
    real fs_[9], gs_[5], Tr;
    node_collide<real, 5>(p, freeze, f[n], g[n], rho, ux, uy, Fx[n], Fy[n], S2[n], dpdT[n], divu, T1[n], T2[n], fs_, gs_,
                       Tr);
    if (n < RPT) {  // own node: history after this step
      Tn1[n] = Tr;
      Tn2[n] = T1[n];
    }
    const int sx = mx - DX, sy = my - DY;
    auto putf = [&](int i, int dx, int dy, real v) {
      if (in_s(sx + dx, sy + dy)) L.sf[i][sy + dy][sx + dx] = v;
    };
    auto putg = [&](int i, int dx, int dy, real v) {
      if (in_s(sx + dx, sy + dy)) L.sg[i][sy + dy][sx + dx] = v;
    };
    const bool wall_n = walls && yw == ny - 1, wall_s = walls && yw == 0;
    if (freeze) {
#pragma unroll
      for (int i = 0; i < 9; ++i) putf(i, 0, 0, fs_[i]);
    } else {
      putf(0, 0, 0, fs_[0]);
      putf(1, 1, 0, fs_[1]);
      putf(3, -1, 0, fs_[3]);
      if (wall_n) {
        putf(4, 0, 0, fs_[2]);
        putf(7, 0, 0, fs_[5]);
        putf(8, 0, 0, fs_[6]);
      } else {
        putf(2, 0, 1, fs_[2]);
        putf(5, 1, 1, fs_[5]);
        putf(6, -1, 1, fs_[6]);
      }
      if (wall_s) {
        putf(2, 0, 0, fs_[4]);
        putf(5, 0, 0, fs_[7]);
        putf(6, 0, 0, fs_[8]);
      } else {
        putf(4, 0, -1, fs_[4]);
        putf(7, -1, -1, fs_[7]);
        putf(8, 1, -1, fs_[8]);
      }
    }
    const real ircv = L.m1.irc[my][mx];
    putg(0, 0, 0, g[n][0] + (gs_[0] - g[n][0]) * ircv);
    const bool out_e = tb && xw == nx - 1, out_w = tb && xw == 0;
    const bool out_n = (walls || tb) && yw == ny - 1, out_s = (walls || tb) && yw == 0;
    const real two_w = p.two_w1h;
    if (out_e) {
      const real up = -gs_[1] + two_w * (p.T_box - p.T_ref);
      putg(3, 0, 0, g[n][3] + (up - g[n][3]) * ircv);
    } else {
      const real gold = L.m1.g[0][my][mx + 1];
      putg(1, 1, 0, gold + (gs_[1] - gold) * L.m1.irc[my][mx + 1]);
    }
    if (out_w) {
      const real up = -gs_[3] + two_w * (p.T_box - p.T_ref);
      putg(1, 0, 0, g[n][1] + (up - g[n][1]) * ircv);
    } else {
      const real gold = L.m1.g[2][my][mx - 1];
      putg(3, -1, 0, gold + (gs_[3] - gold) * L.m1.irc[my][mx - 1]);
    }
    if (out_n) {
      const real Tn = tb ? p.T_box : p.T_top;
      const real up = -gs_[2] + two_w * (Tn - p.T_ref);
      putg(4, 0, 0, g[n][4] + (up - g[n][4]) * ircv);
    } else {
      const real gold = L.m1.g[1][my + 1][mx];
      putg(2, 0, 1, gold + (gs_[2] - gold) * L.m1.irc[my + 1][mx]);
    }
    if (out_s) {
      const real Ts = tb ? p.T_box : wall_temperature(p, 0, xw);
      const real up = -gs_[4] + two_w * (Ts - p.T_ref);
      putg(2, 0, 0, g[n][2] + (up - g[n][2]) * ircv);
    } else {
      const real gold = L.m1.g[3][my - 1][mx];
      putg(4, 0, -1, gold + (gs_[4] - gold) * L.m1.irc[my - 1][mx]);
    }
  }
  __syncthreads();  // state complete; the fields of the first step are dead (m2 aliases them)
}

// ------------------------------------------------------------------------- kernels

// Position (bx, by) of tile number `tile` of an instance with ntx x nty tiles.  Tiles are numbered
// in strips of `strip` tile columns, each strip from the bottom row to the top, row by row within it
// (strip >= ntx: whole grid rows in order).  Workgroups take the tiles in this order, each XCD a
// contiguous range of it.  With strips narrower than the grid, the tiles below and above a tile,
// whose rows it reads as halo, are processed shortly before and after it on the same XCD, and its
// halo reads hit that XCD's L2; with whole rows in order they are a grid row of tiles away, which on
// grids beyond the Infinity Cache is too far for the L2 to keep them.
template <typename real>
__device__ __forceinline__ void tile_position(int tile, const InstDesc<real>& D, int& bx, int& by) {
  const int strip = D.strip;
  const int s = (int)fast_div((unsigned)tile, D.div_band);  // tile / (strip * nty)
  const int local = tile - s * strip * D.nty;
  const bool last = D.ntx - s * strip < strip;  // the last strip may be narrower
  const int w = last ? D.ntx - s * strip : strip;
  by = (int)fast_div((unsigned)local, last ? D.div_last : D.div_strip);
  bx = s * strip + (local - by * w);
}

// LDS of one workgroup of shape S: the two-step state, or the one-step fields
template <typename real, class S, int QG>
using TileLds = typename std::conditional<S::DEPTH == 2, Step2Lds<real, S>, StepLds<real, S::EYW, QG>>::type;

// One tile of one launch: tile bid of the launch's tile range at step t (the launch does S::DEPTH
// steps, one where only one is left in the instance's window).  Each launch swaps the A/B buffers
// once, so the source buffer is B exactly when b_base plus the number of launches since t_base is
// odd.  Returns at once for a tile outside every active instance or outside its window (uniform per
// workgroup).
template <typename real, class S, int QG>
__device__ __forceinline__ void step_tile(const InstDesc<real>* __restrict__ table, int ninst, long long t,
                                          const LaunchWin& w, int bid, TileLds<real, S, QG>& lds, int tid) {
  int lo = 0, hi = ninst - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (table[mid].tile_begin <= bid) lo = mid;
    else hi = mid - 1;
  }
  const InstDesc<real>& D = table[lo];
  // step window: from the arguments (single runs launched directly) or from the descriptor
  const long long t_base = w.use ? w.t_base : D.t_base, t_end = w.use ? w.t_end : D.t_end;
  const int b_base = w.use ? w.b_base : D.b_base, h_base = w.use ? w.h_base : D.h_base;
  if (t < t_base || t >= t_end) return;
  const int tile = bid - D.tile_begin;
  if (tile < 0 || tile >= D.ntx * D.nty) return;
  int bx, by;
  tile_position(tile, D, bx, by);
  const int x0 = bx * TX, y0 = by * S::TY;
  const bool odd = ((b_base + (t - t_base) / S::DEPTH) & 1) != 0;
  // the history changes copy once per launch that does two steps (every launch of a two-step
  // shape in the window but possibly the last, which does one step in place)
  const bool hodd = ((h_base + (S::DEPTH == 2 ? (t - t_base) / 2 : 0)) & 1) != 0;
  unsigned err = 0u;
  // interior: the load region lies inside the grid, so no wrap, ghost row, wall or Dirichlet
  // edge is involved
  const bool interior = x0 >= HXW && x0 + TX + HXW <= D.nx && y0 >= HYW && y0 + S::TY + HYW <= D.ny;
  const int gv = general_variant(D.p.thermal_box, D.p.y_walls);
  const LdsState<real, S> none{};
  if constexpr (S::DEPTH == 2) {
    Step2Lds<real, S>& L2 = lds;
    if (t_end - t >= 2) {
      real Tn1[S::RPT], Tn2[S::RPT];
      const bool interior2 =
          x0 >= S::MXH && x0 + TX + S::MXH <= D.nx && y0 >= S::MYH && y0 + S::TY + S::MYH <= D.ny;
      if (interior2) first_step<real, S, 0>(D, L2, odd, hodd, x0, y0, Tn1, Tn2, err, tid);
      else with_general_variant(gv, [&](auto v) { first_step<real, S, decltype(v)::value>(D, L2, odd, hodd, x0, y0, Tn1, Tn2, err, tid); });
      const LdsState<real, S> st{L2.sf, L2.sg, Tn1, Tn2};
      if (interior) step_body<real, S, 0, true>(D, L2.m2, odd, hodd, x0, y0, st, err, tid);
      else with_general_variant(gv, [&](auto v) { step_body<real, S, decltype(v)::value, true>(D, L2.m2, odd, hodd, x0, y0, st, err, tid); });
    } else {
      if (interior) step_body<real, S, 0, false>(D, L2.m2, odd, hodd, x0, y0, none, err, tid);
      else with_general_variant(gv, [&](auto v) { step_body<real, S, decltype(v)::value, false>(D, L2.m2, odd, hodd, x0, y0, none, err, tid); });
    }
  } else {
    StepLds<real, S::EYW, QG>& L = lds;
    if (interior) step_body<real, S, 0, false, QG>(D, L, odd, hodd, x0, y0, none, err, tid);
    else with_general_variant(gv, [&](auto v) { step_body<real, S, decltype(v)::value, false, QG>(D, L, odd, hodd, x0, y0, none, err, tid); });
  }
  // A failing simulation flags every node.  One atomic per thread, or even per wavefront, on one
  // word would serialise the launch, so a wavefront ORs its flags with ballots and sets only the
  // bits the word does not hold yet.
  const unsigned long long e1 = __ballot((err & ERR_RHO) != 0u), e2 = __ballot((err & ERR_T) != 0u),
                           e4 = __ballot((err & ERR_PSI) != 0u);
  if ((e1 | e2 | e4) != 0ull && (threadIdx.x & 63u) == 0u) {
    const unsigned bits = (e1 ? ERR_RHO : 0u) | (e2 ? ERR_T : 0u) | (e4 ? ERR_PSI : 0u);
    const unsigned held = __hip_atomic_load(D.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if ((held & bits) != bits) atomicOr(D.err, bits);
  }
}

// One workgroup per tile.  A launch of shape S advances every active instance by S::DEPTH steps
// (one step if only one is left in its budget).  The device clock counts steps; launch k of a group
// does step t = clock + k DEPTH (or w.t + k DEPTH with the window in the arguments).
template <typename real, class S, int QG>
__global__ __launch_bounds__(S::NT) void step_kernel(const InstDesc<real>* __restrict__ table, int ninst,
                                                     const long long* __restrict__ clock, int k, LaunchWin w) {
  static_assert(QG == 5 || (QG == 9 && S::DEPTH == 1), "D2Q9 thermal populations: one step per launch");
  // ---- which tile (uniform per workgroup).  Workgroups are dispatched to the 8 XCDs round-robin;
  // remap so that each XCD takes a contiguous range of tiles: neighbouring tiles then share one L2,
  // where their halo reads hit and where the partial cache lines of the shifted (pushed) stores of
  // two neighbours are merged before they are written back.
  const int nwg = gridDim.x;
  const int xcd = blockIdx.x % NXCD;
  const int per = nwg / NXCD, rem = nwg % NXCD;
  const int bid = xcd * per + (xcd < rem ? xcd : rem) + blockIdx.x / NXCD;
  const long long t = (w.use ? w.t : *clock) + (long long)k * S::DEPTH;
  __shared__ TileLds<real, S, QG> lds;
  step_tile<real, S, QG>(table, ninst, t, w, bid, lds, (int)threadIdx.x);
}

// Tile shapes compiled into the library, per precision: (tile height, wavefronts, steps per
// launch).  Index 0 is the shape for small grids, index 1 the one for grids of many tiles; the
// others are candidates for the autotuner.  All shapes give bit-identical results.  Two-step
// shapes need the grid to be larger than their wide halo region (lbm_shape_info reports it).
#define LBM_F32_SHAPES(X) \
  X(0, 16, 16, 1) X(1, 16, 8, 1) X(2, 8, 8, 1) X(3, 32, 16, 1) X(4, 8, 4, 1) X(5, 4, 4, 1) X(6, 16, 16, 2) X(7, 8, 8, 2)
#define LBM_F64_SHAPES(X) X(0, 16, 8, 1) X(1, 8, 8, 1) X(2, 16, 16, 1) X(3, 8, 4, 1) X(4, 4, 4, 1)

// Clock advance after a group of step launches (a kernel, so that it can live in a graph).
__global__ void clock_advance_kernel(long long* clock, long long n) {
  if (threadIdx.x == 0 && blockIdx.x == 0) clock[0] = clock[0] + n;
}

// Step window and device clock of a single run, set on its stream before the graph replays of an
// lbm_step call: steps [t_base, t_end) of the clock, starting from the B buffers if b_base is 1.
// (A kernel takes its arguments at enqueue, so no host buffer has to outlive the call.)
template <typename real>
__global__ void set_window_kernel(InstDesc<real>* d, long long* clock, long long t_base, int b_base, int h_base,
                                  long long t_end) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    d->t_base = t_base;
    d->b_base = b_base;
    d->h_base = h_base;
    d->t_end = t_end;
    clock[0] = t_base;
  }
}

// Open top boundary, after the step of launch k of a one-step shape: the populations that enter
// the top row N from outside (c_y = -1) follow the convective outflow condition
//   f_i(x, N, t+1) = [f_i(x, N, t) + U f_i(x, N-1, t+1)] / (1 + U),
// U = j_y / rho of the top node at time t clipped to [0, 1].  f(t) is in the step's source
// buffers, f(t+1) of row N-1 in its destination buffers.  The step kernel has left the outgoing
// populations of the top row (c_y = +1) in the slots of the entering ones; their sum, subtracted
// from that of the entering values, is the mass the domain gains through the top in this step,
// added to the instance's FP64 mass in a fixed order (per-thread column sums, then the lanes and
// wavefronts in a fixed tree), so rho_ave follows the mean density.  Workgroup b serves table
// entry b (entries without an open top, or outside their window, return at once); its threads
// stride over the columns.
constexpr int OPEN_NT = 256;

// The open-top pass for one table entry D after the step at t, by the first OPEN_NT threads of the
// workgroup (the others wait at its barriers), so that the order of its sums does not depend on
// the workgroup size.  part: OPEN_NT / 64 doubles of LDS.
template <typename real>
__device__ __forceinline__ void open_top_body(const InstDesc<real>& D, long long t, const LaunchWin& w,
                                              double* part) {
  if (!D.p.open_top) return;
  const long long t_base = w.use ? w.t_base : D.t_base, t_end = w.use ? w.t_end : D.t_end;
  const int b_base = w.use ? w.b_base : D.b_base;
  if (t < t_base || t >= t_end) return;
  const bool odd = ((b_base + (t - t_base)) & 1) != 0;
  const real* __restrict__ fs = odd ? D.fB : D.fA;
  real* __restrict__ fd = odd ? D.fA : D.fB;
  const size_t N = (size_t)D.nx * (size_t)D.ny;
  const bool active = threadIdx.x < (unsigned)OPEN_NT;
  double gain = 0.0;
  for (int x = (int)threadIdx.x; active && x < D.nx; x += OPEN_NT) {
    const size_t top = (size_t)(D.ny - 1) * (size_t)D.nx + (size_t)x, below = top - (size_t)D.nx;
    real f[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = fs[i * N + top];
    const real rho = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
    const real jy = (f[2] - f[4]) + ((f[5] + f[6]) - (f[7] + f[8]));
    real U = jy / rho;
    U = U < real(0) ? real(0) : (U > real(1) ? real(1) : U);
    const real out = (fd[4 * N + top] + fd[7 * N + top]) + fd[8 * N + top];
    const real n4 = (f[4] + U * fd[4 * N + below]) / (real(1) + U);
    const real n7 = (f[7] + U * fd[7 * N + below]) / (real(1) + U);
    const real n8 = (f[8] + U * fd[8 * N + below]) / (real(1) + U);
    fd[4 * N + top] = n4;
    fd[7 * N + top] = n7;
    fd[8 * N + top] = n8;
    gain += ((double)n4 + (double)n7 + (double)n8) - (double)out;
  }
  for (int s = 32; s > 0; s >>= 1) gain += __shfl_xor(gain, s, 64);
  if (active && (threadIdx.x & 63u) == 0u) part[threadIdx.x >> 6] = gain;
  __syncthreads();
  if (threadIdx.x == 0) {
    double total = 0.0;
    for (int v = 0; v < OPEN_NT / 64; ++v) total += part[v];
    const double m = D.live->mass + total;
    D.live->mass = m;
    D.live->rho_ave = m / (double)N;
  }
  __syncthreads();
}

// Open top boundary, after the step of launch k of a one-step shape: the populations that enter
// the top row N from outside (c_y = -1) follow the convective outflow condition
//   f_i(x, N, t+1) = [f_i(x, N, t) + U f_i(x, N-1, t+1)] / (1 + U),
// U = j_y / rho of the top node at time t clipped to [0, 1].  f(t) is in the step's source
// buffers, f(t+1) of row N-1 in its destination buffers.  The step kernel has left the outgoing
// populations of the top row (c_y = +1) in the slots of the entering ones; their sum, subtracted
// from that of the entering values, is the mass the domain gains through the top in this step,
// added to the instance's FP64 mass in a fixed order (per-thread column sums, then the lanes and
// wavefronts in a fixed tree), so rho_ave follows the mean density.  Workgroup b serves table
// entry b (entries without an open top, or outside their window, return at once); its threads
// stride over the columns.
template <typename real>
__global__ __launch_bounds__(OPEN_NT) void open_top_kernel(const InstDesc<real>* __restrict__ table,
                                                           const long long* __restrict__ clock, int k, LaunchWin w) {
  __shared__ double part[OPEN_NT / 64];
  const long long t = (w.use ? w.t : *clock) + k;
  open_top_body<real>(table[blockIdx.x], t, w, part);
}

}  // namespace lbm
