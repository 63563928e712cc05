// The fused time step: one workgroup per TX x TY tile of one simulation.
//
// Phases (each separated by a workgroup barrier; the arithmetic of a node never depends on
// where its tile lies, so a node's result is the same in a single run and in a batch):
//   1  load f and g of the tile plus a halo (HXW columns, HYW rows); per node rho, j, T
//      (Eqs. 11, 25) and psi (Eq. 10 and the text after Eq. 9) into LDS; own nodes keep f, g
//      in registers.  Wall tiles then fill the ghost rows with the wetting density of Eq. (54)
//      at the wall temperature.
//   2  on the tile plus one halo node: interaction force (Eq. 9), buoyancy, velocity (Eq. 11).
//   3  own nodes: div u (isotropic stencil, mirrored ghost velocity at walls), grad T from the
//      D2Q5 non-equilibrium moments (Eqs. 49-50), Q (Eq. 20), S (Eq. 24, backward second
//      difference of T), MRT collision of f with Li's forcing (Eqs. 5, 7, 8), MRT collision of
//      g (Eq. 39), push-streaming of f (Eq. 6, halfway bounce-back at walls) and of g with the
//      rho c_v-weighted blend at the destination (Eq. 39; anti-bounce-back at Dirichlet edges).
#pragma once
#include "lbm_device.hpp"

namespace lbm {

template <typename real>
struct StepLds {
  real rho[EYW][EXW];
  real psi[EYW][EXW];
  real ux[EYW][EXW];  // holds j_x after phase 1, u_x after phase 2
  real uy[EYW][EXW];
  real g[4][EYW][EXW];  // pre-collision g_1..g_4 (needed at the streaming destination)
};

// position of halo cell r of the load region (ring around the TX x TY interior)
__device__ __forceinline__ void ring_cell(int r, int& ex, int& ey) {
  if (r < 2 * EXW) {
    ey = r / EXW;
    ex = r - ey * EXW;
  } else if (r < 4 * EXW) {
    const int q = r - 2 * EXW;
    ey = EYW - 2 + q / EXW;
    ex = q % EXW;
  } else {
    const int q = r - 4 * EXW;
    ey = HYW + q / (2 * HXW);
    const int c = q % (2 * HXW);
    ex = c < HXW ? c : TX + HXW + (c - HXW);
  }
}

// position of halo cell r of the velocity region (one node around the interior)
__device__ __forceinline__ void uring_cell(int r, int& ex, int& ey) {
  if (r < 2 * (TX + 2)) {
    const int side = r / (TX + 2);
    ey = side ? EYW - HYW : HYW - 1;
    ex = HXW - 1 + (r - side * (TX + 2));
  } else {
    const int q = r - 2 * (TX + 2);
    ey = HYW + q / 2;
    ex = (q & 1) ? HXW + TX : HXW - 1;
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

template <typename real>
__device__ __forceinline__ void load_node(const real* __restrict__ fs, const real* __restrict__ gs, size_t N, int o,
                                          real (&f)[9], real (&g)[5]) {
#pragma unroll
  for (int i = 0; i < 9; ++i) f[i] = fs[i * N + o];
#pragma unroll
  for (int i = 0; i < 5; ++i) g[i] = gs[i * N + o];
}

// rho, j, T of a node and its LDS entries (Eqs. 11 and 25), psi with error checks
template <typename real>
__device__ __forceinline__ void node_macro_to_lds(StepLds<real>& L, int ex, int ey, const DevParams<real>& p,
                                                  const real (&f)[9], const real (&g)[5], unsigned& err) {
  const real rho = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
  const real jx = (f[1] - f[3]) + ((f[5] - f[6]) + (f[8] - f[7]));
  const real jy = (f[2] - f[4]) + ((f[5] + f[6]) - (f[7] + f[8]));
  const real T = p.T_ref + (((g[0] + g[1]) + (g[2] + g[3])) + g[4]);
  real psi = real(0);
  if (!(rho > real(0)) || !isfinite(rho)) err |= ERR_RHO;
  else if (!(T > real(0)) || !isfinite(T)) err |= ERR_T;
  else psi = pseudo(p, rho, T, err);
  L.rho[ey][ex] = rho;
  L.psi[ey][ex] = psi;
  L.ux[ey][ex] = jx;
  L.uy[ey][ex] = jy;
  L.g[0][ey][ex] = g[1];
  L.g[1][ey][ex] = g[2];
  L.g[2][ey][ex] = g[3];
  L.g[3][ey][ex] = g[4];
}

template <typename real>
__device__ __forceinline__ void zero_lds_cell(StepLds<real>& L, int ex, int ey) {
  L.rho[ey][ex] = real(0);
  L.psi[ey][ex] = real(0);
  L.ux[ey][ex] = real(0);
  L.uy[ey][ex] = real(0);
#pragma unroll
  for (int k = 0; k < 4; ++k) L.g[k][ey][ex] = real(0);
}

// Interaction force F_m = -G psi(x) sum_i varpi_i psi(x + c_i) c_i (Eq. 9), varpi = 1/3, 1/12
template <typename real>
__device__ __forceinline__ void interaction_force(const StepLds<real>& L, int ex, int ey, real G, real& fx, real& fy) {
  const real pE = L.psi[ey][ex + 1], pN = L.psi[ey + 1][ex], pW = L.psi[ey][ex - 1], pS = L.psi[ey - 1][ex];
  const real pNE = L.psi[ey + 1][ex + 1], pNW = L.psi[ey + 1][ex - 1], pSW = L.psi[ey - 1][ex - 1],
             pSE = L.psi[ey - 1][ex + 1];
  const real sx = real(1.0 / 3.0) * (pE - pW) + real(1.0 / 12.0) * ((pNE - pNW) + (pSE - pSW));
  const real sy = real(1.0 / 3.0) * (pN - pS) + real(1.0 / 12.0) * ((pNE + pNW) - (pSE + pSW));
  const real c = -G * L.psi[ey][ex];
  fx = c * sx;
  fy = c * sy;
}

template <typename real>
__global__ __launch_bounds__(NT) void step_kernel(const InstDesc<real>* __restrict__ table, int ninst,
                                                  const long long* __restrict__ clock, int k) {
  // ---- which simulation and which tile (uniform per workgroup)
  const int bid = blockIdx.x;
  int lo = 0, hi = ninst - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (table[mid].tile_begin <= bid) lo = mid;
    else hi = mid - 1;
  }
  const InstDesc<real>& D = table[lo];
  const long long t = *clock + k;
  if (t < D.t_start || t >= D.t_end) return;
  const int tile = bid - D.tile_begin;
  if (tile < 0 || tile >= D.ntx * D.nty) return;
  const int by = tile / D.ntx;
  const int bx = tile - by * D.ntx;
  const int x0 = bx * TX, y0 = by * TY;
  const int nx = D.nx, ny = D.ny;
  const size_t N = (size_t)nx * (size_t)ny;
  const bool odd = ((t - D.t_start) & 1) != 0;
  const real* __restrict__ fs = odd ? D.fB : D.fA;
  const real* __restrict__ gs = odd ? D.gB : D.gA;
  real* __restrict__ fd = odd ? D.fA : D.fB;
  real* __restrict__ gd = odd ? D.gA : D.gB;
  real* __restrict__ Th = D.Th;
  const DevParams<real> p = D.p;
  const int walls = p.y_walls;
  const bool freeze = (p.flags & FL_FREEZE_FLOW) != 0;

  __shared__ StepLds<real> L;
  const int tid = threadIdx.x;
  const int tx = tid & (TX - 1);
  const int ty = tid >> 6;
  unsigned err = 0u;

  // ---- phase 1: own nodes (kept in registers) and the halo ring
  const int xg = x0 + tx;
  const int xw = wrapi(xg, nx);
  real f[RPT][9], g[RPT][5];
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int ey = HYW + ty + 4 * r;
    const int yg = y0 + ty + 4 * r;
    if (row_kind(yg, ny, walls) == 0) {
      const int yw = walls ? yg : wrapi(yg, ny);
      load_node(fs, gs, N, yw * nx + xw, f[r], g[r]);
      node_macro_to_lds(L, HXW + tx, ey, p, f[r], g[r], err);
    } else {
#pragma unroll
      for (int i = 0; i < 9; ++i) f[r][i] = real(0);
#pragma unroll
      for (int i = 0; i < 5; ++i) g[r][i] = real(0);
      zero_lds_cell(L, HXW + tx, ey);
    }
  }
  for (int r = tid; r < RING; r += NT) {
    int ex, ey;
    ring_cell(r, ex, ey);
    const int yg = y0 - HYW + ey;
    if (row_kind(yg, ny, walls) == 0) {
      const int yw = walls ? yg : wrapi(yg, ny);
      const int xr = wrapi(x0 - HXW + ex, nx);
      real fr[9], gr[5];
      load_node(fs, gs, N, yw * nx + xr, fr, gr);
      node_macro_to_lds(L, ex, ey, p, fr, gr, err);
    } else {
      zero_lds_cell(L, ex, ey);
    }
  }
  __syncthreads();

  // ---- phase 1b: wetting ghost rows, rho_0 = rho_2 + tan(pi/2 - theta) |rho_{x+1,1} - rho_{x-1,1}|
  if (walls) {
    const int eyb = -1 - (y0 - HYW);  // LDS row of y = -1
    const int eyt = ny - (y0 - HYW);  // LDS row of y = ny
    const bool hasb = eyb >= 0 && eyb < EYW, hast = eyt >= 0 && eyt < EYW;
    if (hasb || hast) {
      for (int c = tid; c < 2 * EXW; c += NT) {
        const int top = c >= EXW;
        const int ex = c - top * EXW;
        const int ey = top ? eyt : eyb;
        if ((top ? hast : hasb) && ex >= 1 && ex <= EXW - 2) {
          const int d = top ? -1 : 1;  // towards the fluid
          const real tanv = top ? p.tan_top : p.tan_bot;
          const real rg = L.rho[ey + 2 * d][ex] + tanv * fabs(L.rho[ey + d][ex + 1] - L.rho[ey + d][ex - 1]);
          const real Tw = wall_temperature(p, top, wrapi(x0 - HXW + ex, nx));
          L.psi[ey][ex] = pseudo(p, rg, Tw, err);
        }
      }
      __syncthreads();
    }
  }

  // ---- phase 2: forces and velocity on the tile plus one node
  real Fx[RPT], Fy[RPT], Fm2[RPT];
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int ex = HXW + tx, ey = HYW + ty + 4 * r;
    const int yg = y0 + ty + 4 * r;
    Fx[r] = Fy[r] = Fm2[r] = real(0);
    if (row_kind(yg, ny, walls) == 0) {
      const real rho = L.rho[ey][ex];
      real fx = real(0), fy = real(0), fmx = real(0), fmy = real(0);
      if (!freeze) {
        interaction_force(L, ex, ey, p.G, fmx, fmy);
        fx = fmx + (rho - p.rho_ave) * p.gx;
        fy = fmy + (rho - p.rho_ave) * p.gy;
      }
      Fx[r] = fx;
      Fy[r] = fy;
      Fm2[r] = fmx * fmx + fmy * fmy;
      const real ir = real(1) / rho;
      L.ux[ey][ex] = (L.ux[ey][ex] + real(0.5) * fx) * ir;
      L.uy[ey][ex] = (L.uy[ey][ex] + real(0.5) * fy) * ir;
    }
  }
  for (int r = tid; r < URING; r += NT) {
    int ex, ey;
    uring_cell(r, ex, ey);
    const int yg = y0 - HYW + ey;
    if (row_kind(yg, ny, walls) == 0) {
      const real rho = L.rho[ey][ex];
      real fx = real(0), fy = real(0);
      if (!freeze) {
        real fmx, fmy;
        interaction_force(L, ex, ey, p.G, fmx, fmy);
        fx = fmx + (rho - p.rho_ave) * p.gx;
        fy = fmy + (rho - p.rho_ave) * p.gy;
      }
      const real ir = real(1) / rho;
      L.ux[ey][ex] = (L.ux[ey][ex] + real(0.5) * fx) * ir;
      L.uy[ey][ex] = (L.uy[ey][ex] + real(0.5) * fy) * ir;
    }
  }
  __syncthreads();

  // ---- phase 3: collision and streaming of the own nodes
  const real cv = p.cv;
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int ex = HXW + tx, ey = HYW + ty + 4 * r;
    const int yg = y0 + ty + 4 * r;
    if (xg >= nx || yg >= ny) continue;
    const real rho = L.rho[ey][ex];
    const real ux = L.ux[ey][ex], uy = L.uy[ey][ex];
    const real Tr = ((g[r][0] + g[r][1]) + (g[r][2] + g[r][3])) + g[r][4];  // T - T_ref
    const real T = p.T_ref + Tr;
    const int o = yg * nx + xw;

    // div u = 3 sum_i w_i c_i . u(x + c_i); a ghost row carries -u of the fluid row next to it
    real uxn[9], uyn[9];
#pragma unroll
    for (int i = 1; i < 9; ++i) {
      const int cx = (i == 1 || i == 5 || i == 8) ? 1 : ((i == 3 || i == 6 || i == 7) ? -1 : 0);
      const int cy = (i == 2 || i == 5 || i == 6) ? 1 : ((i == 4 || i == 7 || i == 8) ? -1 : 0);
      const bool ghost = walls && ((yg == 0 && cy < 0) || (yg == ny - 1 && cy > 0));
      if (ghost) {
        uxn[i] = -L.ux[ey][ex + cx];
        uyn[i] = -L.uy[ey][ex + cx];
      } else {
        uxn[i] = L.ux[ey + cy][ex + cx];
        uyn[i] = L.uy[ey + cy][ex + cx];
      }
    }
    const real divu = real(1.0 / 3.0) * ((uxn[1] - uxn[3]) + (uyn[2] - uyn[4])) +
                      real(1.0 / 12.0) * (((uxn[5] - uxn[7]) + (uxn[8] - uxn[6])) + ((uyn[5] - uyn[7]) + (uyn[6] - uyn[8])));

    // grad T from m_1, m_2 of the D2Q5 populations (Eqs. 49-50)
    const real dTx = -p.vs1 * (g[r][1] - g[r][3]) * p.inv_cs2h;
    const real dTy = -p.vs1 * (g[r][2] - g[r][4]) * p.inv_cs2h;
    real press, dpdT;
    pr_eos(p, rho, T, press, dpdT);
    const real rcv = rho * cv;
    const real Q = -(rcv * (ux * dTx + uy * dTy) + T * dpdT * divu);
    const real T1 = Th[o];
    const real T2 = Th[N + o];
    const real Ssum = (p.flags & FL_NO_S) ? real(0) : rcv * real(0.5) * ((Tr - T1) - (T1 - T2));
    Th[o] = Tr;
    Th[N + o] = T1;

    // ---- D2Q9 MRT collision with Li's forcing, moments of the orthogonal basis of Eq. (4)
    real fs_[9];
    if (freeze) {
#pragma unroll
      for (int i = 0; i < 9; ++i) fs_[i] = f[r][i];
    } else {
      const real* fi = f[r];
      const real sa = (fi[1] + fi[2]) + (fi[3] + fi[4]);
      const real sd = (fi[5] + fi[6]) + (fi[7] + fi[8]);
      real m1 = -real(4) * fi[0] - sa + real(2) * sd;
      real m2 = real(4) * fi[0] - real(2) * sa + sd;
      const real jx = (fi[1] - fi[3]) + ((fi[5] - fi[6]) + (fi[8] - fi[7]));
      const real jy = (fi[2] - fi[4]) + ((fi[5] + fi[6]) - (fi[7] + fi[8]));
      real m4 = real(-2) * (fi[1] - fi[3]) + ((fi[5] - fi[6]) + (fi[8] - fi[7]));
      real m6 = real(-2) * (fi[2] - fi[4]) + ((fi[5] + fi[6]) - (fi[7] + fi[8]));
      real m7 = (fi[1] - fi[2]) + (fi[3] - fi[4]);
      real m8 = (fi[5] - fi[6]) + (fi[7] - fi[8]);
      const real uu = ux * ux + uy * uy;
      const real fx = Fx[r], fy = Fy[r];
      const real uF = ux * fx + uy * fy;
      const real corr = Fm2[r] / (L.psi[ey][ex] * L.psi[ey][ex]);
      const real F1 = real(6) * uF + p.corr_e * corr;
      const real F2 = -real(6) * uF - p.corr_eps * corr;
      const real F7 = real(2) * (ux * fx - uy * fy);
      const real F8 = ux * fy + uy * fx;
      // m* = m - S (m - m_eq) + (1 - S/2) F  (Eq. 5), m_eq of Eq. (7)
      m1 = m1 - p.s_e * (m1 - rho * (real(-2) + real(3) * uu)) + (real(1) - real(0.5) * p.s_e) * F1;
      m2 = m2 - p.s_eps * (m2 - rho * (real(1) - real(3) * uu)) + (real(1) - real(0.5) * p.s_eps) * F2;
      const real m3 = jx + fx;  // conserved moment: jx - s_j (jx - rho ux) + (1 - s_j/2) Fx = jx + Fx
      m4 = m4 - p.s_q * (m4 + rho * ux) + (real(1) - real(0.5) * p.s_q) * (-fx);
      const real m5 = jy + fy;
      m6 = m6 - p.s_q * (m6 + rho * uy) + (real(1) - real(0.5) * p.s_q) * (-fy);
      m7 = m7 - p.s_p * (m7 - rho * (ux * ux - uy * uy)) + (real(1) - real(0.5) * p.s_p) * F7;
      m8 = m8 - p.s_p * (m8 - rho * ux * uy) + (real(1) - real(0.5) * p.s_p) * F8;
      // f* = M^-1 m* with M^-1 = M^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4)
      const real a0 = rho * real(1.0 / 9.0);
      const real b1 = m1 * real(1.0 / 36.0), b2 = m2 * real(1.0 / 36.0);
      const real c3 = m3 * real(1.0 / 6.0), c4 = m4 * real(1.0 / 12.0);
      const real c5 = m5 * real(1.0 / 6.0), c6 = m6 * real(1.0 / 12.0);
      const real d7 = m7 * real(0.25), d8 = m8 * real(0.25);
      const real axis = a0 - b1 - real(2) * b2;
      const real diag = a0 + real(2) * b1 + b2;
      fs_[0] = a0 - real(4) * b1 + real(4) * b2;
      fs_[1] = axis + (c3 - real(2) * c4) + d7;
      fs_[2] = axis + (c5 - real(2) * c6) - d7;
      fs_[3] = axis - (c3 - real(2) * c4) + d7;
      fs_[4] = axis - (c5 - real(2) * c6) - d7;
      fs_[5] = diag + (c3 + c4) + (c5 + c6) + d8;
      fs_[6] = diag - (c3 + c4) + (c5 + c6) - d8;
      fs_[7] = diag - (c3 + c4) - (c5 + c6) + d8;
      fs_[8] = diag + (c3 + c4) - (c5 + c6) - d8;
    }

    // ---- D2Q5 MRT collision (Eq. 39) with the non-orthogonal basis of Eq. (40)
    real gs_[5];
    {
      const real* gi = g[r];
      const real dm1 = p.vs1 * (gi[1] - gi[3]);
      const real dm2 = p.vs1 * (gi[2] - gi[4]);
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

    // ---- streaming of f: push to x + c_i, halfway bounce-back through the walls
    {
      const int xe = wrapi(xg + 1, nx), xwst = wrapi(xg - 1, nx);
      const bool wall_n = walls && yg == ny - 1, wall_s = walls && yg == 0;
      const int yn = walls ? yg + 1 : wrapi(yg + 1, ny);
      const int ys = walls ? yg - 1 : wrapi(yg - 1, ny);
      real* fd0 = fd;
      if (freeze) {
#pragma unroll
        for (int i = 0; i < 9; ++i) fd0[i * N + o] = fs_[i];
      } else {
        fd0[o] = fs_[0];
        fd0[1 * N + yg * nx + xe] = fs_[1];
        fd0[3 * N + yg * nx + xwst] = fs_[3];
        if (wall_n) {
          fd0[4 * N + o] = fs_[2];
          fd0[7 * N + o] = fs_[5];
          fd0[8 * N + o] = fs_[6];
        } else {
          fd0[2 * N + yn * nx + xw] = fs_[2];
          fd0[5 * N + yn * nx + xe] = fs_[5];
          fd0[6 * N + yn * nx + xwst] = fs_[6];
        }
        if (wall_s) {
          fd0[2 * N + o] = fs_[4];
          fd0[5 * N + o] = fs_[7];
          fd0[6 * N + o] = fs_[8];
        } else {
          fd0[4 * N + ys * nx + xw] = fs_[4];
          fd0[7 * N + ys * nx + xwst] = fs_[7];
          fd0[8 * N + ys * nx + xe] = fs_[8];
        }
      }
    }

    // ---- streaming of g with the modified collision of Eq. (39):
    //      g_i(y, t+1) = g_i(y, t) + [g*_i(y - c_i) - g_i(y, t)] / (rho(y, t) c_v)
    {
      const real ircv = real(1) / rcv;
      gd[o] = g[r][0] + (gs_[0] - g[r][0]) * ircv;
      const int hxs[5] = {0, 1, 0, -1, 0};
      const int hys[5] = {0, 0, 1, 0, -1};
#pragma unroll
      for (int i = 1; i < 5; ++i) {
        const int xd = xg + hxs[i], yd = yg + hys[i];
        const bool out_y = (walls || p.thermal_box) && (yd < 0 || yd >= ny);
        const bool out_x = p.thermal_box && (xd < 0 || xd >= nx);
        const int io = i <= 2 ? i + 2 : i - 2;  // opposite direction
        if (out_x || out_y) {
          // anti-bounce-back: the population entering this node in direction io
          const real Tw = p.thermal_box ? p.T_box : wall_temperature(p, yd < 0 ? 0 : 1, xw);
          const real up = -gs_[i] + real(2) * p.w1h * (Tw - p.T_ref);
          const real gold = g[r][io];
          gd[io * N + o] = gold + (up - gold) * ircv;
        } else {
          const int exd = ex + hxs[i], eyd = ey + hys[i];
          const real gold = L.g[i - 1][eyd][exd];
          const real rd = L.rho[eyd][exd] * cv;
          const int od = (walls ? yd : wrapi(yd, ny)) * nx + wrapi(xd, nx);
          gd[i * N + od] = gold + (gs_[i] - gold) / rd;
        }
      }
    }
  }

  if (err) atomicOr(D.err, err);
}

// Clock advance after a group of step launches (a kernel, so that it can live in a graph).
__global__ void clock_advance_kernel(long long* clock, long long n) {
  if (threadIdx.x == 0 && blockIdx.x == 0) clock[0] = clock[0] + n;
}

}  // namespace lbm
