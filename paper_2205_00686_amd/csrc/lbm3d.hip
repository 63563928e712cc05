// Three-dimensional extension: D3Q19 MRT pseudopotential flow coupled to the paper's temperature
// model on D3Q7 (include/lbm3d.h states the model).  The arithmetic of one node is split into
// three device functions:
//   fields: rho, j, T (Eqs. 11, 25), p and psi (Eq. 10 and the text after Eq. 9), (dp/dT)_rho,
//     1/(rho c_v);
//   force: the interaction force (Eq. 9, D3Q19 weights) and the velocity (Eq. 11);
//   collisions: div u, grad T (Eqs. 49-50), Q (Eq. 20), S (Eq. 24), the D3Q19 MRT collision with
//     Li's forcing (Eqs. 5, 7, 8), the D3Q7 MRT collision (Eq. 39), then the push of f and of g
//     with the rho c_v blend at the destination (Eq. 39), anti-bounce-back at Dirichlet faces and
//     the temperature history.
// Two step paths call them:
//   fused (default): one kernel per step.  A workgroup owns a 64 x TY column tile and marches
//     through a chunk of z planes, keeping psi, u and the values needed at the streaming
//     destinations of the last planes in LDS rings; every population is read and written once.
//   per-node: three kernels per step with the per-node fields in HBM planes between them (kept as
//     the simple reference of the fused path, and used to produce output fields).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <new>
#include <string>

#include "lbm3d.h"
#include "lbm_device.hpp"
#include "host_range.hpp"

namespace lbm3 {
using lbm::DevParams;
using lbm::ERR_PSI;
using lbm::ERR_RHO;
using lbm::ERR_T;

constexpr size_t ALIGN3 = 256;
constexpr size_t CTRL3 = 16 * 1024;     // error word and diagnostics
constexpr size_t PART3 = 32 * 1024;     // reduction partials
constexpr int RED3 = 256;
constexpr int MAXB3 = (int)(PART3 / (2 * sizeof(double)));
constexpr int NSCR = 15;                // per-node field planes
enum { S_RHO, S_PSI, S_JX, S_JY, S_JZ, S_TR, S_DPDT, S_IRC, S_UX, S_UY, S_UZ, S_FX, S_FY, S_FZ, S_S2 };

// D3Q19 velocities: rest, the six axes, the twelve face diagonals
__host__ __device__ constexpr int cx19(int i) {
  constexpr int v[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
  return v[i];
}
__host__ __device__ constexpr int cy19(int i) {
  constexpr int v[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
  return v[i];
}
__host__ __device__ constexpr int cz19(int i) {
  constexpr int v[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
  return v[i];
}
__host__ __device__ constexpr int c2_19(int i) { return cx19(i) * cx19(i) + cy19(i) * cy19(i) + cz19(i) * cz19(i); }
// lattice weights as (numerator over 36)
__host__ __device__ constexpr int w36(int i) { return c2_19(i) == 0 ? 12 : (c2_19(i) == 1 ? 2 : 1); }

// Row k of d'Humieres' orthogonal moment basis evaluated at velocity i (integers)
__host__ __device__ constexpr int mrow(int k, int i) {
  const int x = cx19(i), y = cy19(i), z = cz19(i), c2 = c2_19(i);
  switch (k) {
    case 0: return 1;
    case 1: return 19 * c2 - 30;
    case 2: return (21 * c2 * c2 - 53 * c2 + 24) / 2;
    case 3: return x;
    case 4: return (5 * c2 - 9) * x;
    case 5: return y;
    case 6: return (5 * c2 - 9) * y;
    case 7: return z;
    case 8: return (5 * c2 - 9) * z;
    case 9: return 3 * x * x - c2;
    case 10: return (3 * c2 - 5) * (3 * x * x - c2);
    case 11: return y * y - z * z;
    case 12: return (3 * c2 - 5) * (y * y - z * z);
    case 13: return x * y;
    case 14: return y * z;
    case 15: return x * z;
    case 16: return (y * y - z * z) * x;
    case 17: return (z * z - x * x) * y;
    default: return (x * x - y * y) * z;
  }
}
__host__ __device__ constexpr int mnorm(int k) {
  int s = 0;
  for (int i = 0; i < 19; ++i) s += mrow(k, i) * mrow(k, i);
  return s;
}

// Constants of one simulation in the working precision (derived on the host).
template <typename real>
struct Dev3 {
  DevParams<real> e;           // EOS fields used by pr_eos / psi_from_pressure
  real G, GG, cv, T_ref;
  real s_e, s_eps, s_v;        // MRT rates of the energy rows and of the five stress rows (all others 1)
  real om_e, om_eps, om_v;     // 1 - s/2
  real sig_e, sig_eps;         // (19/2) sigma / (1/s_e - 1/2), -(11/4) sigma / (1/s_eps - 1/2)
  real w0, w1, vs1, vs3, wdot, inv_cs2h, two_w1, T_box;
  int nx, ny, nz, thermal_box;
  unsigned flags;
};

template <typename real>
struct Bufs3 {
  const real* fs;  // source populations
  const real* gs;
  real* fd;        // destination populations
  real* gd;
  real* Th;        // T(t-1) - T_ref, T(t-2) - T_ref
  real* sc;        // per-node field planes
  unsigned* err;
};

__device__ __forceinline__ int wrap1(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

template <typename real>
__device__ __forceinline__ real sum19(const real (&f)[19]) {
  return (((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7]))) +
         (((f[8] + f[9]) + (f[10] + f[11])) + ((f[12] + f[13]) + (f[14] + f[15]))) + ((f[16] + f[17]) + f[18]);
}
template <typename real>
__device__ __forceinline__ real sum7(const real (&g)[7]) {
  return ((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + g[6]);
}

// ---- per-node arithmetic shared by both step paths

// rho, j (Eq. 11 without the force), T - T_ref (Eq. 25), psi (Eq. 10 and the text after Eq. 9),
// (dp/dT)_rho and 1/(rho c_v) of one node; flags an invalid state in err
template <typename real>
__device__ __forceinline__ void node_fields3(const Dev3<real>& p, const real (&f)[19], const real (&g)[7], real& rho,
                                             real& jx, real& jy, real& jz, real& Tr, real& psi, real& dpdT, real& irc,
                                             unsigned& err) {
  rho = sum19(f);
  jx = real(0);
  jy = real(0);
  jz = real(0);
#pragma unroll
  for (int i = 1; i < 19; ++i) {
    if (cx19(i)) jx += cx19(i) > 0 ? f[i] : -f[i];
    if (cy19(i)) jy += cy19(i) > 0 ? f[i] : -f[i];
    if (cz19(i)) jz += cz19(i) > 0 ? f[i] : -f[i];
  }
  Tr = sum7(g);
  const real T = p.T_ref + Tr;
  psi = real(0);
  dpdT = real(0);
  if (!(rho > real(0)) || !isfinite(rho)) {
    err |= ERR_RHO;
  } else if (!(T > real(0)) || !isfinite(T)) {
    err |= ERR_T;
  } else {
    real press;
    lbm::pr_eos(p.e, rho, T, press, dpdT);
    psi = lbm::psi_from_pressure(p.e, rho, press, err);
  }
  irc = lbm::rcp(rho * p.cv);
}

// Interaction force F = -G psi sum_i w_i psi(x + c_i) c_i (Eq. 9) from the neighbour sum
// (sx, sy, sz), the G^2 |sum|^2 that the sigma term of Eq. (8) uses, and u = (j + F/2) / rho
template <typename real>
__device__ __forceinline__ void node_force3(const Dev3<real>& p, bool freeze, real psi, real sx, real sy, real sz,
                                            real jx, real jy, real jz, real irc, real& fx, real& fy, real& fz,
                                            real& s2, real& ux, real& uy, real& uz) {
  fx = real(0);
  fy = real(0);
  fz = real(0);
  s2 = real(0);
  if (!freeze) {
    const real c = -p.G * psi;
    fx = c * sx;
    fy = c * sy;
    fz = c * sz;
    s2 = p.GG * (sx * sx + sy * sy + sz * sz);
  }
  const real ir = irc * p.cv;  // 1/rho
  ux = (jx + real(0.5) * fx) * ir;
  uy = (jy + real(0.5) * fy) * ir;
  uz = (jz + real(0.5) * fz) * ir;
}

// Neighbour term of div u at one node for direction i: 3 w_i c_i . u(x + c_i)
template <typename real>
__device__ __forceinline__ real divu_term(int i, real ux, real uy, real uz) {
  real cu = real(0);
  if (cx19(i)) cu += cx19(i) > 0 ? ux : -ux;
  if (cy19(i)) cu += cy19(i) > 0 ? uy : -uy;
  if (cz19(i)) cu += cz19(i) > 0 ? uz : -uz;
  return real(w36(i) / 12.0) * cu;  // 3 w_i = w36 / 12
}

// Rows of the moment basis that change sign with c (odd in c): the momentum, energy-flux and
// third-order rows
__host__ __device__ constexpr bool odd_row(int r) { return (r >= 3 && r <= 8) || r >= 16; }
// velocities 2k - 1 and 2k are opposite, and every row is even or odd in c as odd_row says
constexpr bool pairs_consistent() {
  for (int k = 1; k < 10; ++k) {
    if (cx19(2 * k) != -cx19(2 * k - 1) || cy19(2 * k) != -cy19(2 * k - 1) || cz19(2 * k) != -cz19(2 * k - 1))
      return false;
    for (int r = 0; r < 19; ++r) {
      const int a = mrow(r, 2 * k - 1), b = mrow(r, 2 * k);
      if (odd_row(r) ? a != -b : a != b) return false;
    }
  }
  for (int r = 0; r < 19; ++r)
    if (odd_row(r) && mrow(r, 0) != 0) return false;
  return true;
}
static_assert(pairs_consistent(), "D3Q19 pair structure of the moment basis");

// D3Q19 MRT collision with Li's forcing: f* = f + M^-1 dm, dm = -S (M f - m_eq) + (1 - S/2) (M G + sigma)
// with m_eq = M f_eq and M G of the forcing term G_i = w_i [3 (c_i - u) . F + 9 (c_i . u)(c_i . F)]
// in closed form.  M and M^-1 = M^T diag(1/|M_r|^2) act on the nine pairs of opposite velocities
// (2k - 1, 2k): an even row sees the pair sums, an odd row the differences.  Rates: s_e, s_eps, the
// viscous rate on the five stress rows (9, 11, 13, 14, 15), 1 on all others.
template <typename real>
__device__ __forceinline__ void flow_collide3(const Dev3<real>& p, const real (&f)[19], real rho, real ux, real uy,
                                              real uz, real Fx, real Fy, real Fz, real S2, real (&fs)[19]) {
  real ps[10], pd[10];
#pragma unroll
  for (int k = 1; k < 10; ++k) {
    ps[k] = f[2 * k - 1] + f[2 * k];
    pd[k] = f[2 * k - 1] - f[2 * k];
  }
  real m[19];
#pragma unroll
  for (int r = 0; r < 19; ++r) {
    real v = mrow(r, 0) != 0 ? real(mrow(r, 0)) * f[0] : real(0);
#pragma unroll
    for (int k = 1; k < 10; ++k) {
      const int c = mrow(r, 2 * k - 1);
      const real x = odd_row(r) ? pd[k] : ps[k];
      if (c == 1) v += x;
      else if (c == -1) v -= x;
      else if (c != 0) v += real(c) * x;
    }
    m[r] = v;
  }
  const real uu = ux * ux + uy * uy + uz * uz;
  const real pxx = rho * (real(2) * ux * ux - uy * uy - uz * uz), pww = rho * (uy * uy - uz * uz);
  const real meq[19] = {rho, rho * (real(-11) + real(19) * uu), rho * (real(3) - real(5.5) * uu),
                        rho * ux, real(-2.0 / 3.0) * rho * ux, rho * uy, real(-2.0 / 3.0) * rho * uy,
                        rho * uz, real(-2.0 / 3.0) * rho * uz, pxx, real(-0.5) * pxx, pww, real(-0.5) * pww,
                        rho * ux * uy, rho * uy * uz, rho * ux * uz, real(0), real(0), real(0)};
  const real uF = ux * Fx + uy * Fy + uz * Fz;
  const real axx = real(2) * ux * Fx - uy * Fy - uz * Fz, aww = uy * Fy - uz * Fz;
  const real SF[19] = {real(0), real(38) * uF + p.sig_e * S2, real(-11) * uF + p.sig_eps * S2,
                       Fx, real(-2.0 / 3.0) * Fx, Fy, real(-2.0 / 3.0) * Fy, Fz, real(-2.0 / 3.0) * Fz,
                       real(2) * axx, -axx, real(2) * aww, -aww,
                       ux * Fy + uy * Fx, uy * Fz + uz * Fy, ux * Fz + uz * Fx, real(0), real(0), real(0)};
  // dm_r / |M_r|^2; the collision leaves the mass unchanged (row 0)
  real dl[19];
  dl[0] = real(0);
#pragma unroll
  for (int r = 1; r < 19; ++r) {
    const bool visc = r == 9 || r == 11 || r == 13 || r == 14 || r == 15;
    const real s = r == 1 ? p.s_e : (r == 2 ? p.s_eps : (visc ? p.s_v : real(1)));
    const real om = r == 1 ? p.om_e : (r == 2 ? p.om_eps : (visc ? p.om_v : real(0.5)));
    dl[r] = (-s * (m[r] - meq[r]) + om * SF[r]) * real(1.0 / double(mnorm(r)));
  }
  real e0 = real(0);
#pragma unroll
  for (int r = 0; r < 19; ++r)
    if (mrow(r, 0) != 0) e0 += real(mrow(r, 0)) * dl[r];
  fs[0] = f[0] + e0;
#pragma unroll
  for (int k = 1; k < 10; ++k) {
    real E = real(0), O = real(0);
#pragma unroll
    for (int r = 0; r < 19; ++r) {
      const int c = mrow(r, 2 * k - 1);
      if (c == 0) continue;
      real& acc = odd_row(r) ? O : E;
      if (c == 1) acc += dl[r];
      else if (c == -1) acc -= dl[r];
      else acc += real(c) * dl[r];
    }
    fs[2 * k - 1] = f[2 * k - 1] + (E + O);
    fs[2 * k] = f[2 * k] + (E - O);
  }
}

// D3Q7 collision of one node (Eq. 39) with the non-orthogonal basis (rows 1, c_x, c_y, c_z, c^2,
// c_x^2 - c_y^2, c_x^2 - c_z^2), m_eq = [T, 0, 0, 0, wdot T, 0, 0], the inverse in closed form;
// grad T from the relaxed first moments (Eqs. 49-50), Q (Eq. 20) and S (Eq. 24) as the source.
// T1, T2: T - T_ref of the two previous steps; dv: div u.
template <typename real>
__device__ __forceinline__ void thermal_collide3(const Dev3<real>& p, const real (&g)[7], real rho, real dpdT,
                                                 real ux, real uy, real uz, real dv, real T1, real T2, real& Tr,
                                                 real (&gs)[7]) {
  const real dm1 = p.vs1 * (g[1] - g[2]), dm2 = p.vs1 * (g[3] - g[4]), dm3 = p.vs1 * (g[5] - g[6]);
  Tr = sum7(g);
  const real T = p.T_ref + Tr;
  const real rcv = rho * p.cv;
  const real Q = -(rcv * (ux * (-dm1 * p.inv_cs2h) + uy * (-dm2 * p.inv_cs2h) + uz * (-dm3 * p.inv_cs2h)) +
                   T * dpdT * dv);
  const real Ssum = (p.flags & lbm::FL_NO_S) ? real(0) : rcv * real(0.5) * ((Tr - T1) - (T1 - T2));
  const real m4 = ((g[1] + g[2]) + (g[3] + g[4])) + (g[5] + g[6]);
  const real m5 = (g[1] + g[2]) - (g[3] + g[4]);
  const real m6 = (g[1] + g[2]) - (g[5] + g[6]);
  const real d4 = p.vs3 * (m4 - p.wdot * Tr), d5 = p.vs3 * m5, d6 = p.vs3 * m6;
  const real A = (d4 + d5 + d6) * real(1.0 / 3.0);
  const real B = A - d5, C = A - d6;
  const real src = Q + Ssum;
  const real s0 = p.w0 * src, s1 = p.w1 * src;
  gs[0] = g[0] + d4 + s0;
  gs[1] = g[1] - real(0.5) * (A + dm1) + s1;
  gs[2] = g[2] - real(0.5) * (A - dm1) + s1;
  gs[3] = g[3] - real(0.5) * (B + dm2) + s1;
  gs[4] = g[4] - real(0.5) * (B - dm2) + s1;
  gs[5] = g[5] - real(0.5) * (C + dm3) + s1;
  gs[6] = g[6] - real(0.5) * (C - dm3) + s1;
}

// Anti-bounce-back value of a population leaving a Dirichlet face at T_box
template <typename real>
__device__ __forceinline__ real abb3(const Dev3<real>& p, real gs_out) {
  return -gs_out + p.two_w1 * (p.T_box - p.T_ref);
}

// a wavefront ORs its flags by ballots (every lane takes part) and one lane sets them
__device__ __forceinline__ void report3(unsigned err, unsigned* word) {
  const unsigned long long e1 = __ballot((err & ERR_RHO) != 0u), e2 = __ballot((err & ERR_T) != 0u),
                           e4 = __ballot((err & ERR_PSI) != 0u);
  if ((e1 | e2 | e4) != 0ull && (threadIdx.x & 63u) == 0u)
    atomicOr(word, (e1 ? ERR_RHO : 0u) | (e2 ? ERR_T : 0u) | (e4 ? ERR_PSI : 0u));
}

// ---- per-node path, kernel 1: per-node fields of the current state
template <typename real>
__global__ __launch_bounds__(256) void fields3_kernel(Dev3<real> p, Bufs3<real> b, size_t N) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned err = 0u;
  if (k < N) {
    real f[19], g[7];
#pragma unroll
    for (int i = 0; i < 19; ++i) f[i] = b.fs[i * N + k];
#pragma unroll
    for (int i = 0; i < 7; ++i) g[i] = b.gs[i * N + k];
    real rho, jx, jy, jz, Tr, psi, dpdT, irc;
    node_fields3(p, f, g, rho, jx, jy, jz, Tr, psi, dpdT, irc, err);
    real* sc = b.sc;
    sc[S_RHO * N + k] = rho;
    sc[S_PSI * N + k] = psi;
    sc[S_JX * N + k] = jx;
    sc[S_JY * N + k] = jy;
    sc[S_JZ * N + k] = jz;
    sc[S_TR * N + k] = Tr;
    sc[S_DPDT * N + k] = dpdT;
    sc[S_IRC * N + k] = irc;
  }
  report3(err, b.err);
}

// ---- per-node path, kernel 2: interaction force (Eq. 9 with the D3Q19 weights 1/6, 1/12) and velocity
template <typename real>
__global__ __launch_bounds__(256) void force3_kernel(Dev3<real> p, Bufs3<real> b, size_t N) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  const int nx = p.nx, ny = p.ny, nz = p.nz;
  const int x = (int)(k % (size_t)nx);
  const int y = (int)((k / (size_t)nx) % (size_t)ny);
  const int z = (int)(k / ((size_t)nx * (size_t)ny));
  const real* sc = b.sc;
  const bool freeze = (p.flags & lbm::FL_FREEZE_FLOW) != 0;
  real sx = real(0), sy = real(0), sz = real(0);
  if (!freeze) {
#pragma unroll
    for (int i = 1; i < 19; ++i) {
      const size_t q = ((size_t)wrap1(z + cz19(i), nz) * ny + wrap1(y + cy19(i), ny)) * nx + wrap1(x + cx19(i), nx);
      const real wp = (c2_19(i) == 1 ? real(1.0 / 6.0) : real(1.0 / 12.0)) * sc[S_PSI * N + q];
      if (cx19(i)) sx += cx19(i) > 0 ? wp : -wp;
      if (cy19(i)) sy += cy19(i) > 0 ? wp : -wp;
      if (cz19(i)) sz += cz19(i) > 0 ? wp : -wp;
    }
  }
  real fx, fy, fz, s2, ux, uy, uz;
  node_force3(p, freeze, sc[S_PSI * N + k], sx, sy, sz, sc[S_JX * N + k], sc[S_JY * N + k], sc[S_JZ * N + k],
              sc[S_IRC * N + k], fx, fy, fz, s2, ux, uy, uz);
  real* w = b.sc;
  w[S_UX * N + k] = ux;
  w[S_UY * N + k] = uy;
  w[S_UZ * N + k] = uz;
  w[S_FX * N + k] = fx;
  w[S_FY * N + k] = fy;
  w[S_FZ * N + k] = fz;
  w[S_S2 * N + k] = s2;
}

// ---- per-node path, kernel 3: collision and streaming
template <typename real>
__global__ __launch_bounds__(256) void collide3_kernel(Dev3<real> p, Bufs3<real> b, size_t N) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  const int nx = p.nx, ny = p.ny, nz = p.nz;
  const int x = (int)(k % (size_t)nx);
  const int y = (int)((k / (size_t)nx) % (size_t)ny);
  const int z = (int)(k / ((size_t)nx * (size_t)ny));
  auto node = [&](int dx, int dy, int dz) -> size_t {
    return ((size_t)wrap1(z + dz, nz) * ny + wrap1(y + dy, ny)) * nx + wrap1(x + dx, nx);
  };
  const real* sc = b.sc;
  real f[19], g[7];
#pragma unroll
  for (int i = 0; i < 19; ++i) f[i] = b.fs[i * N + k];
#pragma unroll
  for (int i = 0; i < 7; ++i) g[i] = b.gs[i * N + k];
  const real rho = sc[S_RHO * N + k], dpdT = sc[S_DPDT * N + k], irc = sc[S_IRC * N + k];
  const real ux = sc[S_UX * N + k], uy = sc[S_UY * N + k], uz = sc[S_UZ * N + k];
  const real T1 = b.Th[k], T2 = b.Th[N + k];
  const bool freeze = (p.flags & lbm::FL_FREEZE_FLOW) != 0;

  // div u = 3 sum_i w_i c_i . u(x + c_i) (isotropic central difference, D3Q19 weights)
  real dv = real(0);
#pragma unroll
  for (int i = 1; i < 19; ++i) {
    const size_t q = node(cx19(i), cy19(i), cz19(i));
    dv += divu_term<real>(i, sc[S_UX * N + q], sc[S_UY * N + q], sc[S_UZ * N + q]);
  }
  real fs[19];
  if (freeze) {
#pragma unroll
    for (int i = 0; i < 19; ++i) fs[i] = f[i];
  } else {
    flow_collide3(p, f, rho, ux, uy, uz, sc[S_FX * N + k], sc[S_FY * N + k], sc[S_FZ * N + k], sc[S_S2 * N + k], fs);
  }
  real gs[7], Tr;
  thermal_collide3(p, g, rho, dpdT, ux, uy, uz, dv, T1, T2, Tr, gs);

  // streaming of f (periodic push; a frozen flow keeps its populations in place)
#pragma unroll
  for (int i = 0; i < 19; ++i) b.fd[i * N + (freeze ? k : node(cx19(i), cy19(i), cz19(i)))] = fs[i];

  // streaming of g with the blend at the destination (Eq. 39); a population that would leave a
  // Dirichlet box returns to the node in the opposite direction by anti-bounce-back
  b.gd[k] = g[0] + (gs[0] - g[0]) * irc;
#pragma unroll
  for (int i = 1; i < 7; ++i) {
    const int dx = cx19(i), dy = cy19(i), dz = cz19(i);  // the six axes come first in both sets
    const int opp = (i & 1) ? i + 1 : i - 1;
    const bool out = p.thermal_box && (x + dx < 0 || x + dx >= nx || y + dy < 0 || y + dy >= ny || z + dz < 0 ||
                                       z + dz >= nz);
    if (out) {
      b.gd[opp * N + k] = g[opp] + (abb3(p, gs[i]) - g[opp]) * irc;
    } else {
      const size_t q = node(dx, dy, dz);
      const real gold = b.gs[i * N + q];
      b.gd[i * N + q] = gold + (gs[i] - gold) * sc[S_IRC * N + q];
    }
  }
  b.Th[N + k] = T1;
  b.Th[k] = Tr;
}

// ---- fused path: one kernel per step
//
// A workgroup of 64 x TY threads owns the columns of a 64 x TY tile (thread (lx, ly) the column
// x0 + lx, y0 + ly) and marches through planes z0 .. z0 + Z - 1.  The interaction force at plane q
// needs psi at radius 2 in x-y and at q +- 1, and div u at plane z needs u at z +- 1, so iteration
// `it` (it = 0 .. Z + 3) works on three planes at once:
//   load plane p = z0 - 2 + it (f, g of the tile and of the ring of radius 2 around it), fields,
//     psi to the ring of the last three planes;
//   force and velocity at q = p - 1 over the tile and the ring of radius 1 (u to LDS), then the
//     D3Q19 collision and the push of f at q;
//   the divergence contributions of u(q) to the nodes at q - 1, q, q + 1 (running sums), then the
//     D3Q7 collision and the push of g at z = p - 2, whose divergence is now complete.
// The first threads also load the ring nodes (one each).  Per column, f of one plane waits for
// its collision in LDS (FP32; in registers in FP64, whose LDS is full) and g of two planes in
// registers; 1/(rho c_v) and g_1..g_4 of the last four planes (the streaming destinations in x
// and y) are staged in LDS.  In FP32 the loads of the next plane are issued one iteration ahead.
// Every population of the chunk is read from HBM once and written once; the ring reloads hit the
// L2 that neighbouring tiles share (XCD-aware order).  Each node's arithmetic is that of the
// per-node path (the divergence sums its 18 terms in another order).
template <typename real, int TY, bool FST>
struct Fused3Lds {
  real psi[3][TY + 4][68];  // psi of three consecutive planes over the tile and ring of radius 2
  real u[3][TY + 2][66];    // u of plane q over the tile and ring of radius 1
  real st[4][5][TY + 2][66];  // 1/(rho c_v) and g_1..g_4 of four consecutive planes, radius 1
  real fst[FST ? 2 : 1][19][FST ? TY : 1][FST ? 64 : 1];  // f of the tile, planes p - 1 and p
};

template <typename real, int TY>
__global__ __launch_bounds__(64 * TY) void fused3_kernel(Dev3<real> p, Bufs3<real> b, int lz, int ntx, int nty) {
  static_assert(TY >= 8, "the ring of radius 2 must fit the workgroup (272 + 4 TY <= 64 TY)");
  constexpr bool PF = sizeof(real) == 4;  // prefetch of the next plane and f staged in LDS
  __shared__ Fused3Lds<real, TY, PF> L;
  constexpr uint32_t SZ = sizeof(real);
  const int nx = p.nx, ny = p.ny, nz = p.nz;
  const uint32_t nxy = (uint32_t)nx * (uint32_t)ny;
  const bool freeze = (p.flags & lbm::FL_FREEZE_FLOW) != 0;

  // XCD-aware order: the 8 XCDs take workgroups round-robin; each XCD gets a contiguous range of
  // tiles (x fastest, then y, then the z chunk), so tiles that share ring nodes share one L2
  const int nwg = gridDim.x;
  const int xcd = blockIdx.x % lbm::NXCD;
  const int per = nwg / lbm::NXCD, rem = nwg % lbm::NXCD;
  const int wg = xcd * per + (xcd < rem ? xcd : rem) + blockIdx.x / lbm::NXCD;
  const int x0 = (wg % ntx) * 64, y0 = ((wg / ntx) % nty) * TY, z0 = (wg / (ntx * nty)) * lz;
  const int W = min(64, nx - x0), H = min(TY, ny - y0), Z = min(lz, nz - z0);

  // Addressing: a population plane is under 4 GiB (checked on the host), so every access is a
  // uniform plane base plus one 32-bit byte offset per lane.  The byte offsets below: column in the
  // plane (o_), neighbouring columns for the pushes (x_, r_), planes (z_).
  const int t = threadIdx.x;
  const int lx = t & 63, ly = t >> 6;
  const bool own = lx < W && ly < H;
  const int gx = x0 + lx, gy = y0 + ly;
  const uint32_t o_b = own ? ((uint32_t)gy * (uint32_t)nx + (uint32_t)gx) * SZ : 0u;
  const uint32_t xm_b = (gx == 0 ? nx - 1 : gx - 1) * SZ, x0_b = gx * SZ, xp_b = (gx + 1 >= nx ? 0 : gx + 1) * SZ;
  const uint32_t rm_b = (uint32_t)(gy == 0 ? ny - 1 : gy - 1) * nx * SZ, r0_b = (uint32_t)gy * nx * SZ,
                 rp_b = (uint32_t)(gy + 1 >= ny ? 0 : gy + 1) * nx * SZ;
  const uint32_t plane_b = nxy * SZ;
  // ring node of radius 2: two rows below, two rows above (W + 4 wide), then two columns on each side
  const int rw = W + 4, nring = 4 * rw + 4 * H;
  const bool helper = t < nring;
  int hx = 0, hy = 0;
  if (t < 2 * rw) {
    hy = -2 + t / rw;
    hx = -2 + t % rw;
  } else if (t < 4 * rw) {
    hy = H + (t - 2 * rw) / rw;
    hx = -2 + (t - 2 * rw) % rw;
  } else {
    const int s = t - 4 * rw, c = s & 3;
    hy = s >> 2;
    hx = c < 2 ? c - 2 : W + c - 2;
  }
  const bool h1 = helper && hx >= -1 && hx <= W && hy >= -1 && hy <= H;  // also in the ring of radius 1
  const uint32_t h_b =
      helper ? ((uint32_t)wrap1(y0 + hy, ny) * (uint32_t)nx + (uint32_t)wrap1(x0 + hx, nx)) * SZ : 0u;

  // registers carried between iterations (suffix: how many planes behind the loaded plane p)
  real f1[PF ? 1 : 19];                         // without PF: f of plane p - 1 (collided now)
  real g2[7], g1[7];                            // g of planes p - 2 (collided now) and p - 1
  real g6_3 = real(0);                          // g_6 of plane p - 3: destination of the -z push
  real rho2 = real(1), rho1 = real(1), dp2 = real(0), dp1 = real(0);
  real ir3 = real(0), ir2 = real(0), ir1 = real(0);
  real j1x = real(0), j1y = real(0), j1z = real(0), ps1 = real(0);
  real u2x = real(0), u2y = real(0), u2z = real(0);  // u of plane p - 2
  real A0 = real(0), A1 = real(0);              // divergence sums of planes p - 2 and p - 1
  real hj1x = real(0), hj1y = real(0), hj1z = real(0), hps1 = real(0), hir1 = real(0);
  real fn[19], gn[7], hf[19], hg[7];            // own: the next plane (PF); ring node: its plane
#pragma unroll
  for (int i = 0; i < 19; ++i) fn[i] = hf[i] = real(0);
#pragma unroll
  for (int i = 0; i < (PF ? 1 : 19); ++i) f1[i] = real(0);
#pragma unroll
  for (int i = 0; i < 7; ++i) g2[i] = g1[i] = gn[i] = hg[i] = real(0);
  unsigned err = 0u;

  // f, g of the plane at byte offset zb for the own column and the ring node (lanes without one
  // keep zeros).  The plane stride is opaque to the compiler at each use (lbm::opaque), so the
  // plane bases are recomputed in scalar registers next to their loads and stores instead of being
  // kept live (and spilled) across the loop.
  auto stride = [&]() { return lbm::opaque((size_t)nxy * (size_t)nz); };
  auto ld = [](const real* base, size_t off, uint32_t byte) -> real {
    return lbm::ldb<real>(lbm::sbase(lbm::to_global((const char*)(base + off))), byte);
  };
  auto st = [](real* base, size_t off, uint32_t byte, real v) {
    lbm::stb<real>(lbm::sbase(lbm::to_global((char*)(base + off))), byte, v);
  };
  // the planes of one array in order, one 64-bit scalar add per plane (base + i N would multiply)
  auto walk = [&](const real* base) {
    return lbm::PlaneWalk<const char>{lbm::to_global((const char*)base), (ptrdiff_t)(stride() * sizeof(real))};
  };
  auto walk_out = [&](real* base) {
    return lbm::PlaneWalk<char>{lbm::to_global((char*)base), (ptrdiff_t)(stride() * sizeof(real))};
  };
  auto load_plane = [&](uint32_t zb, real(&ff)[19], real(&gg)[7], real(&hff)[19], real(&hgg)[7]) {
    if (own) {
      auto wf = walk(b.fs), wg = walk(b.gs);
#pragma unroll
      for (int i = 0; i < 19; ++i) ff[i] = lbm::ldb<real>(wf.next(), zb + o_b);
#pragma unroll
      for (int i = 0; i < 7; ++i) gg[i] = lbm::ldb<real>(wg.next(), zb + o_b);
    }
    if (helper) {
      auto wf = walk(b.fs), wg = walk(b.gs);
#pragma unroll
      for (int i = 0; i < 19; ++i) hff[i] = lbm::ldb<real>(wf.next(), zb + h_b);
#pragma unroll
      for (int i = 0; i < 7; ++i) hgg[i] = lbm::ldb<real>(wg.next(), zb + h_b);
    }
  };
  if (PF) load_plane((uint32_t)wrap1(z0 - 2, nz) * plane_b, fn, gn, hf, hg);

  for (int it = 0; it < Z + 4; ++it) {
    const int pz = z0 - 2 + it;
    const int s0 = it % 3, st0 = it & 3;
    const bool force_now = it >= 2, flow_now = it >= 3 && it < Z + 3, thermal_now = it >= 4;
    const int zt = pz - 2;  // plane of the D3Q7 collision (inside the chunk when thermal_now)

    // (a) plane p: loads (issued one iteration ahead when prefetching), fields, psi and the staged
    // destination values to LDS
    // own: f of plane p in fn (PF: loaded one iteration ahead) or f0, g of plane p in g0; ring
    // node: hf, hg
    real f0[PF ? 1 : 19], g0[7];
    if constexpr (!PF) {
#pragma unroll
      for (int i = 0; i < 19; ++i) f0[i] = real(0);
      load_plane((uint32_t)wrap1(pz, nz) * plane_b, f0, gn, hf, hg);
    }
#pragma unroll
    for (int i = 0; i < 7; ++i) g0[i] = gn[i];
    real T1 = real(0), T2 = real(0);
    if (own && thermal_now) {
      const size_t N = stride();
      T1 = ld(b.Th, 0, (uint32_t)zt * plane_b + o_b);
      T2 = ld(b.Th, N, (uint32_t)zt * plane_b + o_b);
    }
    real rho0 = real(1), dp0 = real(0), ir0 = real(0), j0x = real(0), j0y = real(0), j0z = real(0), ps0 = real(0);
    if (own) {
      real Tr;
      if constexpr (PF) {
        node_fields3(p, fn, g0, rho0, j0x, j0y, j0z, Tr, ps0, dp0, ir0, err);
#pragma unroll
        for (int i = 0; i < 19; ++i) L.fst[it & 1][i][ly][lx] = fn[i];
      } else {
        node_fields3(p, f0, g0, rho0, j0x, j0y, j0z, Tr, ps0, dp0, ir0, err);
      }
      L.psi[s0][ly + 2][lx + 2] = ps0;
      L.st[st0][0][ly + 1][lx + 1] = ir0;
#pragma unroll
      for (int i = 1; i < 5; ++i) L.st[st0][i][ly + 1][lx + 1] = g0[i];
    }
    real hj0x = real(0), hj0y = real(0), hj0z = real(0), hps0 = real(0), hir0 = real(0);
    if (helper) {
      real hrho, hTr, hdp;
      node_fields3(p, hf, hg, hrho, hj0x, hj0y, hj0z, hTr, hps0, hdp, hir0, err);
      L.psi[s0][hy + 2][hx + 2] = hps0;
      if (h1) {
        L.st[st0][0][hy + 1][hx + 1] = hir0;
#pragma unroll
        for (int i = 1; i < 5; ++i) L.st[st0][i][hy + 1][hx + 1] = hg[i];
      }
    }
    // the next plane's loads go out before this iteration's stores, so that waiting for them
    // never waits for the stores (one in-order counter covers both)
    if (PF && it + 1 < Z + 4) load_plane((uint32_t)wrap1(pz + 1, nz) * plane_b, fn, gn, hf, hg);
    __syncthreads();

    // (b) plane q = p - 1: force and velocity over radius 1, D3Q19 collision and push of f
    real uqx = real(0), uqy = real(0), uqz = real(0);
    if (force_now) {
      const int sm = (it + 1) % 3, sq = (it + 2) % 3;  // slots of planes q - 1 and q (q + 1 is s0)
      auto psum = [&](int cx, int cy, real& sx, real& sy, real& sz) {
        sx = sy = sz = real(0);
        if (freeze) return;
#pragma unroll
        for (int i = 1; i < 19; ++i) {
          const int sl = cz19(i) > 0 ? s0 : (cz19(i) < 0 ? sm : sq);
          const real wp = (c2_19(i) == 1 ? real(1.0 / 6.0) : real(1.0 / 12.0)) *
                          L.psi[sl][cy + cy19(i) + 2][cx + cx19(i) + 2];
          if (cx19(i)) sx += cx19(i) > 0 ? wp : -wp;
          if (cy19(i)) sy += cy19(i) > 0 ? wp : -wp;
          if (cz19(i)) sz += cz19(i) > 0 ? wp : -wp;
        }
      };
      if (own) {
        real sx, sy, sz, Fx, Fy, Fz, S2;
        psum(lx, ly, sx, sy, sz);
        node_force3(p, freeze, ps1, sx, sy, sz, j1x, j1y, j1z, ir1, Fx, Fy, Fz, S2, uqx, uqy, uqz);
        L.u[0][ly + 1][lx + 1] = uqx;
        L.u[1][ly + 1][lx + 1] = uqy;
        L.u[2][ly + 1][lx + 1] = uqz;
        if (flow_now) {
          const int q = pz - 1;
          const uint32_t zq_b = (uint32_t)q * plane_b;
          real fq[19];  // f of plane q
          if constexpr (PF) {
#pragma unroll
            for (int i = 0; i < 19; ++i) fq[i] = L.fst[(it + 1) & 1][i][ly][lx];
          } else {
#pragma unroll
            for (int i = 0; i < 19; ++i) fq[i] = f1[i];
          }
          auto wd = walk_out(b.fd);
          if (freeze) {
#pragma unroll
            for (int i = 0; i < 19; ++i) lbm::stb<real>(wd.next(), zq_b + o_b, fq[i]);
          } else {
            real fs[19];
            flow_collide3(p, fq, rho1, uqx, uqy, uqz, Fx, Fy, Fz, S2, fs);
            const uint32_t zm_b = (uint32_t)(q == 0 ? nz - 1 : q - 1) * plane_b;
            const uint32_t zp_b = (uint32_t)(q + 1 >= nz ? 0 : q + 1) * plane_b;
#pragma unroll
            for (int i = 0; i < 19; ++i) {
              const uint32_t zz = cz19(i) > 0 ? zp_b : (cz19(i) < 0 ? zm_b : zq_b);
              const uint32_t rr = cy19(i) > 0 ? rp_b : (cy19(i) < 0 ? rm_b : r0_b);
              const uint32_t xx = cx19(i) > 0 ? xp_b : (cx19(i) < 0 ? xm_b : x0_b);
              lbm::stb<real>(wd.next(), zz + rr + xx, fs[i]);
            }
          }
        }
      }
      if (h1) {
        real sx, sy, sz, Fx, Fy, Fz, S2, hux, huy, huz;
        psum(hx, hy, sx, sy, sz);
        node_force3(p, freeze, hps1, sx, sy, sz, hj1x, hj1y, hj1z, hir1, Fx, Fy, Fz, S2, hux, huy, huz);
        L.u[0][hy + 1][hx + 1] = hux;
        L.u[1][hy + 1][hx + 1] = huy;
        L.u[2][hy + 1][hx + 1] = huz;
      }
    }
    __syncthreads();

    // (c) divergence contributions of u(q), then plane zt = p - 2: D3Q7 collision and push of g
    real A2 = real(0);
    if (own && force_now) {
      auto U = [&](int c, int dx, int dy) -> real { return L.u[c][ly + 1 + dy][lx + 1 + dx]; };
#pragma unroll
      for (int i = 1; i < 19; ++i) {
        // node (x, y, q - cz_i) has its neighbour in direction i at (x + cx_i, y + cy_i, q)
        const real v = divu_term<real>(i, U(0, cx19(i), cy19(i)), U(1, cx19(i), cy19(i)), U(2, cx19(i), cy19(i)));
        if (cz19(i) > 0) A0 += v;
        else if (cz19(i) == 0) A1 += v;
        else A2 += v;
      }
    }
    if (own && thermal_now) {
      real gs[7], Tr;
      thermal_collide3(p, g2, rho2, dp2, u2x, u2y, u2z, A0, T1, T2, Tr, gs);
      const size_t N = stride();
      const uint32_t zz_b = (uint32_t)zt * plane_b;
      const int sd = (it + 2) & 3;  // staging slot of plane zt
      auto wd = walk_out(b.gd);
      lbm::stb<real>(wd.next(), zz_b + o_b, g2[0] + (gs[0] - g2[0]) * ir2);
#pragma unroll
      for (int i = 1; i < 7; ++i) {
        const auto pl = wd.next();  // plane i
        const int dx = cx19(i), dy = cy19(i), dz = cz19(i);
        const int opp = (i & 1) ? i + 1 : i - 1;
        const bool out = p.thermal_box && (gx + dx < 0 || gx + dx >= nx || gy + dy < 0 || gy + dy >= ny ||
                                           zt + dz < 0 || zt + dz >= nz);
        if (out) {
          st(b.gd, opp * N, zz_b + o_b, g2[opp] + (abb3(p, gs[i]) - g2[opp]) * ir2);
        } else {
          real gold, ird;
          uint32_t dst;
          if (dz > 0) {
            gold = g1[5];
            ird = ir1;
            dst = (uint32_t)(zt + 1 >= nz ? 0 : zt + 1) * plane_b + o_b;
          } else if (dz < 0) {
            gold = g6_3;
            ird = ir3;
            dst = (uint32_t)(zt == 0 ? nz - 1 : zt - 1) * plane_b + o_b;
          } else {
            gold = L.st[sd][i][ly + 1 + dy][lx + 1 + dx];
            ird = L.st[sd][0][ly + 1 + dy][lx + 1 + dx];
            dst = zz_b + (dy > 0 ? rp_b : (dy < 0 ? rm_b : r0_b)) + (dx > 0 ? xp_b : (dx < 0 ? xm_b : x0_b));
          }
          lbm::stb<real>(pl, dst, gold + (gs[i] - gold) * ird);
        }
      }
      st(b.Th, N, zz_b + o_b, T1);
      st(b.Th, 0, zz_b + o_b, Tr);
    }

    // rotate the registers by one plane
    A0 = A1;
    A1 = A2;
    u2x = uqx;
    u2y = uqy;
    u2z = uqz;
    g6_3 = g2[6];
#pragma unroll
    for (int i = 0; i < 7; ++i) {
      g2[i] = g1[i];
      g1[i] = g0[i];
    }
    if constexpr (!PF) {
#pragma unroll
      for (int i = 0; i < 19; ++i) f1[i] = f0[i];
    }
    rho2 = rho1;
    rho1 = rho0;
    dp2 = dp1;
    dp1 = dp0;
    ir3 = ir2;
    ir2 = ir1;
    ir1 = ir0;
    j1x = j0x;
    j1y = j0y;
    j1z = j0z;
    ps1 = ps0;
    hj1x = hj0x;
    hj1y = hj0y;
    hj1z = hj0z;
    hps1 = hps0;
    hir1 = hir0;
  }
  report3(err, b.err);
}

// f = f_eq (Eq. 3 on D3Q19), g = what T (Eq. 22) relative to T_ref, history = T - T_ref
template <typename real>
__global__ void init3_kernel(const double* __restrict__ in, real* f, real* g, real* Th, size_t N, double w0, double w1,
                             double T_ref) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  const double rho = in[k], ux = in[N + k], uy = in[2 * N + k], uz = in[3 * N + k], T = in[4 * N + k];
  const double uu = ux * ux + uy * uy + uz * uz;
  for (int i = 0; i < 19; ++i) {
    const double cu = cx19(i) * ux + cy19(i) * uy + cz19(i) * uz;
    f[i * N + k] = (real)(w36(i) / 36.0 * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu));
  }
  const double Tr = T - T_ref;
  g[k] = (real)(w0 * Tr);
  for (int i = 1; i < 7; ++i) g[i * N + k] = (real)(w1 * Tr);
  Th[k] = (real)Tr;
  Th[N + k] = (real)Tr;
}

// rho, u, T of the per-node planes to FP64 staging
template <typename real>
__global__ void out3_kernel(const real* sc, double* out, size_t N, double T_ref) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  out[k] = (double)sc[S_RHO * N + k];
  out[N + k] = (double)sc[S_UX * N + k];
  out[2 * N + k] = (double)sc[S_UY * N + k];
  out[3 * N + k] = (double)sc[S_UZ * N + k];
  out[4 * N + k] = T_ref + (double)sc[S_TR * N + k];
}

// deterministic FP64 sums of rho and rho c_v T: fixed ranges per workgroup, fixed tree order
template <typename real>
__global__ __launch_bounds__(RED3) void diag3_partial(const real* f, const real* g, size_t N, double cv, double T_ref,
                                                      size_t per, double* part) {
  __shared__ double sm[RED3], se[RED3];
  const size_t begin = (size_t)blockIdx.x * per, end = begin + per < N ? begin + per : N;
  double m = 0.0, e = 0.0;
  for (size_t k = begin + threadIdx.x; k < end; k += RED3) {
    real ff[19], gg[7];
    for (int i = 0; i < 19; ++i) ff[i] = f[i * N + k];
    for (int i = 0; i < 7; ++i) gg[i] = g[i * N + k];
    const double r = (double)sum19(ff);
    m += r;
    e += r * cv * (T_ref + (double)sum7(gg));
  }
  sm[threadIdx.x] = m;
  se[threadIdx.x] = e;
  __syncthreads();
  for (int s = RED3 / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sm[threadIdx.x] += sm[threadIdx.x + s];
      se[threadIdx.x] += se[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sm[0];
    part[2 * blockIdx.x + 1] = se[0];
  }
}
__global__ __launch_bounds__(RED3) void diag3_final(const double* part, int n, double* out) {
  __shared__ double sm[RED3], se[RED3];
  double m = 0.0, e = 0.0;
  for (int k = threadIdx.x; k < n; k += RED3) {
    m += part[2 * k];
    e += part[2 * k + 1];
  }
  sm[threadIdx.x] = m;
  se[threadIdx.x] = e;
  __syncthreads();
  for (int s = RED3 / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sm[threadIdx.x] += sm[threadIdx.x + s];
      se[threadIdx.x] += se[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = sm[0];
    out[1] = se[0];
  }
}

size_t al(size_t b) { return (b + ALIGN3 - 1) / ALIGN3 * ALIGN3; }

}  // namespace lbm3

using namespace lbm3;

struct lbm3d_ctx {
  lbm3d_params prm{};
  hipStream_t stream = nullptr;
  int device = 0;
  char* base = nullptr;
  size_t N = 0, rsz = 4;
  void *fA = nullptr, *gA = nullptr, *fB = nullptr, *gB = nullptr, *Th = nullptr, *sc = nullptr;
  unsigned* d_err = nullptr;
  double* d_diag = nullptr;
  double* d_part = nullptr;
  int gen = 0;
  int64_t steps = 0;
  double T_ref = 0.0;
  bool initialised = false, failed = false;
  std::string last_error;
};

namespace {

lbm_status fail3(lbm3d_ctx* h, lbm_status s, const std::string& m) {
  if (h) h->last_error = m;
  return s;
}
#define HIP3(h, call)                                                                                           \
  do {                                                                                                          \
    hipError_t e_ = (call);                                                                                     \
    if (e_ != hipSuccess) return fail3((h), LBM_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

double pr_kappa3(const lbm3d_params* p) {
  return 0.37464 + 1.54226 * p->acentric - 0.26992 * p->acentric * p->acentric;
}

template <typename real>
Dev3<real> derive3(const lbm3d_params* p, double T_ref) {
  Dev3<real> d{};
  const double Tc = 0.0778 * p->a / (0.45724 * p->b * p->R);
  d.e.a = (real)p->a;
  d.e.b = (real)p->b;
  d.e.R = (real)p->R;
  d.e.Tc = (real)Tc;
  d.e.kappa = (real)pr_kappa3(p);
  d.e.opk = (real)(1.0 + pr_kappa3(p));
  d.e.inv_G = (real)(1.0 / p->G);
  d.G = (real)p->G;
  d.GG = (real)(p->G * p->G);
  d.cv = (real)p->cv;
  d.T_ref = (real)T_ref;
  const double sv = 1.0 / (3.0 * p->nu + 0.5);
  d.s_e = (real)p->s_e;
  d.s_eps = (real)p->s_eps;
  d.s_v = (real)sv;
  d.om_e = (real)(1.0 - 0.5 * p->s_e);
  d.om_eps = (real)(1.0 - 0.5 * p->s_eps);
  d.om_v = (real)(1.0 - 0.5 * sv);
  d.sig_e = (real)(9.5 * p->sigma / (1.0 / p->s_e - 0.5));
  d.sig_eps = (real)(-2.75 * p->sigma / (1.0 / p->s_eps - 0.5));
  const double cs2h = p->wdot / 3.0;
  d.w0 = (real)(1.0 - p->wdot);
  d.w1 = (real)(p->wdot / 6.0);
  d.vs1 = (real)(1.0 / (p->lambda / cs2h + 0.5));
  d.vs3 = (real)p->vs3;
  d.wdot = (real)p->wdot;
  d.inv_cs2h = (real)(1.0 / cs2h);
  d.two_w1 = (real)(p->wdot / 3.0);
  d.T_box = (real)p->T_box;
  d.nx = p->nx;
  d.ny = p->ny;
  d.nz = p->nz;
  d.thermal_box = p->thermal_box ? 1 : 0;
  d.flags = p->flags;
  return d;
}

template <typename real>
Bufs3<real> bufs(lbm3d_ctx* h) {
  Bufs3<real> b{};
  const bool odd = h->gen != 0;
  b.fs = (const real*)(odd ? h->fB : h->fA);
  b.gs = (const real*)(odd ? h->gB : h->gA);
  b.fd = (real*)(odd ? h->fA : h->fB);
  b.gd = (real*)(odd ? h->gA : h->gB);
  b.Th = (real*)h->Th;
  b.sc = (real*)h->sc;
  b.err = h->d_err;
  return b;
}

template <typename real>
void launch_fields(lbm3d_ctx* h) {
  const int nb = (int)((h->N + 255) / 256);
  const Dev3<real> p = derive3<real>(&h->prm, h->T_ref);
  const Bufs3<real> b = bufs<real>(h);
  fields3_kernel<real><<<nb, 256, 0, h->stream>>>(p, b, h->N);
  force3_kernel<real><<<nb, 256, 0, h->stream>>>(p, b, h->N);
}

// Column tiles of the fused path (64 x FUSED_TY) and planes per workgroup.  A workgroup fills a
// compute unit (its registers allow one per CU), so a launch takes ceil(workgroups / 256) rounds of
// (planes + 4) iterations each (the 4 extra planes are the chunk's halo in z).  Without a choice of
// the caller the number of z chunks minimises that; ties go to fewer chunks.
constexpr int FUSED_TY = 8;
constexpr int NCU3 = 256;

void fused_geometry(const lbm3d_params* p, int& ntx, int& nty, int& lz, int& nwg) {
  ntx = (p->nx + 63) / 64;
  nty = (p->ny + FUSED_TY - 1) / FUSED_TY;
  const long long cols = (long long)ntx * nty;
  int nch = 1;
  if (p->z_chunk > 0) {
    nch = (p->nz + p->z_chunk - 1) / p->z_chunk;
  } else {
    long long best = -1;
    for (int c = 1; c <= p->nz; ++c) {
      const int l = (p->nz + c - 1) / c;
      if ((p->nz + l - 1) / l != c) continue;  // same chunk length as a smaller count
      const long long cost = (cols * c + NCU3 - 1) / NCU3 * (l + 4);
      if (best < 0 || cost < best) {
        best = cost;
        nch = c;
      }
    }
  }
  lz = (p->nz + nch - 1) / nch;
  nch = (p->nz + lz - 1) / lz;
  nwg = (int)(cols * nch);
}

template <typename real>
void launch_step3(lbm3d_ctx* h) {
  if (h->prm.path == LBM3D_PATH_FUSED) {
    int ntx, nty, lz, nwg;
    fused_geometry(&h->prm, ntx, nty, lz, nwg);
    fused3_kernel<real, FUSED_TY><<<nwg, 64 * FUSED_TY, 0, h->stream>>>(
        derive3<real>(&h->prm, h->T_ref), bufs<real>(h), lz, ntx, nty);
    return;
  }
  launch_fields<real>(h);
  const int nb = (int)((h->N + 255) / 256);
  collide3_kernel<real><<<nb, 256, 0, h->stream>>>(derive3<real>(&h->prm, h->T_ref), bufs<real>(h), h->N);
}

lbm_status check3(lbm3d_ctx* h) {
  unsigned e = 0;
  HIP3(h, hipMemcpyAsync(&e, h->d_err, sizeof(e), hipMemcpyDeviceToHost, h->stream));
  HIP3(h, hipStreamSynchronize(h->stream));
  if (e) {
    h->failed = true;
    return fail3(h, LBM_E_NUMERIC, "numerical failure on the device (density, temperature or pseudopotential)");
  }
  return LBM_OK;
}

bool pos(double v) { return std::isfinite(v) && v > 0.0; }

}  // namespace

extern "C" {

void lbm3d_params_default(lbm3d_params* p, int32_t nx, int32_t ny, int32_t nz) {
  std::memset(p, 0, sizeof(*p));
  p->nx = nx;
  p->ny = ny;
  p->nz = nz;
  p->precision = LBM_FP32;
  p->a = 3.0 / 49.0;
  p->b = 2.0 / 21.0;
  p->R = 1.0;
  p->acentric = 0.344;
  p->G = -1.0;
  p->nu = 0.1;
  p->s_e = p->s_eps = 1.0;
  p->sigma = 1.25;
  p->lambda = 1.0 / 3.0;
  p->cv = 5.0;
  p->wdot = 2.0 / 3.0;
  p->vs3 = 1.0;
}

lbm_status lbm3d_validate(const lbm3d_params* p) {
  if (!p || p->nx < 3 || p->ny < 3 || p->nz < 3) return LBM_E_INVAL;
  if (p->precision != LBM_FP32 && p->precision != LBM_FP64) return LBM_E_INVAL;
  const double plane = (double)p->nx * p->ny * p->nz * (p->precision == LBM_FP64 ? 8.0 : 4.0);
  if (plane > 4294967295.0) return LBM_E_INVAL;
  auto rate = [](double s) { return std::isfinite(s) && s > 0.0 && s < 2.0; };
  if (!(p->nu > 0.0) || !(p->lambda > 0.0) || !(p->cv > 0.0) || !(p->wdot > 0.0 && p->wdot < 1.0)) return LBM_E_INVAL;
  if (!rate(p->s_e) || !rate(p->s_eps) || !rate(p->vs3) || !rate(1.0 / (3.0 * p->nu + 0.5)) ||
      !rate(1.0 / (p->lambda / (p->wdot / 3.0) + 0.5)))
    return LBM_E_INVAL;
  if (!(p->a > 0.0) || !(p->b > 0.0) || !(p->R > 0.0) || !(p->G < 0.0) || !std::isfinite(p->sigma)) return LBM_E_INVAL;
  if ((p->flags & ~(uint32_t)(LBM_FREEZE_FLOW | LBM_NO_S)) != 0) return LBM_E_INVAL;
  if (p->thermal_box && !pos(p->T_box)) return LBM_E_INVAL;
  if (p->z_chunk < 0 || (p->path != LBM3D_PATH_FUSED && p->path != LBM3D_PATH_PER_NODE)) return LBM_E_INVAL;
  return LBM_OK;
}

size_t lbm3d_footprint_bytes(const lbm3d_params* p) {
  if (lbm3d_validate(p) != LBM_OK) return 0;
  const size_t N = (size_t)p->nx * p->ny * p->nz, r = p->precision == LBM_FP64 ? 8 : 4;
  return CTRL3 + PART3 + 2 * al(19 * N * r) + 2 * al(7 * N * r) + al(2 * N * r) + al(NSCR * N * r);
}

lbm_status lbm3d_create(const lbm3d_params* p, void* dev_mem, size_t bytes, void* hip_stream, lbm3d_ctx** out) {
  if (!out) return LBM_E_INVAL;
  *out = nullptr;
  if (lbm3d_validate(p) != LBM_OK) return LBM_E_INVAL;
  if (!dev_mem || ((uintptr_t)dev_mem % ALIGN3) != 0) return LBM_E_INVAL;
  if (bytes < lbm3d_footprint_bytes(p)) return LBM_E_NOMEM;
  lbm3d_ctx* h = new (std::nothrow) lbm3d_ctx();
  if (!h) return LBM_E_NOMEM;
  h->prm = *p;
  h->stream = (hipStream_t)hip_stream;
  if (hipGetDevice(&h->device) != hipSuccess) {
    delete h;
    return LBM_E_DEVICE;
  }
  h->N = (size_t)p->nx * p->ny * p->nz;
  h->rsz = p->precision == LBM_FP64 ? 8 : 4;
  char* q = (char*)dev_mem;
  h->base = q;
  h->d_err = (unsigned*)q;
  h->d_diag = (double*)(q + 256);
  q += CTRL3;
  h->d_part = (double*)q;
  q += PART3;
  const size_t N = h->N, r = h->rsz;
  h->fA = q; q += al(19 * N * r);
  h->fB = q; q += al(19 * N * r);
  h->gA = q; q += al(7 * N * r);
  h->gB = q; q += al(7 * N * r);
  h->Th = q; q += al(2 * N * r);
  h->sc = q;
  *out = h;
  return LBM_OK;
}

lbm_status lbm3d_init(lbm3d_ctx* h, const double* rho, const double* ux, const double* uy, const double* uz,
                      const double* T) {
  lbm::HostRange range_("lbm3d_init");
  if (!h || !rho || !ux || !uy || !uz || !T) return LBM_E_INVAL;
  const size_t N = h->N;
  double sumT = 0.0, rmin = std::numeric_limits<double>::infinity();
  for (size_t k = 0; k < N; ++k) {
    if (!pos(rho[k]) || !pos(T[k]) || !std::isfinite(ux[k]) || !std::isfinite(uy[k]) || !std::isfinite(uz[k]))
      return fail3(h, LBM_E_INVAL, "initial fields must be finite with rho > 0 and T > 0");
    sumT += T[k];
    rmin = std::min(rmin, rho[k]);
  }
  if (rmin * h->prm.cv < 1.0) return fail3(h, LBM_E_INVAL, "min(rho) * c_v < 1");
  h->T_ref = h->prm.precision == LBM_FP64 ? sumT / (double)N : (double)(float)(sumT / (double)N);
  double* stage = (double*)h->fB;  // 19 N reals hold 5 N doubles in either precision
  const double* src[5] = {rho, ux, uy, uz, T};
  for (int i = 0; i < 5; ++i)
    HIP3(h, hipMemcpyAsync(stage + i * N, src[i], N * sizeof(double), hipMemcpyHostToDevice, h->stream));
  const int nb = (int)((N + 255) / 256);
  const double w0 = 1.0 - h->prm.wdot, w1 = h->prm.wdot / 6.0;
  if (h->prm.precision == LBM_FP64)
    init3_kernel<double><<<nb, 256, 0, h->stream>>>(stage, (double*)h->fA, (double*)h->gA, (double*)h->Th, N, w0, w1,
                                                     h->T_ref);
  else
    init3_kernel<float><<<nb, 256, 0, h->stream>>>(stage, (float*)h->fA, (float*)h->gA, (float*)h->Th, N, w0, w1,
                                                    h->T_ref);
  HIP3(h, hipGetLastError());
  HIP3(h, hipMemsetAsync(h->d_err, 0, sizeof(unsigned), h->stream));
  HIP3(h, hipStreamSynchronize(h->stream));
  h->gen = 0;
  h->steps = 0;
  h->initialised = true;
  h->failed = false;
  return LBM_OK;
}

lbm_status lbm3d_step(lbm3d_ctx* h, int64_t n) {
  lbm::HostRange range_("lbm3d_step");
  if (!h || n < 0) return LBM_E_INVAL;
  if (!h->initialised) return fail3(h, LBM_E_STATE, "lbm3d_step before lbm3d_init");
  if (h->failed) return fail3(h, LBM_E_STATE, "context has failed: " + h->last_error);
  for (int64_t s = 0; s < n; ++s) {
    if (h->prm.precision == LBM_FP64) launch_step3<double>(h);
    else launch_step3<float>(h);
    h->gen ^= 1;
  }
  HIP3(h, hipGetLastError());
  h->steps += n;
  return LBM_OK;
}

lbm_status lbm3d_sync(lbm3d_ctx* h) {
  if (!h) return LBM_E_INVAL;
  return check3(h);
}

lbm_status lbm3d_read_fields(lbm3d_ctx* h, double* rho, double* ux, double* uy, double* uz, double* T) {
  lbm::HostRange range_("lbm3d_read_fields");
  if (!h) return LBM_E_INVAL;
  if (!h->initialised) return fail3(h, LBM_E_STATE, "read before init");
  if (h->prm.precision == LBM_FP64) launch_fields<double>(h);
  else launch_fields<float>(h);
  const size_t N = h->N;
  double* stage = (double*)(h->gen ? h->fA : h->fB);  // the buffer the next step writes
  const int nb = (int)((N + 255) / 256);
  if (h->prm.precision == LBM_FP64)
    out3_kernel<double><<<nb, 256, 0, h->stream>>>((const double*)h->sc, stage, N, h->T_ref);
  else
    out3_kernel<float><<<nb, 256, 0, h->stream>>>((const float*)h->sc, stage, N, h->T_ref);
  HIP3(h, hipGetLastError());
  double* dst[5] = {rho, ux, uy, uz, T};
  for (int i = 0; i < 5; ++i)
    if (dst[i]) HIP3(h, hipMemcpyAsync(dst[i], stage + i * N, N * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  return check3(h);
}

lbm_status lbm3d_diagnostics(lbm3d_ctx* h, double* mass, double* energy) {
  if (!h || !mass || !energy) return LBM_E_INVAL;
  if (!h->initialised) return fail3(h, LBM_E_STATE, "diagnostics before init");
  const size_t N = h->N;
  size_t per = (N + MAXB3 - 1) / MAXB3;
  if (per < (size_t)RED3) per = RED3;
  const int nparts = (int)((N + per - 1) / per);
  const void* f = h->gen ? h->fB : h->fA;
  const void* g = h->gen ? h->gB : h->gA;
  if (h->prm.precision == LBM_FP64)
    diag3_partial<double><<<nparts, RED3, 0, h->stream>>>((const double*)f, (const double*)g, N, h->prm.cv, h->T_ref,
                                                          per, h->d_part);
  else
    diag3_partial<float><<<nparts, RED3, 0, h->stream>>>((const float*)f, (const float*)g, N, h->prm.cv, h->T_ref,
                                                         per, h->d_part);
  diag3_final<<<1, RED3, 0, h->stream>>>(h->d_part, nparts, h->d_diag);
  HIP3(h, hipGetLastError());
  double out[2];
  HIP3(h, hipMemcpyAsync(out, h->d_diag, sizeof(out), hipMemcpyDeviceToHost, h->stream));
  lbm_status s = check3(h);
  *mass = out[0];
  *energy = out[1];
  return s;
}

int64_t lbm3d_steps_done(const lbm3d_ctx* h) { return h ? h->steps : -1; }

}  // extern "C"

namespace {
// Trailer of a saved three-dimensional state (after the planes), checked on load.
struct State3Trailer {
  char magic[8];      // "LBM3D"
  int32_t version;    // STATE3_VERSION
  int32_t precision;
  int32_t nx, ny, nz;
  int32_t reserved;
  int64_t steps;
  double T_ref;       // storage offset of g and the history
};
static_assert(sizeof(State3Trailer) == 48, "state trailer layout");
constexpr int32_t STATE3_VERSION = 2;
constexpr char STATE3_MAGIC[8] = {'L', 'B', 'M', '3', 'D', 0, 0, 0};
size_t planes3_bytes(const lbm3d_ctx* h) { return 28 * h->N * h->rsz; }
}  // namespace

extern "C" {

size_t lbm3d_state_bytes(const lbm3d_ctx* h) { return h ? planes3_bytes(h) + sizeof(State3Trailer) : 0; }

lbm_status lbm3d_save_state(lbm3d_ctx* h, void* host, size_t bytes) {
  if (!h || !host) return LBM_E_INVAL;
  if (!h->initialised) return fail3(h, LBM_E_STATE, "lbm3d_save_state before lbm3d_init");
  if (bytes < lbm3d_state_bytes(h)) return fail3(h, LBM_E_INVAL, "host buffer smaller than lbm3d_state_bytes");
  char* q = (char*)host;
  const size_t N = h->N, r = h->rsz;
  HIP3(h, hipMemcpyAsync(q, h->gen ? h->fB : h->fA, 19 * N * r, hipMemcpyDeviceToHost, h->stream));
  HIP3(h, hipMemcpyAsync(q + 19 * N * r, h->gen ? h->gB : h->gA, 7 * N * r, hipMemcpyDeviceToHost, h->stream));
  HIP3(h, hipMemcpyAsync(q + 26 * N * r, h->Th, 2 * N * r, hipMemcpyDeviceToHost, h->stream));
  HIP3(h, hipStreamSynchronize(h->stream));
  State3Trailer t{};
  std::memcpy(t.magic, STATE3_MAGIC, sizeof(t.magic));
  t.version = STATE3_VERSION;
  t.precision = h->prm.precision;
  t.nx = h->prm.nx;
  t.ny = h->prm.ny;
  t.nz = h->prm.nz;
  t.steps = h->steps;
  t.T_ref = h->T_ref;
  std::memcpy(q + planes3_bytes(h), &t, sizeof(t));
  return check3(h);
}

lbm_status lbm3d_load_state(lbm3d_ctx* h, const void* host, size_t bytes) {
  if (!h || !host) return LBM_E_INVAL;
  if (bytes != lbm3d_state_bytes(h)) return fail3(h, LBM_E_INVAL, "buffer size differs from lbm3d_state_bytes");
  const char* q = (const char*)host;
  State3Trailer t;
  std::memcpy(&t, q + planes3_bytes(h), sizeof(t));
  if (std::memcmp(t.magic, STATE3_MAGIC, sizeof(t.magic)) != 0 || t.version != STATE3_VERSION)
    return fail3(h, LBM_E_INVAL, "not a saved three-dimensional state of this library version");
  if (t.precision != h->prm.precision || t.nx != h->prm.nx || t.ny != h->prm.ny || t.nz != h->prm.nz)
    return fail3(h, LBM_E_INVAL, "saved state of another precision or grid");
  if (t.steps < 0 || !std::isfinite(t.T_ref)) return fail3(h, LBM_E_INVAL, "corrupt state trailer");
  const size_t N = h->N, r = h->rsz;
  h->steps = t.steps;
  h->T_ref = t.T_ref;
  h->gen = 0;  // the state goes to the A buffers
  HIP3(h, hipMemcpyAsync(h->fA, q, 19 * N * r, hipMemcpyHostToDevice, h->stream));
  HIP3(h, hipMemcpyAsync(h->gA, q + 19 * N * r, 7 * N * r, hipMemcpyHostToDevice, h->stream));
  HIP3(h, hipMemcpyAsync(h->Th, q + 26 * N * r, 2 * N * r, hipMemcpyHostToDevice, h->stream));
  const unsigned zero = 0;
  HIP3(h, hipMemcpyAsync(h->d_err, &zero, sizeof(zero), hipMemcpyHostToDevice, h->stream));
  HIP3(h, hipStreamSynchronize(h->stream));
  h->initialised = true;
  h->failed = false;
  return LBM_OK;
}

lbm_status lbm3d_destroy(lbm3d_ctx* h) {
  if (!h) return LBM_E_INVAL;
  delete h;
  return LBM_OK;
}

}  // extern "C"
