// Three-dimensional extension: D3Q19 MRT pseudopotential flow coupled to the paper's temperature
// model on D3Q7 (include/lbm3d.h states the model).  One step is three kernels over the grid,
// one thread per node:
//   1 fields: rho, j, T (Eqs. 11, 25), p and psi (Eq. 10 and the text after Eq. 9), (dp/dT)_rho,
//     1/(rho c_v), to per-node planes;
//   2 forces: the interaction force (Eq. 9, D3Q19 weights) and the velocity (Eq. 11);
//   3 collision and streaming: div u, grad T (Eqs. 49-50), Q (Eq. 20), S (Eq. 24), the D3Q19 MRT
//     collision with Li's forcing (Eqs. 5, 7, 8), the D3Q7 MRT collision (Eq. 39), push of f
//     and of g with the rho c_v blend at the destination (Eq. 39), anti-bounce-back at
//     Dirichlet faces, the temperature history.
// The per-node fields go through HBM between the kernels; the two-dimensional path keeps them
// in LDS instead (the same fusion in three dimensions is the next step for this path).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <new>
#include <string>

#include "lbm3d.h"
#include "lbm_device.hpp"

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
  real s[19];                  // MRT rates
  real om[19];                 // 1 - s/2
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

// ---- kernel 1: per-node fields of the current state
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
    const real rho = sum19(f);
    real jx = real(0), jy = real(0), jz = real(0);
#pragma unroll
    for (int i = 1; i < 19; ++i) {
      if (cx19(i)) jx += cx19(i) > 0 ? f[i] : -f[i];
      if (cy19(i)) jy += cy19(i) > 0 ? f[i] : -f[i];
      if (cz19(i)) jz += cz19(i) > 0 ? f[i] : -f[i];
    }
    const real Tr = sum7(g);
    const real T = p.T_ref + Tr;
    real psi = real(0), dpdT = real(0);
    if (!(rho > real(0)) || !isfinite(rho)) {
      err |= ERR_RHO;
    } else if (!(T > real(0)) || !isfinite(T)) {
      err |= ERR_T;
    } else {
      real press;
      lbm::pr_eos(p.e, rho, T, press, dpdT);
      psi = lbm::psi_from_pressure(p.e, rho, press, err);
    }
    real* sc = b.sc;
    sc[S_RHO * N + k] = rho;
    sc[S_PSI * N + k] = psi;
    sc[S_JX * N + k] = jx;
    sc[S_JY * N + k] = jy;
    sc[S_JZ * N + k] = jz;
    sc[S_TR * N + k] = Tr;
    sc[S_DPDT * N + k] = dpdT;
    sc[S_IRC * N + k] = lbm::rcp(rho * p.cv);
  }
  // a wavefront ORs its flags by ballots (every lane takes part) and one lane sets them
  const unsigned long long e1 = __ballot((err & ERR_RHO) != 0u), e2 = __ballot((err & ERR_T) != 0u),
                           e4 = __ballot((err & ERR_PSI) != 0u);
  if ((e1 | e2 | e4) != 0ull && (threadIdx.x & 63u) == 0u)
    atomicOr(b.err, (e1 ? ERR_RHO : 0u) | (e2 ? ERR_T : 0u) | (e4 ? ERR_PSI : 0u));
}

// ---- kernel 2: interaction force (Eq. 9 with the D3Q19 weights 1/6, 1/12) and velocity
template <typename real>
__global__ __launch_bounds__(256) void force3_kernel(Dev3<real> p, Bufs3<real> b, size_t N) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  const int nx = p.nx, ny = p.ny, nz = p.nz;
  const int x = (int)(k % (size_t)nx);
  const int y = (int)((k / (size_t)nx) % (size_t)ny);
  const int z = (int)(k / ((size_t)nx * (size_t)ny));
  const real* sc = b.sc;
  real fx = real(0), fy = real(0), fz = real(0), s2 = real(0);
  if (!(p.flags & lbm::FL_FREEZE_FLOW)) {
    real sx = real(0), sy = real(0), sz = real(0);
#pragma unroll
    for (int i = 1; i < 19; ++i) {
      const size_t q = ((size_t)wrap1(z + cz19(i), nz) * ny + wrap1(y + cy19(i), ny)) * nx + wrap1(x + cx19(i), nx);
      const real wp = (c2_19(i) == 1 ? real(1.0 / 6.0) : real(1.0 / 12.0)) * sc[S_PSI * N + q];
      if (cx19(i)) sx += cx19(i) > 0 ? wp : -wp;
      if (cy19(i)) sy += cy19(i) > 0 ? wp : -wp;
      if (cz19(i)) sz += cz19(i) > 0 ? wp : -wp;
    }
    const real c = -p.G * sc[S_PSI * N + k];
    fx = c * sx;
    fy = c * sy;
    fz = c * sz;
    s2 = p.GG * (sx * sx + sy * sy + sz * sz);
  }
  const real ir = sc[S_IRC * N + k] * p.cv;  // 1/rho
  real* w = b.sc;
  w[S_UX * N + k] = (sc[S_JX * N + k] + real(0.5) * fx) * ir;
  w[S_UY * N + k] = (sc[S_JY * N + k] + real(0.5) * fy) * ir;
  w[S_UZ * N + k] = (sc[S_JZ * N + k] + real(0.5) * fz) * ir;
  w[S_FX * N + k] = fx;
  w[S_FY * N + k] = fy;
  w[S_FZ * N + k] = fz;
  w[S_S2 * N + k] = s2;
}

// ---- kernel 3: collision and streaming
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
  const real rho = sc[S_RHO * N + k], Tr = sc[S_TR * N + k], dpdT = sc[S_DPDT * N + k], irc = sc[S_IRC * N + k];
  const real ux = sc[S_UX * N + k], uy = sc[S_UY * N + k], uz = sc[S_UZ * N + k];
  const real Fx = sc[S_FX * N + k], Fy = sc[S_FY * N + k], Fz = sc[S_FZ * N + k], S2 = sc[S_S2 * N + k];
  const real T1 = b.Th[k], T2 = b.Th[N + k];
  const bool freeze = (p.flags & lbm::FL_FREEZE_FLOW) != 0;

  // div u = 3 sum_i w_i c_i . u(x + c_i) (isotropic central difference, D3Q19 weights)
  real dv = real(0);
#pragma unroll
  for (int i = 1; i < 19; ++i) {
    const size_t q = node(cx19(i), cy19(i), cz19(i));
    real cu = real(0);
    if (cx19(i)) cu += cx19(i) > 0 ? sc[S_UX * N + q] : -sc[S_UX * N + q];
    if (cy19(i)) cu += cy19(i) > 0 ? sc[S_UY * N + q] : -sc[S_UY * N + q];
    if (cz19(i)) cu += cz19(i) > 0 ? sc[S_UZ * N + q] : -sc[S_UZ * N + q];
    dv += real(w36(i) / 12.0) * cu;  // 3 w_i = w36 / 12
  }
  // grad T from the relaxed first moments of the D3Q7 populations (Eqs. 49-50)
  const real dm1 = p.vs1 * (g[1] - g[2]), dm2 = p.vs1 * (g[3] - g[4]), dm3 = p.vs1 * (g[5] - g[6]);
  const real T = p.T_ref + Tr;
  const real rcv = rho * p.cv;
  const real Q = -(rcv * (ux * (-dm1 * p.inv_cs2h) + uy * (-dm2 * p.inv_cs2h) + uz * (-dm3 * p.inv_cs2h)) +
                   T * dpdT * dv);
  const real Ssum = (p.flags & lbm::FL_NO_S) ? real(0) : rcv * real(0.5) * ((Tr - T1) - (T1 - T2));

  // D3Q19 MRT collision with Li's forcing: f* = f + M^-1 dm, dm = -S M (f - f_eq) + (1 - S/2) (M G + sigma)
  real fs[19];
  if (freeze) {
#pragma unroll
    for (int i = 0; i < 19; ++i) fs[i] = f[i];
  } else {
    const real uu = ux * ux + uy * uy + uz * uz;
    real dfe[19], G[19];
#pragma unroll
    for (int i = 0; i < 19; ++i) {
      const real cu = real(cx19(i)) * ux + real(cy19(i)) * uy + real(cz19(i)) * uz;
      const real w = real(w36(i) / 36.0);
      dfe[i] = f[i] - w * rho * (real(1) + real(3) * cu + real(4.5) * cu * cu - real(1.5) * uu);
      const real cF = real(cx19(i)) * Fx + real(cy19(i)) * Fy + real(cz19(i)) * Fz;
      const real uF = ux * Fx + uy * Fy + uz * Fz;
      G[i] = w * (real(3) * (cF - uF) + real(9) * cu * cF);
    }
    real dm[19];
#pragma unroll
    for (int r = 0; r < 19; ++r) {
      real d = real(0), fm = real(0);
#pragma unroll
      for (int i = 0; i < 19; ++i) {
        const int c = mrow(r, i);
        if (c != 0) {
          d += real(c) * dfe[i];
          fm += real(c) * G[i];
        }
      }
      if (r == 1) fm += p.sig_e * S2;
      if (r == 2) fm += p.sig_eps * S2;
      dm[r] = -p.s[r] * d + p.om[r] * fm;
    }
#pragma unroll
    for (int i = 0; i < 19; ++i) {
      real v = real(0);
#pragma unroll
      for (int r = 0; r < 19; ++r) {
        const int c = mrow(r, i);
        if (c != 0) v += real(double(c) / double(mnorm(r))) * dm[r];
      }
      fs[i] = f[i] + v;
    }
  }

  // D3Q7 MRT collision (Eq. 39) with the non-orthogonal basis (rows 1, c_x, c_y, c_z, c^2,
  // c_x^2 - c_y^2, c_x^2 - c_z^2), m_eq = [T, 0, 0, 0, wdot T, 0, 0]; the inverse in closed form
  real gs[7];
  {
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
      const real up = -gs[i] + p.two_w1 * (p.T_box - p.T_ref);
      b.gd[opp * N + k] = g[opp] + (up - g[opp]) * irc;
    } else {
      const size_t q = node(dx, dy, dz);
      const real gold = b.gs[i * N + q];
      b.gd[i * N + q] = gold + (gs[i] - gold) * sc[S_IRC * N + q];
    }
  }
  b.Th[N + k] = T1;
  b.Th[k] = Tr;
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
  const double S[19] = {1, p->s_e, p->s_eps, 1, 1, 1, 1, 1, 1, sv, 1, sv, 1, sv, sv, sv, 1, 1, 1};
  for (int r = 0; r < 19; ++r) {
    d.s[r] = (real)S[r];
    d.om[r] = (real)(1.0 - 0.5 * S[r]);
  }
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

template <typename real>
void launch_step3(lbm3d_ctx* h) {
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

lbm_status lbm3d_destroy(lbm3d_ctx* h) {
  if (!h) return LBM_E_INVAL;
  delete h;
  return LBM_OK;
}

}  // extern "C"
