// Device-side pieces of the fused thermal pseudopotential LBM step for gfx950.
//
// Data layout in HBM (structure of arrays, x fastest, so that a wavefront of 64 lanes along
// x reads and writes 64 consecutive values of one population):
//   f[9][ny][nx], g[5][ny][nx]  in two copies A/B (read one, write the other, swap per launch)
//   Th[2][ny][nx]               temperature history T(t-1), T(t-2), also in two copies A/B: a
//                               two-step launch reads the history of its neighbours' nodes,
//                               which must not change under it
//
// Temperature storage: g_i is kept as g_i - what_i T_ref and the history as T - T_ref, with T_ref
// a per-simulation constant (the mean initial temperature).  Relaxation, grad T, the
// rho c_v blend, the second time difference and anti-bounce-back are all invariant under this
// shift; only the EOS and Q use the absolute T = T_ref + sum_i g_i.  In FP32 it keeps the
// resolution of T where it matters (T varies by a few percent around T_ref).
//
// Velocity sets (Eqs. 2 and 26): D2Q9 c_0 = (0,0), c_1..4 = (1,0),(0,1),(-1,0),(0,-1),
// c_5..8 = (1,1),(-1,1),(-1,-1),(1,-1); the D2Q5 set is c_0..c_4 of the same list.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

constexpr int TX = 64;        // tile width  (one wavefront along x)
constexpr int NXCD = 8;       // accelerator complex dies of an MI355X (each with its own L2)
constexpr int HXW = 3;        // halo columns per side (wetting ghost needs rho at radius 3)
constexpr int HYW = 2;        // halo rows per side (psi at radius 2 for div u)
constexpr int EXW = TX + 2 * HXW;

// Workgroup shape of the step kernel: a TX x TY_ tile updated by WAVES_ wavefronts of 64 lanes
// along x, DEPTH_ time steps per launch; each thread owns RPT rows of its column.  A two-step
// launch loads the wide region of MXH columns and MYH rows around the tile (MX x MY cells).
template <int TY_, int WAVES_, int DEPTH_ = 1>
struct Shape {
  static constexpr int TY = TY_;
  static constexpr int WAVES = WAVES_;
  static constexpr int DEPTH = DEPTH_;
  static constexpr int NT = 64 * WAVES_;
  static constexpr int RPT = TY_ / WAVES_;
  static constexpr int EYW = TY_ + 2 * HYW;
  static constexpr int RING = EXW * EYW - TX * TY_;             // halo cells of the load region
  static constexpr int URING = (TX + 2) * (TY_ + 2) - TX * TY_;  // halo cells of the velocity region
  static constexpr int MXH = HXW + 4, MYH = HYW + 3;
  static constexpr int MX = TX + 2 * MXH, MY = TY_ + 2 * MYH;
  static_assert(RPT * WAVES_ == TY_, "rows per thread must divide the tile height");
  static_assert(DEPTH_ == 1 || DEPTH_ == 2, "one or two steps per launch");
};

// error bits of the device error word
constexpr unsigned ERR_RHO = 1u;   // density <= 0 or not finite
constexpr unsigned ERR_T = 2u;     // temperature <= 0 or not finite
constexpr unsigned ERR_PSI = 4u;   // pseudopotential argument < 0

constexpr unsigned FL_FREEZE_FLOW = 1u;
constexpr unsigned FL_NO_S = 2u;
constexpr unsigned FL_BGK = 8u;

// Constants of one simulation, derived once on the host in FP64 and stored in the working
// precision.
template <typename real>
struct DevParams {
  real a, b, R, G, Tc, kappa;       // Peng-Robinson EOS (Eq. 10), interaction strength (Eq. 9)
  real inv_Tc, inv_G;
  real s_e, s_eps, s_q, s_p;        // D2Q9 MRT rates (Eq. 5)
  real corr_e, corr_eps;            // sigma / (1/s - 1/2) of Li's forcing (Eq. 8)
  real cv, wdot, w0h, w1h;          // thermal weights of the rest and axis velocities (Eq. 26)
  real vs1, vs3, vs4, inv_cs2h;     // D2Q5 MRT rates (vs1 = 1/tau_g, also the D2Q9 BGK rate); 1/chat_s^2
  real gx, gy, rho_ave;             // buoyancy
  real T_box, T_top, T_bot, hot_dT, hot_x0, inv_2s2;
  real tan_bot, tan_top;            // tan(pi/2 - theta) of the wetting rule (Eq. 54)
  real T_ref;                       // g and the history are stored relative to T_ref (see below)
  // Derived on the host: without scalar floating-point units, a constant computed in the kernel
  // costs a vector instruction per wavefront, as much as per-node arithmetic.
  real om_e, om_eps, om_q, om_p;    // 1 - s/2 of the forcing term (Eq. 5)
  real opk, GG, two_w1h;            // 1 + kappa; G^2; 2 w_axis
  int y_walls, thermal_box;
  unsigned flags;
  int qg;                           // velocities of the thermal lattice: 5 or 9
  // (after the fields of the D2Q5 path, whose offsets, and so the kernel's scalar loads, they keep)
  real w2h, two_w2h;                // D2Q9 thermal lattice: weight of a diagonal velocity, twice it
  int open_top;                     // with walls: the top is open (outflow boundary)
  // rho_ave of the buoyancy is the current mean density of the domain, read from InstLive at each
  // launch (an open top, where mass leaves and enters); 0: the constant rho_ave above
  int live_rho_ave;
};

// Quantities of one simulation that the device updates as it runs (in its control block).  The
// mass changes only where populations cross an open top; the boundary pass after each step adds
// that flux, so rho_ave follows the mean density of the domain (Section 4.3) without a reduction
// over the grid.
struct InstLive {
  double mass;     // total mass sum(rho), FP64
  double rho_ave;  // mass / (nx ny)
};

// Division by a constant that is fixed per instance, as a multiply-high, an add and two shifts
// (Granlund and Montgomery, division by invariant integers using multiplication, 1994: the
// round-up method for N = 32 bits).  Exact for every 32-bit unsigned numerator; the constants
// come from make_fast_div on the host.  Used where the tile index is split into the tile's column
// and row, which a generic integer division would do with a few dozen scalar instructions.
struct FastDiv {
  unsigned m, s1, s2;
};

__host__ __device__ __forceinline__ unsigned fast_div(unsigned n, FastDiv d) {
  const unsigned t = (unsigned)(((unsigned long long)d.m * n) >> 32);
  return (t + ((n - t) >> d.s1)) >> d.s2;
}

// l = ceil(log2 d); m = floor(2^32 (2^l - d) / d) + 1 (taken modulo 2^32); s1 = min(l, 1);
// s2 = max(l - 1, 0).  d >= 1.
inline FastDiv make_fast_div(unsigned d) {
  unsigned l = 0;
  while (l < 32 && (1ull << l) < d) ++l;
  const unsigned long long two_l = 1ull << l;
  const unsigned m = (unsigned)(((two_l - d) << 32) / d + 1);
  return FastDiv{m, l < 1 ? l : 1u, l > 1 ? l - 1 : 0u};
}

// One simulation as seen by the step kernel.  The step kernel serves single runs (a one-entry
// table) and batches (many entries) with the same code.
template <typename real>
struct InstDesc {
  real* fA;
  real* gA;
  real* fB;
  real* gB;
  real* ThA;
  real* ThB;
  unsigned* err;
  int nx, ny;
  int ntx, nty;        // tiles along x and y
  int strip;           // tile order: strips of this many tile columns (>= ntx: whole rows)
  FastDiv div_band;    // division by strip * nty (tiles in one strip)
  FastDiv div_strip;   // division by the strip width, and by the width of the last strip
  FastDiv div_last;
  int tile_begin;      // first workgroup index of this instance in the launch
  int b_base;          // 1 if the current state is in the B buffers at clock t_base
  int h_base;          // 1 if the temperature history is in ThB at clock t_base
  long long t_base;    // clock value from which launches advance this instance
  long long t_end;     // clock value at which it stops
  InstLive* live;      // mass and current rho_ave (the instance's control block)
  DevParams<real> p;
};

// Step window of a single run passed to a launch by value (use = 1) instead of through the device
// clock and the descriptor: launch k of the call does step t + k DEPTH of the window
// [t_base, t_end), whose first step starts from the B buffers if b_base is 1 (h_base: the
// temperature history).  Graph replays and batches pass use = 0 and read both from memory.
struct LaunchWin {
  long long t, t_base, t_end;
  int b_base, h_base, use;
};

// Pointers into device memory.  The step kernel takes its buffers from a descriptor table in
// memory, so the compiler cannot infer their address space; declaring it makes every access a
// global (not flat) instruction, which does not share the LDS wait counter.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gptr<T> to_global(T* p) {
  return (gptr<T>)p;
}

// Global accesses as (uniform base, 32-bit byte offset per lane): the base lives in scalar
// registers and one vector register carries the offset, so an access costs no vector
// arithmetic.  A plane holds fewer than 2^32 bytes (checked by lbm_validate).
// A base computed by uniform arithmetic is passed through readfirstlane (it already is uniform,
// so this costs two scalar moves), which keeps the compiler from folding the plane offset into a
// 64-bit per-lane address.
template <typename T>
__device__ __forceinline__ gptr<T> sbase(gptr<T> ptr) {
  const unsigned long long v = (unsigned long long)ptr;
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
  return (gptr<T>)(((unsigned long long)hi << 32) | lo);
}
// A uniform value the compiler must take as unknown at each use (an empty asm statement that
// claims to change it).  Plane bases derived from an opaque plane stride are recomputed in
// scalar registers next to their accesses instead of being hoisted and kept live (and spilled to
// vector lanes) across the kernel.
template <typename T>
__device__ __forceinline__ T opaque(T v) {
  asm volatile("" : "+s"(v));
  return v;
}
// Successive planes of one array, first to last: each step adds the (opaque) plane stride to a
// running base, one 64-bit scalar add per plane where base + i * stride takes a 64-bit multiply.
template <typename T>
struct PlaneWalk {
  gptr<T> p;
  ptrdiff_t stride;
  __device__ __forceinline__ gptr<T> next() {
    const gptr<T> b = sbase(p);
    p = p + opaque(stride);
    return b;
  }
};
template <typename real>
__device__ __forceinline__ real ldb(gptr<const char> base, unsigned off) {
  return *(gptr<const real>)(base + off);
}
template <typename real>
__device__ __forceinline__ void stb(gptr<char> base, unsigned off, real v) {
  *(gptr<real>)(base + off) = v;
}

// Reciprocal and square root: hardware instructions (1 ulp) in FP32, IEEE-exact in FP64.
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double fsqrt(double x) { return sqrt(x); }

// Periodic wrap of an index.  On grids at least as large as a tile plus its halo the index is
// less than one period away from [0, n) and one compare with add/subtract suffices; smaller
// grids (flag `tiny`, uniform per launch) take the modulo.
__device__ __forceinline__ int wrapi(int v, int n, bool tiny) {
  if (__builtin_expect(tiny, 0)) {
    v %= n;
    return v < 0 ? v + n : v;
  }
  v = v < 0 ? v + n : v;
  return v >= n ? v - n : v;
}

// Reciprocal square root: hardware instruction in FP32, IEEE-exact in FP64.
__device__ __forceinline__ float frsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double frsqrt(double x) { return 1.0 / sqrt(x); }

// Peng-Robinson pressure (Eq. 10): p = rho R T/(1 - b rho) - a phi(T) rho^2/(1 + 2 b rho - b^2 rho^2),
// phi(T) = s^2, s = 1 + kappa (1 - sqrt(T/Tc)); with it (dp/dT)_rho, where
// dphi/dT = -kappa s / sqrt(T Tc).  One reciprocal square root (sqrt(T/Tc) = T / sqrt(T Tc)) and
// one reciprocal of the product of the two denominators.
template <typename real>
__device__ __forceinline__ void pr_eos(const DevParams<real>& p, real rho, real T, real& press, real& dpdT) {
  const real rs = frsqrt(T * p.Tc);  // 1/sqrt(T Tc)
  const real sq = T * rs;            // sqrt(T/Tc)
  const real s = p.opk - p.kappa * sq;
  const real br = p.b * rho;
  const real den1 = real(1) - br;
  const real den2 = real(1) + br * (real(2) - br);
  const real i12 = rcp(den1 * den2);
  const real rRi1 = rho * p.R * (den2 * i12);       // rho R / (1 - b rho)
  const real t = p.a * s * (rho * rho) * (den1 * i12);  // a s rho^2 / (1 + 2 b rho - b^2 rho^2)
  press = rRi1 * T - s * t;
  dpdT = rRi1 + p.kappa * rs * t;
}

template <typename real>
__device__ __forceinline__ real pr_pressure(const DevParams<real>& p, real rho, real T) {
  real press, dpdT;
  pr_eos(p, rho, T, press, dpdT);
  return press;
}

// Pseudopotential psi = sqrt(2 (p_EOS - rho c_s^2) / G) (text after Eq. 9); flags a negative
// argument.
template <typename real>
__device__ __forceinline__ real psi_from_pressure(const DevParams<real>& p, real rho, real press, unsigned& err) {
  const real arg = real(2) * (press - rho * real(1.0 / 3.0)) * p.inv_G;
  if (!(arg >= real(0))) {
    err |= ERR_PSI;
    return real(0);
  }
  return fsqrt(arg);
}

template <typename real>
__device__ __forceinline__ real pseudo(const DevParams<real>& p, real rho, real T, unsigned& err) {
  return psi_from_pressure(p, rho, pr_pressure(p, rho, T), err);
}

// Wall temperature at column x for a link leaving through the bottom (side 0) or top (side 1).
template <typename real>
__device__ __forceinline__ real wall_temperature(const DevParams<real>& p, int side, int x) {
  if (p.thermal_box) return p.T_box;
  if (side == 0) {
    const real d = real(x) - p.hot_x0;
    return p.T_bot + p.hot_dT * exp(-d * d * p.inv_2s2);
  }
  return p.T_top;
}

}  // namespace lbm
