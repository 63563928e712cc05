// Per-call kernels around the step: initial state, field readout, FP64 diagnostics.
#pragma once
#include "lbm_device.hpp"

namespace lbm {

// f_i = f_i^eq(rho, u) (Eq. 3), g_i = what_i T (Eq. 22), both history levels = T.
// Inputs are FP64 fields staged in device memory: in[0..N) rho, [N..2N) ux, [2N..3N) uy,
// [3N..4N) T.  Thermal weights: w0h (rest), w1h (axes), w2h (diagonals of the D2Q9 thermal
// lattice, qg = 9).
template <typename real>
__global__ void init_kernel(const double* __restrict__ in, real* __restrict__ f, real* __restrict__ g,
                            real* __restrict__ Th, size_t N, int qg, double w0h, double w1h, double w2h,
                            double T_ref) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  const double rho = in[k], ux = in[N + k], uy = in[2 * N + k], T = in[3 * N + k];
  const double uu = ux * ux + uy * uy;
  const double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
  const int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  const int cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const double cu = cx[i] * ux + cy[i] * uy;
    f[i * N + k] = (real)(w[i] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu));
  }
  const double Tr = T - T_ref;  // stored relative to T_ref
  g[k] = (real)(w0h * Tr);
#pragma unroll
  for (int i = 1; i < 5; ++i) g[i * N + k] = (real)(w1h * Tr);
  if (qg == 9) {
#pragma unroll
    for (int i = 5; i < 9; ++i) g[i * N + k] = (real)(w2h * Tr);
  }
  Th[k] = (real)Tr;
  Th[N + k] = (real)Tr;
}

// rho and T - T_ref at a fluid node (already wrapped), summed in the order of the step kernel
template <typename real>
__device__ __forceinline__ void rho_T(const real* __restrict__ f, const real* __restrict__ g, size_t N, int o,
                                      int qg, real& rho, real& Tr) {
  rho = ((f[o] + f[N + o]) + (f[2 * N + o] + f[3 * N + o])) +
        ((f[4 * N + o] + f[5 * N + o]) + (f[6 * N + o] + f[7 * N + o])) + f[8 * N + o];
  if (qg == 9)
    Tr = ((g[o] + g[N + o]) + (g[2 * N + o] + g[3 * N + o])) +
         ((g[4 * N + o] + g[5 * N + o]) + (g[6 * N + o] + g[7 * N + o])) + g[8 * N + o];
  else
    Tr = ((g[o] + g[N + o]) + (g[2 * N + o] + g[3 * N + o])) + g[4 * N + o];
}

// psi at (x, y) with wrapping and, in walled domains, the wetting ghost rows (Eq. 54)
template <typename real>
__device__ real psi_any(const DevParams<real>& p, const real* __restrict__ f, const real* __restrict__ g, int nx,
                        int ny, size_t N, int x, int y, unsigned& err) {
  x = wrapi(x, nx, true);
  if (!p.y_walls) y = wrapi(y, ny, true);
  real rho, T;
  if (y == ny && p.open_top) {
    rho_T(f, g, N, (ny - 1) * nx + x, p.qg, rho, T);  // above an open top: zero gradient
    T = p.T_ref + T;
  } else if (y == -1 || y == ny) {
    const int top = y == ny;
    const int y1 = top ? ny - 1 : 0, y2 = top ? ny - 2 : 1;
    real r2, r1p, r1m, tt;
    rho_T(f, g, N, y2 * nx + x, p.qg, r2, tt);
    rho_T(f, g, N, y1 * nx + wrapi(x + 1, nx, true), p.qg, r1p, tt);
    rho_T(f, g, N, y1 * nx + wrapi(x - 1, nx, true), p.qg, r1m, tt);
    rho = r2 + (top ? p.tan_top : p.tan_bot) * fabs(r1p - r1m);
    T = wall_temperature(p, top, x);
  } else {
    rho_T(f, g, N, y * nx + x, p.qg, rho, T);
    T = p.T_ref + T;
  }
  return pseudo(p, rho, T, err);
}

// rho, u (with half the force of the current state, Eq. 11; the buoyancy with the current rho_ave)
// and T to FP64 staging:
// out[0..N) rho, [N..2N) ux, [2N..3N) uy, [3N..4N) T.
template <typename real>
__global__ void fields_kernel(DevParams<real> p, const InstLive* __restrict__ live, const real* __restrict__ f,
                              const real* __restrict__ g, int nx, int ny, double* __restrict__ out,
                              unsigned* __restrict__ errw) {
  const size_t N = (size_t)nx * ny;
  if (p.live_rho_ave) p.rho_ave = (real)live->rho_ave;  // the current mean density (open top)
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  const int x = (int)(k % nx), y = (int)(k / nx);
  unsigned err = 0u;
  const int o = (int)k;
  real rho, Tr;
  rho_T(f, g, N, o, p.qg, rho, Tr);
  real jx = (f[N + o] - f[3 * N + o]) + ((f[5 * N + o] - f[6 * N + o]) + (f[8 * N + o] - f[7 * N + o]));
  real jy = (f[2 * N + o] - f[4 * N + o]) + ((f[5 * N + o] + f[6 * N + o]) - (f[7 * N + o] + f[8 * N + o]));
  real fx = real(0), fy = real(0);
  if (!(p.flags & FL_FREEZE_FLOW)) {
    const real pc = psi_any(p, f, g, nx, ny, N, x, y, err);
    const real pE = psi_any(p, f, g, nx, ny, N, x + 1, y, err), pW = psi_any(p, f, g, nx, ny, N, x - 1, y, err);
    const real pN = psi_any(p, f, g, nx, ny, N, x, y + 1, err), pS = psi_any(p, f, g, nx, ny, N, x, y - 1, err);
    const real pNE = psi_any(p, f, g, nx, ny, N, x + 1, y + 1, err);
    const real pNW = psi_any(p, f, g, nx, ny, N, x - 1, y + 1, err);
    const real pSW = psi_any(p, f, g, nx, ny, N, x - 1, y - 1, err);
    const real pSE = psi_any(p, f, g, nx, ny, N, x + 1, y - 1, err);
    const real sx = real(1.0 / 3.0) * (pE - pW) + real(1.0 / 12.0) * ((pNE - pNW) + (pSE - pSW));
    const real sy = real(1.0 / 3.0) * (pN - pS) + real(1.0 / 12.0) * ((pNE + pNW) - (pSE + pSW));
    fx = -p.G * pc * sx + (rho - p.rho_ave) * p.gx;
    fy = -p.G * pc * sy + (rho - p.rho_ave) * p.gy;
  }
  out[k] = (double)rho;
  out[N + k] = (double)((jx + real(0.5) * fx) / rho);
  out[2 * N + k] = (double)((jy + real(0.5) * fy) / rho);
  out[3 * N + k] = (double)p.T_ref + (double)Tr;
  if (err) atomicOr(errw, err);
}

// Vapour count per row for the bubble-departure readout: one workgroup per row y of the chunk
// [y0, y0 + gridDim.x), counting the columns x of [x_lo, x_lo + width) (taken modulo nx) whose
// density, summed in the working precision exactly as for the field readout, is below thr.
constexpr int VAP_NT = 256;

template <typename real>
__global__ __launch_bounds__(VAP_NT) void vapour_rows_kernel(const real* __restrict__ f, int nx, size_t N, int y0,
                                                             int x_lo, int width, real thr, int* __restrict__ counts) {
  __shared__ int part[VAP_NT / 64];
  const int y = y0 + blockIdx.x;
  int c = 0;
  for (int i = threadIdx.x; i < width; i += VAP_NT) {
    const int x = wrapi(x_lo + i, nx, true);
    const int o = y * nx + x;
    const real rho = ((f[o] + f[N + o]) + (f[2 * N + o] + f[3 * N + o])) +
                     ((f[4 * N + o] + f[5 * N + o]) + (f[6 * N + o] + f[7 * N + o])) + f[8 * N + o];
    c += rho < thr ? 1 : 0;
  }
  for (int s = 32; s > 0; s >>= 1) c += __shfl_down(c, s, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < VAP_NT / 64; ++w) t += part[w];
    counts[blockIdx.x] = t;
  }
}

// Vapour components for the bubble-departure readout of Section 4.3: the connected sets of
// nodes in rows [y_lo, y_lo + rows) whose density (summed in the working precision as for the
// field readout, compared in FP64) is below a threshold, 8-connected, periodic in x.  The label
// array has one int per node of the rows, indexed k = (y - y_lo) nx + x:
//   -1            not vapour;
//   0 <= p <= k   a vapour node whose parent is p (p = k: a root).
// Union-find: every link goes from a root to a smaller index with an atomic minimum, so a root is
// always the smallest index of its tree and the final roots do not depend on the order in which
// the links were made.  Parents only decrease, so every walk to a root ends.
constexpr int CC_NT = 256;

struct CompStat {  // per component: integer sums and bounds, so atomics give order-free results
  int root, area, y_min, y_max, x_min, x_max;
  unsigned long long y_sum;
};

__device__ __forceinline__ int cc_load(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of node k, halving the path on the way: each visited node is pointed at its grandparent (an
// ancestor, so the node stays in its tree; an atomic minimum, so parents still only decrease).
// Every iteration moves k to a strictly smaller index, so the walk ends.
__device__ __forceinline__ int cc_find(int* lab, int k) {
  for (;;) {
    const int p = cc_load(lab + k);
    if (p == k) return k;
    const int gp = cc_load(lab + p);
    if (gp == p) return p;
    atomicMin(lab + k, gp);
    k = gp;
  }
}

// Join the trees of vapour nodes a and b.  A failed link (the root a got a parent meanwhile)
// retries from that parent, so the larger root strictly decreases from one try to the next.
__device__ void cc_union(int* lab, int a, int b) {
  for (;;) {
    a = cc_find(lab, a);
    b = cc_find(lab, b);
    if (a == b) return;
    if (a < b) {
      const int t = a;
      a = b;
      b = t;
    }
    const int old = atomicMin(lab + a, b);
    if (old == a) return;
    a = old;
  }
}

template <typename real>
__global__ __launch_bounds__(CC_NT) void cc_init_kernel(const real* __restrict__ f, int nx, size_t N, int y_lo,
                                                        int n, double thr, int* __restrict__ lab) {
  const int k = blockIdx.x * CC_NT + threadIdx.x;
  if (k >= n) return;
  const int o = y_lo * nx + k;
  const real rho = ((f[o] + f[N + o]) + (f[2 * N + o] + f[3 * N + o])) +
                   ((f[4 * N + o] + f[5 * N + o]) + (f[6 * N + o] + f[7 * N + o])) + f[8 * N + o];
  lab[k] = (double)rho < thr ? k : -1;
}

// Each vapour node joins its vapour neighbours east, north-west, north and north-east (the other
// four directions are the same pairs seen from the other node).
__global__ __launch_bounds__(CC_NT) void cc_union_kernel(int* __restrict__ lab, int nx, int rows) {
  const int k = blockIdx.x * CC_NT + threadIdx.x;
  if (k >= nx * rows || cc_load(lab + k) < 0) return;
  const int x = k % nx, r = k / nx;
  const int xe = x + 1 == nx ? 0 : x + 1, xw = x == 0 ? nx - 1 : x - 1;
  const int nb[4] = {r * nx + xe, (r + 1) * nx + xw, (r + 1) * nx + x, (r + 1) * nx + xe};
  const int cnt = r + 1 < rows ? 4 : 1;
  for (int j = 0; j < cnt; ++j)
    if (cc_load(lab + nb[j]) >= 0) cc_union(lab, k, nb[j]);
}

// Every vapour node points at its root.
__global__ __launch_bounds__(CC_NT) void cc_flatten_kernel(int* __restrict__ lab, int n) {
  const int k = blockIdx.x * CC_NT + threadIdx.x;
  if (k >= n || cc_load(lab + k) < 0) return;
  __hip_atomic_store(lab + k, cc_find(lab, k), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Each root takes a slot of the table (in no particular order; the host sorts by root) and
// stores -2 - slot in its label; slots beyond cap are counted but not kept.
__global__ __launch_bounds__(CC_NT) void cc_number_kernel(int* __restrict__ lab, int n, int y_lo_nx,
                                                          int* __restrict__ count, CompStat* __restrict__ tab,
                                                          int cap) {
  const int k = blockIdx.x * CC_NT + threadIdx.x;
  if (k >= n || lab[k] != k) return;
  const int id = atomicAdd(count, 1);
  if (id < cap) {
    CompStat c;
    c.root = y_lo_nx + k;
    c.area = 0;
    c.y_min = 0x7fffffff;
    c.y_max = -1;
    c.x_min = 0x7fffffff;
    c.x_max = -1;
    c.y_sum = 0ull;
    tab[id] = c;
  }
  lab[k] = -2 - (id < cap ? id : cap);
}

// Per-component statistics.  Integer atomics make the result independent of their order, but many
// atomics on one address serialise: a component of a million nodes took milliseconds.  So a
// wavefront whose labelled lanes all belong to one component first combines their values with
// cross-lane butterflies and one lane updates the table; mixed wavefronts update it lane by lane.
// Every thread stays to the end (the butterflies read all 64 lanes).
__global__ __launch_bounds__(CC_NT) void cc_stats_kernel(const int* __restrict__ lab, int nx, int n, int y_lo,
                                                         CompStat* __restrict__ tab, int cap) {
  const int k = blockIdx.x * CC_NT + threadIdx.x;
  int id = -1;
  if (k < n) {
    const int v = lab[k];
    if (v != -1) {
      id = v <= -2 ? -2 - v : -2 - lab[v];
      if (id >= cap) id = -1;
    }
  }
  const int x = k < n ? k % nx : 0, y = k < n ? y_lo + k / nx : 0;
  const unsigned long long has = __ballot(id >= 0);
  if (has == 0ull) return;  // uniform: the whole wavefront leaves together
  const int lead = __builtin_amdgcn_readlane(id, __builtin_ctzll(has));
  if (__ballot(id >= 0 && id != lead) == 0ull) {
    const bool mine = id >= 0;
    int area = mine ? 1 : 0, y0 = mine ? y : 0x7fffffff, y1 = mine ? y : -1;
    int x0 = mine ? x : 0x7fffffff, x1 = mine ? x : -1;
    unsigned long long ys = mine ? (unsigned long long)y : 0ull;
#pragma unroll
    for (int s = 32; s > 0; s >>= 1) {
      area += __shfl_xor(area, s, 64);
      y0 = min(y0, __shfl_xor(y0, s, 64));
      y1 = max(y1, __shfl_xor(y1, s, 64));
      x0 = min(x0, __shfl_xor(x0, s, 64));
      x1 = max(x1, __shfl_xor(x1, s, 64));
      ys += __shfl_xor(ys, s, 64);
    }
    if ((int)(threadIdx.x & 63u) == __builtin_ctzll(has)) {
      CompStat& c = tab[lead];
      atomicAdd(&c.area, area);
      atomicMin(&c.y_min, y0);
      atomicMax(&c.y_max, y1);
      atomicMin(&c.x_min, x0);
      atomicMax(&c.x_max, x1);
      atomicAdd(&c.y_sum, ys);
    }
    return;
  }
  if (id < 0) return;
  CompStat& c = tab[id];
  atomicAdd(&c.area, 1);
  atomicMin(&c.y_min, y);
  atomicMax(&c.y_max, y);
  atomicMin(&c.x_min, x);
  atomicMax(&c.x_max, x);
  atomicAdd(&c.y_sum, (unsigned long long)y);
}

// Deterministic FP64 sums of rho and rho c_v T (mass and thermal energy).  Three levels, each in a
// fixed order: a thread adds its nodes of the workgroup's contiguous range; a wavefront adds its
// 64 lanes by a butterfly of cross-lane shuffles (every lane ends with the same sum, the two
// operands of each addition being the same values in either order); the workgroup's wavefronts
// are added in index order from LDS.  A second single-workgroup pass adds the per-workgroup
// partials the same way.  The result depends only on N and the range split, not on scheduling.
constexpr int RED_NT = 256;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int s = 32; s > 0; s >>= 1) v += __shfl_xor(v, s, 64);
  return v;
}

// Sum over the workgroup of (m, e); the result is valid in thread 0.
__device__ __forceinline__ void block_sum2(double& m, double& e) {
  __shared__ double wm[RED_NT / 64], we[RED_NT / 64];
  m = wave_sum(m);
  e = wave_sum(e);
  const int w = (int)threadIdx.x >> 6;
  if ((threadIdx.x & 63u) == 0u) {
    wm[w] = m;
    we[w] = e;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    m = wm[0];
    e = we[0];
#pragma unroll
    for (int k = 1; k < RED_NT / 64; ++k) {
      m += wm[k];
      e += we[k];
    }
  }
}

template <typename real>
__global__ __launch_bounds__(RED_NT) void diag_partial_kernel(const real* __restrict__ f, const real* __restrict__ g,
                                                              size_t N, int qg, double cv, double T_ref,
                                                              size_t per_block, double* __restrict__ partials) {
  const size_t begin = (size_t)blockIdx.x * per_block;
  const size_t end = begin + per_block < N ? begin + per_block : N;
  double m = 0.0, e = 0.0;
  for (size_t k = begin + threadIdx.x; k < end; k += RED_NT) {
    real rho, Tr;
    rho_T(f, g, N, (int)k, qg, rho, Tr);
    m += (double)rho;
    e += (double)rho * cv * (T_ref + (double)Tr);
  }
  block_sum2(m, e);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = m;
    partials[2 * blockIdx.x + 1] = e;
  }
}

// One diagnostics record: the step count it belongs to, mass and energy.
struct DiagRecord {
  long long step;
  double mass;
  double energy;
};

// Adds the partials; writes mass and energy to out[0], out[1] and, if rec is not null, the record
// (step, mass, energy) to *rec.
__global__ __launch_bounds__(RED_NT) void diag_final_kernel(const double* __restrict__ partials, int nparts,
                                                            double* __restrict__ out, DiagRecord* __restrict__ rec,
                                                            long long step) {
  double m = 0.0, e = 0.0;
  for (int k = threadIdx.x; k < nparts; k += RED_NT) {
    m += partials[2 * k];
    e += partials[2 * k + 1];
  }
  block_sum2(m, e);
  if (threadIdx.x == 0) {
    out[0] = m;
    out[1] = e;
    if (rec) *rec = DiagRecord{step, m, e};
  }
}

}  // namespace lbm
