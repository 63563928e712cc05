// Host runtime and C ABI of the thermal pseudopotential LBM library (declared in include/lbm.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "lbm.h"
#include "host_range.hpp"
#include "lbm_aux.hpp"
#include "lbm_step.hpp"
#include "lbm_persist.hpp"

using namespace lbm;

namespace {

constexpr size_t ALIGN = 256;
constexpr size_t CTRL_BYTES = 16384;  // descriptor, clock, error word, diagnostics result
constexpr int MAX_RED_BLOCKS = 2048;
constexpr int GRAPH_STEPS = 64;       // steps captured per replayed graph

size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

// offsets inside the control block
constexpr size_t OFF_DESC = 0;        // InstDesc<real> (single-run table)
constexpr size_t OFF_CLOCK = 4096;    // long long
constexpr size_t OFF_ERR = 4352;      // unsigned
constexpr size_t OFF_DIAG = 4608;     // 2 doubles
constexpr size_t OFF_LIVE = 4864;     // InstLive: FP64 mass and the current rho_ave
constexpr size_t OFF_RING = 8192;     // ring of DIAG_RING diagnostics records (every-k diagnostics)
constexpr int DIAG_RING = 256;
static_assert(OFF_RING + DIAG_RING * sizeof(DiagRecord) <= CTRL_BYTES, "control block layout");
// the reduction partials follow the control block

size_t partial_bytes() { return align_up((size_t)MAX_RED_BLOCKS * 2 * sizeof(double)); }

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

double pr_kappa(const lbm_params* p) {
  const double w = p->acentric;
  return 0.37464 + 1.54226 * w - 0.26992 * w * w;
}

// ---- tile shapes compiled into the library (tile height, wavefronts, steps per launch), per
// precision
struct ShapeDef {
  int ty, waves, depth;
};
#define LBM_SHAPE_DEF(k, ty, w, d) {ty, w, d},
constexpr ShapeDef F32_SHAPES[] = {LBM_F32_SHAPES(LBM_SHAPE_DEF)};
constexpr ShapeDef F64_SHAPES[] = {LBM_F64_SHAPES(LBM_SHAPE_DEF)};
#undef LBM_SHAPE_DEF
constexpr int N_F32_SHAPES = (int)(sizeof(F32_SHAPES) / sizeof(F32_SHAPES[0]));
constexpr int N_F64_SHAPES = (int)(sizeof(F64_SHAPES) / sizeof(F64_SHAPES[0]));

int shape_count(int precision) { return precision == LBM_FP64 ? N_F64_SHAPES : N_F32_SHAPES; }
const ShapeDef& shape_def(int precision, int k) { return precision == LBM_FP64 ? F64_SHAPES[k] : F32_SHAPES[k]; }
int tiles_of(int nx, int ny, int ty) { return ((nx + TX - 1) / TX) * ((ny + ty - 1) / ty); }

// Velocities of the thermal lattice of a parameter set (5 or 9).
int qg_of(const lbm_params* p) { return p->thermal_q == 9 ? 9 : 5; }

// Whether a simulation can use the two-step shapes: their LDS holds the D2Q5 thermal
// populations, and an open top needs its boundary pass between steps.
bool two_step_ok(const lbm_params* p) { return qg_of(p) == 5 && !(p->y_walls && p->open_top); }

// A two-step shape keeps a consistent image of its wide halo region in LDS only if no grid node
// appears in it twice: the grid must be larger than the region in both directions.
bool shape_fits(int precision, bool two_ok, int k, int nx, int ny) {
  const ShapeDef& d = shape_def(precision, k);
  if (d.depth == 1) return true;
  if (!two_ok) return false;
  return nx >= TX + 2 * (HXW + 4) + 1 && ny >= d.ty + 2 * (HYW + 3) + 1;
}

// Shape used when none is requested.  FP32: the two-step 64 x 16 shape where the grid is
// large enough for it (it halves the HBM traffic and the fixed cost of a launch per step);
// otherwise the 1-row-per-thread shape while the grid has fewer tiles than about four per compute
// unit (a single wave of workgroups, whose latency matters), the 2-rows-per-thread shape beyond.
// The autotuner replaces this guess by a measurement.
constexpr int F32_TWO_STEP_DEFAULT = 6;
int default_shape(int precision, bool two_ok, int nx, int ny) {
  if (precision == LBM_FP64) return 0;
  if (shape_fits(precision, two_ok, F32_TWO_STEP_DEFAULT, nx, ny)) return F32_TWO_STEP_DEFAULT;
  return tiles_of(nx, ny, F32_SHAPES[0].ty) >= 1024 ? 1 : 0;
}

}  // namespace

struct lbm_ctx {
  lbm_params prm{};
  hipStream_t stream = nullptr;
  int device = 0;
  char* base = nullptr;  // caller memory
  size_t bytes = 0;
  size_t N = 0;
  size_t rsz = 4;        // bytes per real
  void* fA = nullptr;
  void* gA = nullptr;
  void* fB = nullptr;
  void* gB = nullptr;
  void* ThA = nullptr;
  void* ThB = nullptr;
  long long* d_clock = nullptr;
  unsigned* d_err = nullptr;
  double* d_diag = nullptr;
  double* d_part = nullptr;
  InstLive* d_live = nullptr;
  void* d_desc = nullptr;
  InstDesc<float> desc32{};
  InstDesc<double> desc64{};
  bool initialised = false;
  bool failed = false;
  int64_t steps = 0;
  int64_t batch_unsynced = 0;  // steps a batch has enqueued for this member since its last lbm_batch_sync
  int gen = 0;           // 1 if the current state is in the B buffers
  int hgen = 0;          // 1 if the temperature history is in ThB (it moves only on two-step launches)
  long long clock = 0;   // host mirror of the context's device clock (advanced by its own launches)
  double rho_ave = 0.0;  // rho_ave of the buoyancy at init (constant unless it follows the mean)
  double T_ref = 0.0;  // storage offset of g and the history (exact in the working precision)
  int shape_req = -1;  // requested tile shape (-1: chosen from the grid size)
  int order_req = 0;   // requested tile order (0: chosen from the grid size, 1: whole rows, k: strips of k)
  int shape = 0;       // tile shape in use
  int ntiles = 0;
  InstLive live0{};      // staging of the live values written at init / load (outlives the copy)
  DiagRecord* d_ring = nullptr;  // every-k diagnostics records (control block)
  int64_t diag_every = 0;        // 0: no periodic diagnostics
  int64_t diag_enqueued = 0;     // records enqueued since lbm_set_diagnostics_interval
  int64_t diag_read = 0;         // records returned by lbm_read_diagnostics_log
  hipGraphExec_t graph = nullptr;
  std::string last_error;
};

struct lbm_batch {
  std::vector<lbm_ctx*> ctx;
  std::vector<int64_t> remaining;
  std::vector<int64_t> pending;  // steps enqueued since the last sync, per instance
  std::vector<int64_t> pending_launches;  // launches that advanced each instance since the last sync
  std::vector<int64_t> pending_hmoves;    // of these, launches that moved its temperature history
  hipStream_t stream = nullptr;
  int precision = 0;
  int qg = 5;                    // thermal lattice of every member
  char* base = nullptr;
  size_t bytes = 0;
  void* d_table = nullptr;
  long long* d_clock = nullptr;
  long long clock = 0;           // host mirror of the device clock
  int total_tiles = 0;
  int shape = -1;                // tile shape of the batched launches (-1: from the first context)
  hipGraphExec_t graph = nullptr;
  std::vector<lbm_ctx*> graph_layout;  // active instances (in table order) the graph was captured for
  int graph_shape = -1;                // tile shape the graph was captured with
  int noalloc_device = -1;             // device whose static batch area the table uses (-1: caller memory)
  GridBar* d_bar = nullptr;            // grid barrier of the persistent launches (batch memory)
  bool persistent = false;             // launches as one persistent kernel per group of steps
  bool persistent_used = false;        // a persistent launch has been enqueued since the last sync
  unsigned spin_limit = 1u << 24;      // bounded wait of the persistent kernel's grid barrier
  int pgrid = 0, pgrid_shape = -1;     // resident workgroups of the persistent kernel (for shape)
  int64_t diag_every = 0;              // members' diagnostics every this many batch steps (0: none)
  int64_t diag_since = 0;              // batch steps since the last such record
  std::vector<char> moved;             // per member: advanced since its last such record
};

// Orders the batch stream after every member's stream: one event recorded on each distinct
// member stream and waited for on the batch stream.
static hipError_t wait_for_members(hipStream_t bs, const std::vector<lbm_ctx*>& ctx) {
  hipEvent_t ev;
  hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
  if (e != hipSuccess) return e;
  std::vector<hipStream_t> seen;
  for (const lbm_ctx* h : ctx) {
    if (e != hipSuccess) break;
    if (h->stream == bs || std::find(seen.begin(), seen.end(), h->stream) != seen.end()) continue;
    seen.push_back(h->stream);
    e = hipEventRecord(ev, h->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(bs, ev, 0);
  }
  const hipError_t d = hipEventDestroy(ev);
  return e != hipSuccess ? e : d;
}

// Default shape of a batch: the two-step shape if every member fits it, else by total size.
static int batch_default_shape(int precision, const std::vector<lbm_ctx*>& ctx) {
  if (precision == LBM_FP64) return 0;
  bool fit = true;
  long long tiles = 0;
  for (const lbm_ctx* h : ctx) {
    fit = fit && shape_fits(precision, two_step_ok(&h->prm), F32_TWO_STEP_DEFAULT, h->prm.nx, h->prm.ny);
    tiles += tiles_of(h->prm.nx, h->prm.ny, F32_SHAPES[0].ty);
  }
  if (fit) return F32_TWO_STEP_DEFAULT;
  return tiles >= 1024 ? 1 : 0;
}

// ------------------------------------------------------------------------------ helpers
static lbm_status fail(lbm_ctx* h, lbm_status s, const std::string& msg) {
  if (h) h->last_error = msg;
  return s;
}

// A member of a batch whose steps have not been brought up to date by lbm_batch_sync: its buffer
// parities are not known on the host, so nothing may read or advance it on its own.
static lbm_status unsynced(lbm_ctx* h, const char* call) {
  return fail(h, LBM_E_STATE, std::string(call) + ": the context has batched steps not yet synchronised (lbm_batch_sync)");
}

#define HIP_OR_FAIL(h, call)                                                               \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail((h), LBM_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Launches of a window of n steps at d steps per launch that move the temperature history to the
// other copy: those that do two steps (a one-step launch updates it in place)
static int64_t history_moves(int64_t n, int d) { return d == 2 ? n / 2 : 0; }

template <typename real>
static DevParams<real> derive(const lbm_params* p, double rho_ave, double T_ref) {
  DevParams<real> d{};
  const double Tc = lbm_critical_temperature(p);
  d.a = (real)p->a;
  d.b = (real)p->b;
  d.R = (real)p->R;
  d.G = (real)p->G;
  d.Tc = (real)Tc;
  d.inv_Tc = (real)(1.0 / Tc);
  d.inv_G = (real)(1.0 / p->G);
  d.kappa = (real)pr_kappa(p);
  d.s_e = (real)p->s_e;
  d.s_eps = (real)p->s_eps;
  d.s_q = (real)p->s_q;
  d.s_p = (real)(1.0 / (3.0 * p->nu + 0.5));
  d.corr_e = (real)(p->sigma / (1.0 / p->s_e - 0.5));
  d.corr_eps = (real)(p->sigma / (1.0 / p->s_eps - 0.5));
  d.cv = (real)p->cv;
  d.qg = qg_of(p);
  // thermal lattice weights, sound speed and the rate tied to lambda (Eqs. 26 and 53; for D2Q9
  // the D2Q9 weights with chat_s^2 = 1/3)
  const double cs2h = d.qg == 9 ? 1.0 / 3.0 : p->wdot / 2.0;
  const double vs1 = 1.0 / (p->lambda / cs2h + 0.5);
  d.wdot = (real)p->wdot;
  d.w0h = (real)(d.qg == 9 ? 4.0 / 9.0 : 1.0 - p->wdot);
  d.w1h = (real)(d.qg == 9 ? 1.0 / 9.0 : p->wdot / 4.0);
  d.w2h = (real)(d.qg == 9 ? 1.0 / 36.0 : 0.0);
  d.vs1 = (real)vs1;
  // BGK (Eq. 21) on D2Q5 is the MRT step with every rate 1/tau_g
  const bool bgk = (p->flags & LBM_BGK) != 0;
  d.vs3 = (real)(bgk ? vs1 : p->vs3);
  d.vs4 = (real)(bgk ? vs1 : p->vs4);
  d.inv_cs2h = (real)(1.0 / cs2h);
  d.gx = (real)p->gx;
  d.gy = (real)p->gy;
  d.rho_ave = (real)rho_ave;
  d.T_box = (real)p->T_box;
  d.T_top = (real)p->T_top;
  d.T_bot = (real)p->T_bot;
  const bool bump = p->hot_sigma > 0.0;
  d.hot_dT = (real)(bump ? p->hot_dT : 0.0);
  d.hot_x0 = (real)p->hot_x0;
  d.inv_2s2 = (real)(bump ? 1.0 / (2.0 * p->hot_sigma * p->hot_sigma) : 0.0);
  d.tan_bot = (real)std::tan(M_PI / 2.0 - p->theta_bot_deg * M_PI / 180.0);
  d.tan_top = (real)std::tan(M_PI / 2.0 - p->theta_top_deg * M_PI / 180.0);
  d.y_walls = p->y_walls ? 1 : 0;
  d.thermal_box = p->thermal_box ? 1 : 0;
  d.open_top = (p->y_walls && p->open_top) ? 1 : 0;
  // where mass crosses an open top, rho_ave (when not given) follows the domain's mean density
  d.live_rho_ave = (d.open_top && std::isnan(p->rho_ave)) ? 1 : 0;
  d.flags = p->flags;
  d.T_ref = (real)T_ref;
  d.om_e = (real)(1.0 - 0.5 * p->s_e);
  d.om_eps = (real)(1.0 - 0.5 * p->s_eps);
  d.om_q = (real)(1.0 - 0.5 * p->s_q);
  d.om_p = (real)(1.0 - 0.5 / (3.0 * p->nu + 0.5));
  d.opk = (real)(1.0 + pr_kappa(p));
  d.GG = (real)(p->G * p->G);
  d.two_w1h = (real)(d.qg == 9 ? 2.0 / 9.0 : p->wdot / 2.0);
  d.two_w2h = (real)(d.qg == 9 ? 2.0 / 36.0 : 0.0);
  return d;
}

static int resident_per_cu(int precision, int qg, int shape);

// Tile columns per strip of the tile order (see tile_position): as requested, or by default strips
// of 8 tiles where a row of tiles is at least half as wide as the number of workgroups an XCD runs
// at once (its compute units times the kernel's resident workgroups per unit): with whole rows, the
// rows of tiles above and below a tile, whose halo it reads, are then too far apart in time for the
// XCD's L2 to still hold them.  Measured on 64 x 16 two-step tiles (one workgroup per compute unit):
// 4096^2 -10 %, 2048^2 -6 %, 1024 x 2048 -3 % per step; on 64 x 8 one-step tiles (three per unit):
// 4096^2 -10 %, but 2048^2 and 1024 x 2048, whose rows fit, +4 to +6 %.
constexpr int DEFAULT_STRIP = 8;
static int tile_strip(const lbm_ctx* h, int ntx, int shape) {
  if (h->order_req == 1) return ntx;
  if (h->order_req >= 2) return std::min(h->order_req, ntx);
  int cus = 256;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device);
  const int per_xcd = resident_per_cu(h->prm.precision, qg_of(&h->prm), shape) * cus / NXCD;
  return 2 * ntx >= per_xcd ? std::min(DEFAULT_STRIP, ntx) : ntx;
}

template <typename real>
static InstDesc<real> make_desc(lbm_ctx* h, int shape) {
  const int ty = shape_def(h->prm.precision, shape).ty;
  InstDesc<real> D{};
  D.fA = (real*)h->fA;
  D.gA = (real*)h->gA;
  D.fB = (real*)h->fB;
  D.gB = (real*)h->gB;
  D.ThA = (real*)h->ThA;
  D.ThB = (real*)h->ThB;
  D.err = h->d_err;
  D.nx = h->prm.nx;
  D.ny = h->prm.ny;
  D.ntx = (h->prm.nx + TX - 1) / TX;
  D.nty = (h->prm.ny + ty - 1) / ty;
  D.strip = tile_strip(h, D.ntx, shape);
  const int nstrips = (D.ntx + D.strip - 1) / D.strip;
  D.div_band = make_fast_div((unsigned)(D.strip * D.nty));
  D.div_strip = make_fast_div((unsigned)D.strip);
  D.div_last = make_fast_div((unsigned)(D.ntx - (nstrips - 1) * D.strip));
  D.tile_begin = 0;
  D.b_base = 0;
  D.h_base = 0;
  D.t_base = 0;
  D.t_end = std::numeric_limits<long long>::max();
  D.live = h->d_live;
  D.p = derive<real>(&h->prm, h->rho_ave, h->T_ref);
  return D;
}

static lbm_status check_device_error(lbm_ctx* h) {
  unsigned e = 0;
  HIP_OR_FAIL(h, hipMemcpyAsync(&e, h->d_err, sizeof(unsigned), hipMemcpyDeviceToHost, h->stream));
  HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
  if (e) {
    h->failed = true;
    std::string m = "numerical failure on the device:";
    if (e & ERR_RHO) m += " density not positive/finite;";
    if (e & ERR_T) m += " temperature not positive/finite;";
    if (e & ERR_PSI) m += " pseudopotential argument negative (density above the EOS limit);";
    return fail(h, LBM_E_NUMERIC, m);
  }
  return LBM_OK;
}

static bool set_device(lbm_ctx* h) {
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return false;
  if (cur != h->device) return hipSetDevice(h->device) == hipSuccess;
  return true;
}

// One launch of the step kernel of tile shape S and thermal lattice QG over `grid` workgroups.
// Two-step shapes exist for the D2Q5 lattice only (shape_fits keeps the others from here).
template <typename real, class S>
static void launch_shape(int qg, int grid, hipStream_t st, const void* table, int ninst, const long long* clk,
                         int k, const LaunchWin& w) {
  const InstDesc<real>* t = (const InstDesc<real>*)table;
  if (qg == 9) {
    if constexpr (S::DEPTH == 1) step_kernel<real, S, 9><<<grid, S::NT, 0, st>>>(t, ninst, clk, k, w);
  } else {
    step_kernel<real, S, 5><<<grid, S::NT, 0, st>>>(t, ninst, clk, k, w);
  }
}

// Window of launches that read the device clock and the descriptors (graph replays, batches).
constexpr LaunchWin FROM_CLOCK{0, 0, 0, 0, 0, 0};

// Persistent kernel of shape S: one launch of nl launch steps, or (grid = 0) the number of its
// workgroups that fit on one compute unit at once.
template <typename real, class S>
static int persist_shape(int qg, int grid, hipStream_t st, const void* table, int ninst, const long long* clk,
                         int total_tiles, int nl, int open, GridBar* bar, unsigned spin) {
  const InstDesc<real>* t = (const InstDesc<real>*)table;
  int nb = 0;
  if (qg == 9) {
    if constexpr (S::DEPTH == 1) {
      if (grid == 0) (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, persist_kernel<real, S, 9>, S::NT, 0);
      else persist_kernel<real, S, 9><<<grid, S::NT, 0, st>>>(t, ninst, clk, total_tiles, nl, open, bar, spin);
    }
  } else {
    if (grid == 0) (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, persist_kernel<real, S, 5>, S::NT, 0);
    else persist_kernel<real, S, 5><<<grid, S::NT, 0, st>>>(t, ninst, clk, total_tiles, nl, open, bar, spin);
  }
  return nb;
}

// Workgroups of the step kernel of a shape that fit on one compute unit at once (from the kernel's
// occupancy; 1 if it cannot be queried), cached per precision, thermal lattice and shape.
template <typename real, class S>
static int step_occupancy(int qg) {
  int nb = 0;
  if (qg == 9) {
    if constexpr (S::DEPTH == 1) (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, step_kernel<real, S, 9>, S::NT, 0);
  } else {
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, step_kernel<real, S, 5>, S::NT, 0);
  }
  return nb > 0 ? nb : 1;
}

static int resident_per_cu(int precision, int qg, int shape) {
  static int cache[2][2][16] = {};
  int& c = cache[precision == LBM_FP64 ? 1 : 0][qg == 9 ? 1 : 0][shape & 15];
  if (c == 0) {
#define LBM_OCC_F32(kk, ty, w, d) \
  case kk:                        \
    c = step_occupancy<float, Shape<ty, w, d>>(qg); \
    break;
#define LBM_OCC_F64(kk, ty, w, d) \
  case kk:                        \
    c = step_occupancy<double, Shape<ty, w, d>>(qg); \
    break;
    if (precision == LBM_FP64) {
      switch (shape) { LBM_F64_SHAPES(LBM_OCC_F64) default: c = 1; break; }
    } else {
      switch (shape) { LBM_F32_SHAPES(LBM_OCC_F32) default: c = 1; break; }
    }
#undef LBM_OCC_F32
#undef LBM_OCC_F64
  }
  return c;
}

static int persist_step(int precision, int qg, int shape, int grid, hipStream_t st, const void* table, int ninst,
                        const long long* clk, int total_tiles, int nl, int open, GridBar* bar, unsigned spin) {
#define LBM_PERSIST_F32(kk, ty, w, d) \
  case kk:                            \
    return persist_shape<float, Shape<ty, w, d>>(qg, grid, st, table, ninst, clk, total_tiles, nl, open, bar, spin);
#define LBM_PERSIST_F64(kk, ty, w, d) \
  case kk:                            \
    return persist_shape<double, Shape<ty, w, d>>(qg, grid, st, table, ninst, clk, total_tiles, nl, open, bar, spin);
  if (precision == LBM_FP64) {
    switch (shape) { LBM_F64_SHAPES(LBM_PERSIST_F64) default: break; }
  } else {
    switch (shape) { LBM_F32_SHAPES(LBM_PERSIST_F32) default: break; }
  }
#undef LBM_PERSIST_F32
#undef LBM_PERSIST_F64
  return 0;
}

// ------------------------------------------------------------------------------ static batch area
// For callers that cannot allocate device memory, a batch's instance table and clock (the memory
// lbm_batch_create takes from the caller) can live in this static array instead: one area per
// device, holding up to LBM_BATCH_NOALLOC_MAX instances, kept until the process ends.  Host code
// never uses the array's name as an address: its device address is taken once per device with
// hipGetSymbolAddress (with that device current) and kept in g_area_ptr.  One batch uses a
// device's area at a time (g_area_busy); its table and clock are rewritten by every
// lbm_batch_step before any launch reads them, so nothing in it has to start at zero.
constexpr int MAX_DEVICES = 64;
constexpr size_t STATIC_AREA_BYTES =
    (ALIGN + (size_t)LBM_BATCH_NOALLOC_MAX * sizeof(InstDesc<double>) + ALIGN - 1) / ALIGN * ALIGN;
__device__ __align__(256) char scratch[STATIC_AREA_BYTES];

static std::mutex g_area_mu;
static void* g_area_ptr[MAX_DEVICES] = {};
static bool g_area_busy[MAX_DEVICES] = {};

// Device address of device dev's area (dev current); called with g_area_mu held.
static lbm_status static_area(int dev, void** out) {
  if (!g_area_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return LBM_E_DEVICE;
    g_area_ptr[dev] = ptr;
  }
  *out = g_area_ptr[dev];
  return LBM_OK;
}

// Frees the area of batch b for the next one once b's launches have finished.
static lbm_status release_static_area(lbm_batch* b) {
  const hipError_t e = hipStreamSynchronize(b->stream);
  std::lock_guard<std::mutex> lock(g_area_mu);
  g_area_busy[b->noalloc_device] = false;
  return e == hipSuccess ? LBM_OK : LBM_E_DEVICE;
}

// ------------------------------------------------------------------------------ C ABI
extern "C" {

void lbm_params_default(lbm_params* p, int32_t nx, int32_t ny) {
  std::memset(p, 0, sizeof(*p));
  p->nx = nx;
  p->ny = ny;
  p->precision = LBM_FP32;
  p->a = 3.0 / 49.0;
  p->b = 2.0 / 21.0;
  p->R = 1.0;
  p->acentric = 0.344;
  p->G = -1.0;
  p->nu = 0.1;
  p->s_e = p->s_eps = p->s_q = 1.0;
  p->sigma = 1.25;
  p->lambda = 1.0 / 3.0;
  p->cv = 5.0;
  p->wdot = 2.0 / 3.0;
  p->vs3 = p->vs4 = 1.0;
  p->rho_ave = std::numeric_limits<double>::quiet_NaN();
  p->theta_bot_deg = p->theta_top_deg = 90.0;
}

double lbm_critical_temperature(const lbm_params* p) { return 0.0778 * p->a / (0.45724 * p->b * p->R); }

lbm_status lbm_validate(const lbm_params* p) {
  if (!p) return LBM_E_INVAL;
  if (p->nx < 3 || p->ny < 3) return LBM_E_INVAL;
  if (p->precision != LBM_FP32 && p->precision != LBM_FP64) return LBM_E_INVAL;
  // the step kernel addresses a plane with 32-bit byte offsets
  const double plane_bytes = (double)p->nx * (double)p->ny * (p->precision == LBM_FP64 ? 8.0 : 4.0);
  if (plane_bytes > 4294967295.0) return LBM_E_INVAL;
  auto rate_ok = [](double s) { return std::isfinite(s) && s > 0.0 && s < 2.0; };
  if (!(p->nu > 0.0) || !(p->lambda > 0.0) || !(p->cv > 0.0)) return LBM_E_INVAL;
  if (!(p->wdot > 0.0 && p->wdot < 1.0)) return LBM_E_INVAL;
  const double sp = 1.0 / (3.0 * p->nu + 0.5);
  const double vs1 = 1.0 / (p->lambda / (p->thermal_q == 9 ? 1.0 / 3.0 : p->wdot / 2.0) + 0.5);
  if (!rate_ok(p->s_e) || !rate_ok(p->s_eps) || !rate_ok(p->s_q) || !rate_ok(sp) || !rate_ok(vs1) ||
      !rate_ok(p->vs3) || !rate_ok(p->vs4))
    return LBM_E_INVAL;
  if (!(p->a > 0.0) || !(p->b > 0.0) || !(p->R > 0.0) || !(p->G < 0.0)) return LBM_E_INVAL;
  if (!std::isfinite(p->sigma) || !std::isfinite(p->gx) || !std::isfinite(p->gy)) return LBM_E_INVAL;
  if (p->y_walls) {
    if (!finite_pos(p->T_bot) || !finite_pos(p->T_top)) return LBM_E_INVAL;
    if (!(p->theta_bot_deg > 0.0 && p->theta_bot_deg < 180.0 && p->theta_top_deg > 0.0 &&
          p->theta_top_deg < 180.0))
      return LBM_E_INVAL;
  }
  if (p->thermal_box && !finite_pos(p->T_box)) return LBM_E_INVAL;
  if (p->thermal_q != 0 && p->thermal_q != 5 && p->thermal_q != 9) return LBM_E_INVAL;
  if (p->open_top && !p->y_walls) return LBM_E_INVAL;
  if ((p->flags & ~(uint32_t)(LBM_FREEZE_FLOW | LBM_NO_S | LBM_BGK)) != 0) return LBM_E_INVAL;
  return LBM_OK;
}

size_t lbm_footprint_bytes(const lbm_params* p) {
  if (lbm_validate(p) != LBM_OK) return 0;
  const size_t N = (size_t)p->nx * (size_t)p->ny;
  const size_t r = p->precision == LBM_FP64 ? 8 : 4;
  const size_t q = (size_t)qg_of(p);
  return CTRL_BYTES + partial_bytes() + 2 * align_up(9 * N * r) + 2 * align_up(q * N * r) + 2 * align_up(2 * N * r);
}

lbm_status lbm_create(const lbm_params* p, void* dev_mem, size_t bytes, void* hip_stream, lbm_ctx** out) {
  if (!out) return LBM_E_INVAL;
  *out = nullptr;
  if (lbm_validate(p) != LBM_OK) return LBM_E_INVAL;
  if (!dev_mem || ((uintptr_t)dev_mem % ALIGN) != 0) return LBM_E_INVAL;
  if (bytes < lbm_footprint_bytes(p)) return LBM_E_NOMEM;
  lbm_ctx* h = new (std::nothrow) lbm_ctx();
  if (!h) return LBM_E_NOMEM;
  h->prm = *p;
  h->stream = (hipStream_t)hip_stream;
  if (hipGetDevice(&h->device) != hipSuccess) {
    delete h;
    return LBM_E_DEVICE;
  }
  h->base = (char*)dev_mem;
  h->bytes = bytes;
  h->N = (size_t)p->nx * (size_t)p->ny;
  h->rsz = p->precision == LBM_FP64 ? 8 : 4;
  char* q = h->base;
  h->d_desc = q + OFF_DESC;
  h->d_clock = (long long*)(q + OFF_CLOCK);
  h->d_err = (unsigned*)(q + OFF_ERR);
  h->d_diag = (double*)(q + OFF_DIAG);
  h->d_live = (InstLive*)(q + OFF_LIVE);
  h->d_ring = (DiagRecord*)(q + OFF_RING);
  q += CTRL_BYTES;
  h->d_part = (double*)q;
  q += partial_bytes();
  const size_t qg = (size_t)qg_of(p);
  h->fA = q; q += align_up(9 * h->N * h->rsz);
  h->gA = q; q += align_up(qg * h->N * h->rsz);
  h->fB = q; q += align_up(9 * h->N * h->rsz);
  h->gB = q; q += align_up(qg * h->N * h->rsz);
  h->ThA = q; q += align_up(2 * h->N * h->rsz);
  h->ThB = q;
  h->shape_req = -1;
  h->shape = default_shape(p->precision, two_step_ok(p), p->nx, p->ny);
  h->ntiles = tiles_of(p->nx, p->ny, shape_def(p->precision, h->shape).ty);
  *out = h;
  return LBM_OK;
}

lbm_status lbm_destroy(lbm_ctx* h) {
  if (!h) return LBM_E_INVAL;
  if (h->graph) (void)hipGraphExecDestroy(h->graph);
  delete h;
  return LBM_OK;
}

static lbm_status upload_desc(lbm_ctx* h) {
  if (h->prm.precision == LBM_FP64) {
    h->desc64 = make_desc<double>(h, h->shape);
    HIP_OR_FAIL(h, hipMemcpyAsync(h->d_desc, &h->desc64, sizeof(h->desc64), hipMemcpyHostToDevice, h->stream));
  } else {
    h->desc32 = make_desc<float>(h, h->shape);
    HIP_OR_FAIL(h, hipMemcpyAsync(h->d_desc, &h->desc32, sizeof(h->desc32), hipMemcpyHostToDevice, h->stream));
  }
  return LBM_OK;
}

static lbm_status write_clock(lbm_ctx* h) {
  long long c = h->clock;
  HIP_OR_FAIL(h, hipMemcpyAsync(h->d_clock, &c, sizeof(c), hipMemcpyHostToDevice, h->stream));
  HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
  return LBM_OK;
}

lbm_status lbm_init(lbm_ctx* h, const double* rho, const double* ux, const double* uy, const double* T) {
  lbm::HostRange range_("lbm_init");
  if (!h || !rho || !ux || !uy || !T) return LBM_E_INVAL;
  if (h->batch_unsynced) return unsynced(h, "lbm_init");
  if (!set_device(h)) return fail(h, LBM_E_DEVICE, "hipSetDevice failed");
  const size_t N = h->N;
  double sum = 0.0, sumT = 0.0, rmin = std::numeric_limits<double>::infinity();
  for (size_t k = 0; k < N; ++k) {
    if (!finite_pos(rho[k]) || !finite_pos(T[k]) || !std::isfinite(ux[k]) || !std::isfinite(uy[k]))
      return fail(h, LBM_E_INVAL, "initial fields must be finite with rho > 0 and T > 0");
    sum += rho[k];
    sumT += T[k];
    rmin = std::min(rmin, rho[k]);
  }
  // storage offset of the temperature populations, exactly representable in the working precision
  h->T_ref = h->prm.precision == LBM_FP64 ? sumT / (double)N : (double)(float)(sumT / (double)N);
  if (rmin * h->prm.cv < 1.0)
    return fail(h, LBM_E_INVAL, "min(rho) * c_v < 1: the modified collision would weight old populations negatively");
  h->rho_ave = std::isnan(h->prm.rho_ave) ? sum / (double)N : h->prm.rho_ave;
  // stage the FP64 fields in the B copy of f (at least 4 N doubles in either precision)
  double* stage = (double*)h->fB;
  HIP_OR_FAIL(h, hipMemcpyAsync(stage, rho, N * sizeof(double), hipMemcpyHostToDevice, h->stream));
  HIP_OR_FAIL(h, hipMemcpyAsync(stage + N, ux, N * sizeof(double), hipMemcpyHostToDevice, h->stream));
  HIP_OR_FAIL(h, hipMemcpyAsync(stage + 2 * N, uy, N * sizeof(double), hipMemcpyHostToDevice, h->stream));
  HIP_OR_FAIL(h, hipMemcpyAsync(stage + 3 * N, T, N * sizeof(double), hipMemcpyHostToDevice, h->stream));
  const int nb = (int)((N + 255) / 256);
  const int qg = qg_of(&h->prm);
  // weights of the thermal lattice (Eq. 26; the D2Q9 weights for qg = 9)
  const double w0 = qg == 9 ? 4.0 / 9.0 : 1.0 - h->prm.wdot;
  const double w1 = qg == 9 ? 1.0 / 9.0 : h->prm.wdot / 4.0;
  const double w2 = qg == 9 ? 1.0 / 36.0 : 0.0;
  if (h->prm.precision == LBM_FP64) {
    init_kernel<double><<<nb, 256, 0, h->stream>>>(stage, (double*)h->fA, (double*)h->gA, (double*)h->ThA, N, qg,
                                                    w0, w1, w2, h->T_ref);
  } else {
    init_kernel<float><<<nb, 256, 0, h->stream>>>(stage, (float*)h->fA, (float*)h->gA, (float*)h->ThA, N, qg, w0,
                                                   w1, w2, h->T_ref);
  }
  HIP_OR_FAIL(h, hipGetLastError());
  unsigned zero = 0;
  HIP_OR_FAIL(h, hipMemcpyAsync(h->d_err, &zero, sizeof(zero), hipMemcpyHostToDevice, h->stream));
  h->live0 = InstLive{sum, sum / (double)N};
  HIP_OR_FAIL(h, hipMemcpyAsync(h->d_live, &h->live0, sizeof(InstLive), hipMemcpyHostToDevice, h->stream));
  h->steps = 0;
  h->gen = 0;
  h->hgen = 0;
  h->clock = 0;
  lbm_status s = upload_desc(h);
  if (s != LBM_OK) return s;
  s = write_clock(h);
  if (s != LBM_OK) return s;
  if (h->graph) {
    (void)hipGraphExecDestroy(h->graph);
    h->graph = nullptr;
  }
  h->initialised = true;
  h->failed = false;
  return LBM_OK;
}

// The open-top boundary pass after launch k, one workgroup per table entry.
static void launch_open_top(int precision, int ninst, hipStream_t st, const void* table, const long long* clk,
                            int k, const LaunchWin& w) {
  if (precision == LBM_FP64)
    open_top_kernel<double><<<ninst, OPEN_NT, 0, st>>>((const InstDesc<double>*)table, clk, k, w);
  else
    open_top_kernel<float><<<ninst, OPEN_NT, 0, st>>>((const InstDesc<float>*)table, clk, k, w);
}

static void launch_step(int precision, int qg, int shape, int grid, hipStream_t st, const void* table, int ninst,
                        const long long* clk, int k, const LaunchWin& win) {
#define LBM_LAUNCH_F32(kk, ty, w, d) \
  case kk:                           \
    launch_shape<float, Shape<ty, w, d>>(qg, grid, st, table, ninst, clk, k, win); \
    break;
#define LBM_LAUNCH_F64(kk, ty, w, d) \
  case kk:                           \
    launch_shape<double, Shape<ty, w, d>>(qg, grid, st, table, ninst, clk, k, win); \
    break;
  if (precision == LBM_FP64) {
    switch (shape) { LBM_F64_SHAPES(LBM_LAUNCH_F64) default: break; }
  } else {
    switch (shape) { LBM_F32_SHAPES(LBM_LAUNCH_F32) default: break; }
  }
#undef LBM_LAUNCH_F32
#undef LBM_LAUNCH_F64
}

// n launches of the step kernel (each followed by the open-top boundary pass where the
// simulation has one).  With w.use the launches take their step window from w; otherwise they read
// the device clock and the descriptor, and the clock is advanced by the steps they span (the form
// captured in a graph).
static lbm_status launch_steps(lbm_ctx* h, int n, const LaunchWin& w) {
  const int d = shape_def(h->prm.precision, h->shape).depth;
  const bool open = h->prm.y_walls && h->prm.open_top;
  for (int k = 0; k < n; ++k) {
    launch_step(h->prm.precision, qg_of(&h->prm), h->shape, h->ntiles, h->stream, h->d_desc, 1, h->d_clock, k, w);
    if (open) launch_open_top(h->prm.precision, 1, h->stream, h->d_desc, h->d_clock, k, w);
  }
  if (!w.use) clock_advance_kernel<<<1, 64, 0, h->stream>>>(h->d_clock, (long long)n * d);
  HIP_OR_FAIL(h, hipGetLastError());
  return LBM_OK;
}

static lbm_status build_graph(lbm_ctx* h) {
  hipGraph_t g = nullptr;
  HIP_OR_FAIL(h, hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
  lbm_status s = launch_steps(h, GRAPH_STEPS / shape_def(h->prm.precision, h->shape).depth, FROM_CLOCK);
  hipError_t e = hipStreamEndCapture(h->stream, &g);
  if (s != LBM_OK) {
    if (g) (void)hipGraphDestroy(g);
    return s;
  }
  if (e != hipSuccess) return fail(h, LBM_E_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(&h->graph, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    h->graph = nullptr;
    return fail(h, LBM_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  return LBM_OK;
}

// n steps from the current state as one step window: steps [clock, clock + n) from the current
// buffers; a launch of a two-step shape does one step where only one is left.  Whole groups of
// GRAPH_STEPS steps are graph replays, which read the window and the clock from device memory (set
// by one small kernel per window); the remaining launches take the window as an argument.
static lbm_status step_window(lbm_ctx* h, int64_t n) {
  const int d = shape_def(h->prm.precision, h->shape).depth;
  const int64_t launches = (n + d - 1) / d;
  const int64_t per_graph = GRAPH_STEPS / d;
  // the legacy null stream cannot be captured
  const int64_t replays = h->stream != nullptr ? launches / per_graph : 0;
  if (replays > 0) {
    if (!h->graph) {
      lbm_status s = build_graph(h);
      if (s != LBM_OK) return s;
    }
    if (h->prm.precision == LBM_FP64)
      set_window_kernel<double><<<1, 64, 0, h->stream>>>((InstDesc<double>*)h->d_desc, h->d_clock, h->clock, h->gen,
                                                         h->hgen, h->clock + n);
    else
      set_window_kernel<float><<<1, 64, 0, h->stream>>>((InstDesc<float>*)h->d_desc, h->d_clock, h->clock, h->gen,
                                                        h->hgen, h->clock + n);
    HIP_OR_FAIL(h, hipGetLastError());
    for (int64_t r = 0; r < replays; ++r) HIP_OR_FAIL(h, hipGraphLaunch(h->graph, h->stream));
  }
  const int64_t left = launches - replays * per_graph;
  if (left > 0) {
    const LaunchWin w{h->clock + replays * per_graph * d, h->clock, h->clock + n, h->gen, h->hgen, 1};
    lbm_status s = launch_steps(h, (int)left, w);
    if (s != LBM_OK) return s;
  }
  h->clock += (long long)launches * d;
  h->steps += n;
  h->gen ^= (int)(launches & 1);
  h->hgen ^= (int)(history_moves(n, d) & 1);
  return LBM_OK;
}

static lbm_status enqueue_diagnostics(lbm_ctx* h, DiagRecord* rec);

lbm_status lbm_step(lbm_ctx* h, int64_t n) {
  lbm::HostRange range_("lbm_step");
  if (!h || n < 0) return LBM_E_INVAL;
  if (!h->initialised) return fail(h, LBM_E_STATE, "lbm_step before lbm_init");
  if (h->batch_unsynced) return unsynced(h, "lbm_step");
  if (h->failed) return fail(h, LBM_E_STATE, "context has failed: " + h->last_error);
  if (n == 0) return LBM_OK;
  if (!set_device(h)) return fail(h, LBM_E_DEVICE, "hipSetDevice failed");
  if (h->diag_every <= 0) return step_window(h, n);
  // every-k diagnostics: windows that end at the multiples of k, each followed by the reduction
  // into the next slot of the ring
  while (n > 0) {
    const int64_t to_mark = h->diag_every - h->steps % h->diag_every;
    const int64_t m = std::min(n, to_mark);
    lbm_status s = step_window(h, m);
    if (s != LBM_OK) return s;
    n -= m;
    if (h->steps % h->diag_every == 0) {
      s = enqueue_diagnostics(h, h->d_ring + h->diag_enqueued % DIAG_RING);
      if (s != LBM_OK) return s;
      ++h->diag_enqueued;
    }
  }
  return LBM_OK;
}

int64_t lbm_steps_done(const lbm_ctx* h) { return h ? h->steps : -1; }

int lbm_shape_count(int precision) {
  if (precision != LBM_FP32 && precision != LBM_FP64) return 0;
  return shape_count(precision);
}

lbm_status lbm_shape_info(int precision, int k, int* tile_x, int* tile_y, int* waves, int* steps_per_launch) {
  if ((precision != LBM_FP32 && precision != LBM_FP64) || k < 0 || k >= shape_count(precision)) return LBM_E_INVAL;
  const ShapeDef& d = shape_def(precision, k);
  if (tile_x) *tile_x = TX;
  if (tile_y) *tile_y = d.ty;
  if (waves) *waves = d.waves;
  if (steps_per_launch) *steps_per_launch = d.depth;
  return LBM_OK;
}

int lbm_shape_fits(const lbm_params* p, int k) {
  if (!p || lbm_validate(p) != LBM_OK || k < 0 || k >= shape_count(p->precision)) return 0;
  return shape_fits(p->precision, two_step_ok(p), k, p->nx, p->ny) ? 1 : 0;
}

lbm_status lbm_set_shape(lbm_ctx* h, int k) {
  if (!h || k < -1 || k >= shape_count(h->prm.precision)) return LBM_E_INVAL;
  if (k >= 0 && !shape_fits(h->prm.precision, two_step_ok(&h->prm), k, h->prm.nx, h->prm.ny))
    return fail(h, LBM_E_INVAL, "two-step tile shape on a grid smaller than its halo region");
  h->shape_req = k;
  const int s = k < 0 ? default_shape(h->prm.precision, two_step_ok(&h->prm), h->prm.nx, h->prm.ny) : k;
  if (s == h->shape) return LBM_OK;
  h->shape = s;
  h->ntiles = tiles_of(h->prm.nx, h->prm.ny, shape_def(h->prm.precision, s).ty);
  if (h->graph) {
    (void)hipGraphExecDestroy(h->graph);
    h->graph = nullptr;
  }
  if (h->initialised) {
    if (!set_device(h)) return fail(h, LBM_E_DEVICE, "hipSetDevice failed");
    lbm_status st = upload_desc(h);  // ordered on the stream after the launches already enqueued
    if (st != LBM_OK) return st;
    HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
  }
  return LBM_OK;
}

int lbm_get_shape(const lbm_ctx* h) { return h ? h->shape : -1; }

lbm_status lbm_set_tile_order(lbm_ctx* h, int order) {
  if (!h || order < 0) return LBM_E_INVAL;
  h->order_req = order;
  if (h->initialised) {
    if (!set_device(h)) return fail(h, LBM_E_DEVICE, "hipSetDevice failed");
    lbm_status st = upload_desc(h);  // ordered on the stream after the launches already enqueued
    if (st != LBM_OK) return st;
    HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
  }
  return LBM_OK;
}

int lbm_get_tile_order(const lbm_ctx* h) {
  if (!h) return -1;
  const int ntx = (h->prm.nx + TX - 1) / TX;
  return tile_strip(h, ntx, h->shape);
}

lbm_status lbm_sync(lbm_ctx* h) {
  if (!h) return LBM_E_INVAL;
  if (!h->initialised) return fail(h, LBM_E_STATE, "lbm_sync before lbm_init");
  if (!set_device(h)) return fail(h, LBM_E_DEVICE, "hipSetDevice failed");
  return check_device_error(h);
}

// current source buffers (B after an odd number of launches)
static void current_buffers(lbm_ctx* h, void*& f, void*& g, void*& fo) {
  const bool odd = (h->gen & 1) != 0;
  f = odd ? h->fB : h->fA;
  g = odd ? h->gB : h->gA;
  fo = odd ? h->fA : h->fB;
}

// current temperature history (follows the buffers of f and g)
static void* current_history(lbm_ctx* h) { return (h->hgen & 1) ? h->ThB : h->ThA; }

lbm_status lbm_read_fields(lbm_ctx* h, double* rho, double* ux, double* uy, double* T) {
  lbm::HostRange range_("lbm_read_fields");
  if (!h) return LBM_E_INVAL;
  if (!h->initialised) return fail(h, LBM_E_STATE, "lbm_read_fields before lbm_init");
  if (h->batch_unsynced) return unsynced(h, "lbm_read_fields");
  if (!set_device(h)) return fail(h, LBM_E_DEVICE, "hipSetDevice failed");
  lbm_status s = check_device_error(h);
  if (s != LBM_OK) return s;
  void *f, *g, *fo;
  current_buffers(h, f, g, fo);
  double* stage = (double*)fo;
  const size_t N = h->N;
  const int nb = (int)((N + 255) / 256);
  if (h->prm.precision == LBM_FP64)
    fields_kernel<double><<<nb, 256, 0, h->stream>>>(h->desc64.p, h->d_live, (const double*)f, (const double*)g,
                                                      h->prm.nx, h->prm.ny, stage, h->d_err);
  else
    fields_kernel<float><<<nb, 256, 0, h->stream>>>(h->desc32.p, h->d_live, (const float*)f, (const float*)g,
                                                     h->prm.nx, h->prm.ny, stage, h->d_err);
  HIP_OR_FAIL(h, hipGetLastError());
  double* outs[4] = {rho, ux, uy, T};
  for (int c = 0; c < 4; ++c)
    if (outs[c])
      HIP_OR_FAIL(h, hipMemcpyAsync(outs[c], stage + c * N, N * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
  return check_device_error(h);
}

// The FP64 mass and energy reduction of the current state on the context's stream: result in
// d_diag and, if rec is not null, as a record of the current step count at *rec.
static lbm_status enqueue_diagnostics_of(lbm_ctx* h, hipStream_t stream, const void* f, const void* g,
                                         DiagRecord* rec, long long step) {
  const size_t N = h->N;
  size_t per = (N + MAX_RED_BLOCKS - 1) / MAX_RED_BLOCKS;
  per = std::max<size_t>(per, RED_NT);
  const int nparts = (int)((N + per - 1) / per);
  if (h->prm.precision == LBM_FP64)
    diag_partial_kernel<double><<<nparts, RED_NT, 0, stream>>>(
        (const double*)f, (const double*)g, N, qg_of(&h->prm), h->prm.cv, h->T_ref, per, h->d_part);
  else
    diag_partial_kernel<float><<<nparts, RED_NT, 0, stream>>>(
        (const float*)f, (const float*)g, N, qg_of(&h->prm), h->prm.cv, h->T_ref, per, h->d_part);
  diag_final_kernel<<<1, RED_NT, 0, stream>>>(h->d_part, nparts, h->d_diag, rec, step);
  HIP_OR_FAIL(h, hipGetLastError());
  return LBM_OK;
}

static lbm_status enqueue_diagnostics(lbm_ctx* h, DiagRecord* rec) {
  void *f, *g, *fo;
  current_buffers(h, f, g, fo);
  return enqueue_diagnostics_of(h, h->stream, f, g, rec, (long long)h->steps);
}

lbm_status lbm_diagnostics(lbm_ctx* h, double* mass, double* energy) {
  lbm::HostRange range_("lbm_diagnostics");
  if (!h) return LBM_E_INVAL;
  if (!h->initialised) return fail(h, LBM_E_STATE, "lbm_diagnostics before lbm_init");
  if (h->batch_unsynced) return unsynced(h, "lbm_diagnostics");
  if (!set_device(h)) return fail(h, LBM_E_DEVICE, "hipSetDevice failed");
  lbm_status st = enqueue_diagnostics(h, nullptr);
  if (st != LBM_OK) return st;
  double out[2];
  HIP_OR_FAIL(h, hipMemcpyAsync(out, h->d_diag, sizeof(out), hipMemcpyDeviceToHost, h->stream));
  HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
  if (mass) *mass = out[0];
  if (energy) *energy = out[1];
  return check_device_error(h);
}

lbm_status lbm_set_diagnostics_interval(lbm_ctx* h, int64_t k) {
  if (!h || k < 0) return LBM_E_INVAL;
  h->diag_every = k;
  h->diag_enqueued = 0;
  h->diag_read = 0;
  return LBM_OK;
}

lbm_status lbm_read_diagnostics_log(lbm_ctx* h, int64_t* steps, double* mass, double* energy, int max, int* count) {
  if (!h || !count || max < 0 || (max > 0 && (!steps || !mass || !energy))) return LBM_E_INVAL;
  *count = 0;
  if (!h->initialised) return fail(h, LBM_E_STATE, "lbm_read_diagnostics_log before lbm_init");
  if (h->batch_unsynced) return unsynced(h, "lbm_read_diagnostics_log");
  if (!set_device(h)) return fail(h, LBM_E_DEVICE, "hipSetDevice failed");
  DiagRecord ring[DIAG_RING];
  HIP_OR_FAIL(h, hipMemcpyAsync(ring, h->d_ring, sizeof(ring), hipMemcpyDeviceToHost, h->stream));
  HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
  // records still in the ring: the last DIAG_RING enqueued; older unread ones were overwritten
  int64_t first = std::max(h->diag_read, h->diag_enqueued - DIAG_RING);
  int c = 0;
  for (int64_t r = first; r < h->diag_enqueued && c < max; ++r, ++c) {
    const DiagRecord& d = ring[r % DIAG_RING];
    steps[c] = d.step;
    mass[c] = d.mass;
    energy[c] = d.energy;
  }
  h->diag_read = first + c;
  *count = c;
  return check_device_error(h);
}

lbm_status lbm_vapour_rows(lbm_ctx* h, double rho_threshold, int x_lo, int x_hi, int32_t* counts) {
  lbm::HostRange range_("lbm_vapour_rows");
  if (!h || !counts || !std::isfinite(rho_threshold) || x_hi <= x_lo || x_hi - x_lo > h->prm.nx) return LBM_E_INVAL;
  if (!h->initialised) return fail(h, LBM_E_STATE, "lbm_vapour_rows before lbm_init");
  if (h->batch_unsynced) return unsynced(h, "lbm_vapour_rows");
  if (!set_device(h)) return fail(h, LBM_E_DEVICE, "hipSetDevice failed");
  void *f, *g, *fo;
  current_buffers(h, f, g, fo);
  const int ny = h->prm.ny;
  const int chunk = (int)(partial_bytes() / sizeof(int));  // rows per pass through the partials area
  int* dcount = (int*)h->d_part;
  for (int y0 = 0; y0 < ny; y0 += chunk) {
    const int rows = std::min(chunk, ny - y0);
    if (h->prm.precision == LBM_FP64)
      vapour_rows_kernel<double><<<rows, VAP_NT, 0, h->stream>>>((const double*)f, h->prm.nx, h->N, y0, x_lo,
                                                                 x_hi - x_lo, rho_threshold, dcount);
    else
      vapour_rows_kernel<float><<<rows, VAP_NT, 0, h->stream>>>((const float*)f, h->prm.nx, h->N, y0, x_lo,
                                                                x_hi - x_lo, (float)rho_threshold, dcount);
    HIP_OR_FAIL(h, hipGetLastError());
    HIP_OR_FAIL(h, hipMemcpyAsync(counts + y0, dcount, rows * sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
  }
  return check_device_error(h);
}

lbm_status lbm_vapour_components(lbm_ctx* h, double rho_threshold, int y_lo, int y_hi, lbm_component* out,
                                 int max_out, int* n_total) {
  lbm::HostRange range_("lbm_vapour_components");
  if (!h || !n_total || max_out < 0 || (max_out > 0 && !out) || !std::isfinite(rho_threshold)) return LBM_E_INVAL;
  if (y_lo < 0 || y_hi > h->prm.ny || y_hi <= y_lo) return LBM_E_INVAL;
  *n_total = 0;
  if (!h->initialised) return fail(h, LBM_E_STATE, "lbm_vapour_components before lbm_init");
  if (h->batch_unsynced) return unsynced(h, "lbm_vapour_components");
  if (!set_device(h)) return fail(h, LBM_E_DEVICE, "hipSetDevice failed");
  void *f, *g, *fo;
  current_buffers(h, f, g, fo);
  // Scratch: the labels (4 bytes per node of the rows) in the other f copy, which the next step
  // overwrites before reading it; the table after them if it has room for as many entries as the
  // partials area, else in the partials area; the counter at the start of the partials area.
  const int nx = h->prm.nx, n = nx * (y_hi - y_lo);
  int* lab = (int*)fo;
  int* dcount = (int*)h->d_part;
  const size_t lab_bytes = ((size_t)n * sizeof(int) + 255) & ~(size_t)255;
  const size_t room = 9 * h->N * h->rsz - lab_bytes;  // >= 32 N - 255 bytes, since n <= N
  const size_t part_cap = (partial_bytes() - 256) / sizeof(CompStat);
  CompStat* tab = (CompStat*)((char*)h->d_part + 256);
  size_t cap = part_cap;
  if (room / sizeof(CompStat) > part_cap) {
    tab = (CompStat*)((char*)fo + lab_bytes);
    cap = std::min<size_t>(LBM_MAX_COMPONENTS, room / sizeof(CompStat));
  }
  const int nb = (n + CC_NT - 1) / CC_NT;
  if (h->prm.precision == LBM_FP64)
    cc_init_kernel<double><<<nb, CC_NT, 0, h->stream>>>((const double*)f, nx, h->N, y_lo, n, rho_threshold, lab);
  else
    cc_init_kernel<float><<<nb, CC_NT, 0, h->stream>>>((const float*)f, nx, h->N, y_lo, n, rho_threshold, lab);
  cc_union_kernel<<<nb, CC_NT, 0, h->stream>>>(lab, nx, y_hi - y_lo);
  cc_flatten_kernel<<<nb, CC_NT, 0, h->stream>>>(lab, n);
  HIP_OR_FAIL(h, hipMemsetAsync(dcount, 0, sizeof(int), h->stream));
  cc_number_kernel<<<nb, CC_NT, 0, h->stream>>>(lab, n, y_lo * nx, dcount, tab, (int)cap);
  cc_stats_kernel<<<nb, CC_NT, 0, h->stream>>>(lab, nx, n, y_lo, tab, (int)cap);
  HIP_OR_FAIL(h, hipGetLastError());
  int total = 0;
  HIP_OR_FAIL(h, hipMemcpyAsync(&total, dcount, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
  *n_total = total;
  if ((size_t)total > cap)
    return fail(h, LBM_E_INVAL, "more vapour components than the table holds (" + std::to_string(cap) +
                                    "); narrow the rows or change the threshold");
  std::vector<CompStat> all((size_t)total);
  if (total > 0) {
    HIP_OR_FAIL(h, hipMemcpyAsync(all.data(), tab, (size_t)total * sizeof(CompStat), hipMemcpyDeviceToHost, h->stream));
    HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
  }
  std::sort(all.begin(), all.end(), [](const CompStat& a, const CompStat& b) { return a.root < b.root; });
  for (int i = 0; i < std::min(total, max_out); ++i) {
    const CompStat& c = all[(size_t)i];
    out[i] = lbm_component{c.root, c.area, c.y_min, c.y_max, c.x_min, c.x_max, (int64_t)c.y_sum};
  }
  return check_device_error(h);
}

// planes of the raw state: f (9), g (5 or 9), history (2)
static size_t state_planes(const lbm_ctx* h) { return 9 + (size_t)qg_of(&h->prm) + 2; }

// Trailer of a saved state (after the planes): what the state belongs to, checked on load, and the
// scalars that go with the populations.
struct StateTrailer {
  char magic[8];      // "LBM2D\0\0\0"
  int32_t version;    // STATE_VERSION
  int32_t precision;  // LBM_FP32 / LBM_FP64
  int32_t nx, ny;
  int32_t qg;         // thermal lattice: 5 or 9
  int32_t reserved;
  int64_t steps;
  double rho_ave;     // rho_ave of the buoyancy at init (or as given)
  double T_ref;       // storage offset of g and the history
  double mass;        // FP64 mass the device tracks (it changes through an open top)
};
static_assert(sizeof(StateTrailer) == 64, "state trailer layout");
constexpr int32_t STATE_VERSION = 2;
static const char STATE_MAGIC[8] = {'L', 'B', 'M', '2', 'D', 0, 0, 0};

static size_t planes_bytes(const lbm_ctx* h) { return state_planes(h) * h->N * h->rsz; }

size_t lbm_state_bytes(const lbm_ctx* h) { return h ? planes_bytes(h) + sizeof(StateTrailer) : 0; }

lbm_status lbm_save_state(lbm_ctx* h, void* host, size_t bytes) {
  lbm::HostRange range_("lbm_save_state");
  if (!h || !host) return LBM_E_INVAL;
  if (!h->initialised) return fail(h, LBM_E_STATE, "lbm_save_state before lbm_init");
  if (h->batch_unsynced) return unsynced(h, "lbm_save_state");
  if (bytes < lbm_state_bytes(h)) return fail(h, LBM_E_INVAL, "host buffer smaller than lbm_state_bytes");
  if (!set_device(h)) return fail(h, LBM_E_DEVICE, "hipSetDevice failed");
  void *f, *g, *fo;
  current_buffers(h, f, g, fo);
  char* q = (char*)host;
  const size_t N = h->N, r = h->rsz;
  const size_t Q = (size_t)qg_of(&h->prm);
  InstLive live{};
  HIP_OR_FAIL(h, hipMemcpyAsync(q, f, 9 * N * r, hipMemcpyDeviceToHost, h->stream));
  HIP_OR_FAIL(h, hipMemcpyAsync(q + 9 * N * r, g, Q * N * r, hipMemcpyDeviceToHost, h->stream));
  HIP_OR_FAIL(h, hipMemcpyAsync(q + (9 + Q) * N * r, current_history(h), 2 * N * r, hipMemcpyDeviceToHost,
                                h->stream));
  HIP_OR_FAIL(h, hipMemcpyAsync(&live, h->d_live, sizeof(live), hipMemcpyDeviceToHost, h->stream));
  HIP_OR_FAIL(h, hipStreamSynchronize(h->stream));
  StateTrailer t{};
  std::memcpy(t.magic, STATE_MAGIC, sizeof(t.magic));
  t.version = STATE_VERSION;
  t.precision = h->prm.precision;
  t.nx = h->prm.nx;
  t.ny = h->prm.ny;
  t.qg = qg_of(&h->prm);
  t.steps = h->steps;
  t.rho_ave = h->rho_ave;
  t.T_ref = h->T_ref;
  t.mass = live.mass;
  std::memcpy(q + planes_bytes(h), &t, sizeof(t));
  return check_device_error(h);
}

lbm_status lbm_load_state(lbm_ctx* h, const void* host, size_t bytes) {
  lbm::HostRange range_("lbm_load_state");
  if (!h || !host) return LBM_E_INVAL;
  if (h->batch_unsynced) return unsynced(h, "lbm_load_state");
  if (bytes != lbm_state_bytes(h)) return fail(h, LBM_E_INVAL, "buffer size differs from lbm_state_bytes");
  const char* q = (const char*)host;
  StateTrailer t;
  std::memcpy(&t, q + planes_bytes(h), sizeof(t));
  if (std::memcmp(t.magic, STATE_MAGIC, sizeof(t.magic)) != 0 || t.version != STATE_VERSION)
    return fail(h, LBM_E_INVAL, "not a saved state of this library version");
  if (t.precision != h->prm.precision || t.nx != h->prm.nx || t.ny != h->prm.ny || t.qg != qg_of(&h->prm))
    return fail(h, LBM_E_INVAL, "saved state of another precision, grid or thermal lattice");
  if (t.steps < 0 || !std::isfinite(t.rho_ave) || !std::isfinite(t.T_ref) || !std::isfinite(t.mass))
    return fail(h, LBM_E_INVAL, "corrupt state trailer");
  if (!set_device(h)) return fail(h, LBM_E_DEVICE, "hipSetDevice failed");
  const size_t N = h->N, r = h->rsz;
  h->steps = t.steps;
  h->gen = 0;  // the state goes to the A buffers
  h->hgen = 0;
  h->rho_ave = t.rho_ave;
  h->T_ref = t.T_ref;
  h->live0 = InstLive{t.mass, t.mass / (double)N};
  void *f, *g, *fo;
  current_buffers(h, f, g, fo);
  const size_t Q = (size_t)qg_of(&h->prm);
  HIP_OR_FAIL(h, hipMemcpyAsync(f, q, 9 * N * r, hipMemcpyHostToDevice, h->stream));
  HIP_OR_FAIL(h, hipMemcpyAsync(g, q + 9 * N * r, Q * N * r, hipMemcpyHostToDevice, h->stream));
  HIP_OR_FAIL(h, hipMemcpyAsync(current_history(h), q + (9 + Q) * N * r, 2 * N * r, hipMemcpyHostToDevice,
                                h->stream));
  HIP_OR_FAIL(h, hipMemcpyAsync(h->d_live, &h->live0, sizeof(InstLive), hipMemcpyHostToDevice, h->stream));
  unsigned zero = 0;
  HIP_OR_FAIL(h, hipMemcpyAsync(h->d_err, &zero, sizeof(zero), hipMemcpyHostToDevice, h->stream));
  lbm_status s = upload_desc(h);
  if (s != LBM_OK) return s;
  s = write_clock(h);
  if (s != LBM_OK) return s;
  h->initialised = true;
  h->failed = false;
  return LBM_OK;
}

lbm_status lbm_read_state(lbm_ctx* h, double* f, double* g, double* hist) {
  lbm::HostRange range_("lbm_read_state");
  if (!h) return LBM_E_INVAL;
  if (!h->initialised) return fail(h, LBM_E_STATE, "lbm_read_state before lbm_init");
  if (h->batch_unsynced) return unsynced(h, "lbm_read_state");
  std::vector<char> raw;
  try {
    raw.resize(lbm_state_bytes(h));
  } catch (const std::bad_alloc&) {
    return fail(h, LBM_E_NOMEM, "host buffer for the state");
  }
  lbm_status s = lbm_save_state(h, raw.data(), raw.size());
  if (s != LBM_OK) return s;
  const size_t N = h->N;
  const int qg = qg_of(&h->prm);
  // weights of the thermal lattice (Eq. 26; the D2Q9 weights for qg = 9): g is stored as
  // g_i - what_i T_ref, the history as T - T_ref
  const double w0 = qg == 9 ? 4.0 / 9.0 : 1.0 - h->prm.wdot;
  const double w1 = qg == 9 ? 1.0 / 9.0 : h->prm.wdot / 4.0;
  const double w2 = qg == 9 ? 1.0 / 36.0 : 0.0;
  auto value = [&](size_t plane, size_t k) -> double {
    if (h->prm.precision == LBM_FP64) return ((const double*)raw.data())[plane * N + k];
    return (double)((const float*)raw.data())[plane * N + k];
  };
  for (size_t k = 0; k < N; ++k) {
    if (f)
      for (size_t i = 0; i < 9; ++i) f[i * N + k] = value(i, k);
    if (g)
      for (int i = 0; i < qg; ++i) g[i * N + k] = value(9 + i, k) + (i == 0 ? w0 : i < 5 ? w1 : w2) * h->T_ref;
    if (hist)
      for (size_t j = 0; j < 2; ++j) hist[j * N + k] = value(9 + qg + j, k) + h->T_ref;
  }
  return LBM_OK;
}

// Maxwell equal-area construction (host, FP64): p(rho_g) = p(rho_l) = p_sat and
// integral_{rho_g}^{rho_l} (p - p_sat)/rho^2 drho = 0.  The spinodal points are found by
// golden-section search of p on either side, the integral is done analytically per piece
// with adaptive Gauss-Legendre quadrature, p_sat by bisection.
static double pr_p(const lbm_params* p, double rho, double T) {
  const double Tc = lbm_critical_temperature(p);
  const double s = 1.0 + pr_kappa(p) * (1.0 - std::sqrt(T / Tc));
  const double b = p->b;
  return rho * p->R * T / (1.0 - b * rho) - p->a * s * s * rho * rho / (1.0 + 2.0 * b * rho - b * b * rho * rho);
}

static double gl_integral(const lbm_params* p, double T, double ps, double lo, double hi) {
  // 16-point Gauss-Legendre on 64 panels of (p - ps)/rho^2
  static const double xg[8] = {0.0950125098376374, 0.2816035507792589, 0.4580167776572274, 0.6178762444026438,
                               0.7554044083550030, 0.8656312023878318, 0.9445750230732326, 0.9894009349916499};
  static const double wg[8] = {0.1894506104550685, 0.1826034150449236, 0.1691565193950025, 0.1495959888165767,
                               0.1246289712555339, 0.0951585116824928, 0.0622535239386479, 0.0271524594117541};
  const int panels = 64;
  const double h = (hi - lo) / panels;
  double s = 0.0;
  for (int k = 0; k < panels; ++k) {
    const double c = lo + (k + 0.5) * h, r = 0.5 * h;
    for (int j = 0; j < 8; ++j) {
      for (int sgn = -1; sgn <= 1; sgn += 2) {
        const double x = c + sgn * r * xg[j];
        s += wg[j] * r * (pr_p(p, x, T) - ps) / (x * x);
      }
    }
  }
  return s;
}

static double golden_extremum(const lbm_params* p, double T, double lo, double hi, bool maximum) {
  const double gr = 0.5 * (std::sqrt(5.0) - 1.0);
  double a = lo, b = hi;
  double c = b - gr * (b - a), d = a + gr * (b - a);
  for (int it = 0; it < 200; ++it) {
    const double fc = pr_p(p, c, T), fd = pr_p(p, d, T);
    const bool left = maximum ? (fc > fd) : (fc < fd);
    if (left) b = d;
    else a = c;
    c = b - gr * (b - a);
    d = a + gr * (b - a);
  }
  return 0.5 * (a + b);
}

static double bisect_root(const lbm_params* p, double T, double target, double lo, double hi) {
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (pr_p(p, mid, T) < target) lo = mid;
    else hi = mid;
  }
  return 0.5 * (lo + hi);
}

lbm_status lbm_eos_coexistence(const lbm_params* p, double T, double* rho_l, double* rho_g, double* p_sat) {
  if (!p || !rho_l || !rho_g || !p_sat || !(T > 0.0)) return LBM_E_INVAL;
  const double rmax = (1.0 / p->b) * (1.0 - 1e-9);
  // coarse scan to bracket the local maximum and minimum of the subcritical isotherm
  const int NS = 4000;
  const double h = rmax / NS;
  int kmax = -1, kmin = -1;
  double prev = pr_p(p, h, T);
  bool rising = true;
  for (int k = 2; k < NS; ++k) {
    const double cur = pr_p(p, k * h, T);
    if (rising && cur < prev) {
      kmax = k - 1;
      rising = false;
    } else if (!rising && cur > prev) {
      kmin = k - 1;
      break;
    }
    prev = cur;
  }
  if (kmax < 0 || kmin < 0) return LBM_E_INVAL;
  const double rs_max = golden_extremum(p, T, (kmax - 1) * h, (kmax + 1) * h, true);
  const double rs_min = golden_extremum(p, T, (kmin - 1) * h, (kmin + 1) * h, false);
  double lo = std::max(pr_p(p, rs_min, T), 1e-14), hi = pr_p(p, rs_max, T);
  for (int it = 0; it < 200; ++it) {
    const double ps = 0.5 * (lo + hi);
    const double rg = bisect_root(p, T, ps, 1e-12, rs_max);
    const double rl = bisect_root(p, T, ps, rs_min, rmax);
    if (gl_integral(p, T, ps, rg, rl) > 0) lo = ps;
    else hi = ps;
  }
  *p_sat = 0.5 * (lo + hi);
  *rho_g = bisect_root(p, T, *p_sat, 1e-12, rs_max);
  *rho_l = bisect_root(p, T, *p_sat, rs_min, rmax);
  return LBM_OK;
}

const char* lbm_strerror(lbm_status s) {
  switch (s) {
    case LBM_OK: return "ok";
    case LBM_E_INVAL: return "invalid argument";
    case LBM_E_NOMEM: return "device buffer too small";
    case LBM_E_DEVICE: return "HIP runtime error";
    case LBM_E_NUMERIC: return "numerical failure on the device";
    case LBM_E_STATE: return "call out of order or context failed";
  }
  return "unknown status";
}

const char* lbm_last_error(const lbm_ctx* h) { return h ? h->last_error.c_str() : "null context"; }

// ------------------------------------------------------------------------------ batches
size_t lbm_batch_footprint_bytes(int n) {
  if (n <= 0) return 0;
  return align_up(ALIGN + (size_t)n * sizeof(InstDesc<double>));
}

lbm_status lbm_batch_create(lbm_ctx* const* ctxs, int n, void* dev_mem, size_t bytes, void* hip_stream,
                            lbm_batch** out) {
  if (!out || !ctxs || n <= 0) return LBM_E_INVAL;
  *out = nullptr;
  if (!dev_mem || ((uintptr_t)dev_mem % ALIGN) != 0) return LBM_E_INVAL;
  if (bytes < lbm_batch_footprint_bytes(n)) return LBM_E_NOMEM;
  const int prec = ctxs[0] ? ctxs[0]->prm.precision : -1;
  const int qg = ctxs[0] ? qg_of(&ctxs[0]->prm) : 0;
  for (int i = 0; i < n; ++i)
    if (!ctxs[i] || !ctxs[i]->initialised || ctxs[i]->prm.precision != prec || qg_of(&ctxs[i]->prm) != qg)
      return LBM_E_INVAL;
  for (int i = 0; i < n; ++i)
    if (ctxs[i]->batch_unsynced) return unsynced(ctxs[i], "lbm_batch_create");
  lbm_batch* b = new (std::nothrow) lbm_batch();
  if (!b) return LBM_E_NOMEM;
  b->ctx.assign(ctxs, ctxs + n);
  b->remaining.assign(n, 0);
  b->pending.assign(n, 0);
  b->pending_launches.assign(n, 0);
  b->pending_hmoves.assign(n, 0);
  b->moved.assign(n, 0);
  b->stream = (hipStream_t)hip_stream;
  b->precision = prec;
  b->qg = qg;
  // the batch's work follows whatever is already enqueued on the members' own streams
  if (wait_for_members(b->stream, b->ctx) != hipSuccess) {
    delete b;
    return LBM_E_DEVICE;
  }
  b->shape = batch_default_shape(prec, b->ctx);
  b->base = (char*)dev_mem;
  b->bytes = bytes;
  b->d_clock = (long long*)b->base;
  b->d_bar = (GridBar*)(b->base + 64);
  b->d_table = b->base + ALIGN;
  *out = b;
  return LBM_OK;
}

lbm_status lbm_batch_set_budget(lbm_batch* b, int i, int64_t steps) {
  if (!b || i < 0 || i >= (int)b->ctx.size() || steps < 0) return LBM_E_INVAL;
  if (b->ctx[i]->failed) return LBM_E_STATE;
  b->remaining[i] = steps;
  return LBM_OK;
}

int64_t lbm_batch_remaining(const lbm_batch* b, int i) {
  if (!b || i < 0 || i >= (int)b->ctx.size()) return -1;
  return b->remaining[i];
}

lbm_status lbm_batch_set_shape(lbm_batch* b, int k) {
  if (!b || k < -1 || k >= shape_count(b->precision)) return LBM_E_INVAL;
  if (k >= 0)
    for (lbm_ctx* h : b->ctx)
      if (!shape_fits(b->precision, two_step_ok(&h->prm), k, h->prm.nx, h->prm.ny)) return LBM_E_INVAL;
  if (k < 0) k = batch_default_shape(b->precision, b->ctx);
  b->shape = k;  // tile counts change; the graph is recaptured at the next upload
  return LBM_OK;
}

int lbm_batch_get_shape(const lbm_batch* b) { return b ? b->shape : -1; }

lbm_status lbm_batch_set_persistent(lbm_batch* b, int on, uint32_t spin_limit) {
  if (!b || (on != 0 && on != 1)) return LBM_E_INVAL;
  b->persistent = on != 0;
  b->spin_limit = spin_limit ? spin_limit : (1u << 24);
  if (b->graph) {  // the captured launches change form
    (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
  }
  return LBM_OK;
}

}  // extern "C"

// Table of the batch: active instances first (in the caller's order), then parked ones, so
// that tile_begin is non-decreasing along the table as the kernel's binary search needs.  Each
// active instance runs min(todo, its budget) steps from the current clock.
template <typename real>
static void fill_table(lbm_batch* b, std::vector<InstDesc<real>>& tab, int64_t todo) {
  const int n = (int)b->ctx.size();
  std::vector<int> order;
  for (int i = 0; i < n; ++i)
    if (b->remaining[i] > 0) order.push_back(i);
  for (int i = 0; i < n; ++i)
    if (b->remaining[i] <= 0) order.push_back(i);
  int tiles = 0;
  tab.resize(n);
  for (int j = 0; j < n; ++j) {
    const int i = order[j];
    lbm_ctx* h = b->ctx[i];
    InstDesc<real> D = make_desc<real>(h, b->shape);
    // buffers as left by the context's own steps and the batched launches not yet synced
    D.t_base = b->clock;
    D.b_base = (h->gen ^ (int)(b->pending_launches[i] & 1)) & 1;
    D.h_base = (h->hgen ^ (int)(b->pending_hmoves[i] & 1)) & 1;
    if (b->remaining[i] > 0) {
      D.tile_begin = tiles;
      D.t_end = b->clock + std::min<int64_t>(todo, b->remaining[i]);
      tiles += D.ntx * D.nty;
    } else {
      D.tile_begin = -1;  // fixed up below: parked instances own no workgroups
      D.t_end = D.t_base;
    }
    tab[j] = D;
  }
  for (int j = 0; j < n; ++j)
    if (tab[j].tile_begin < 0) tab[j].tile_begin = tiles;
  b->total_tiles = tiles;
}

extern "C" {

static lbm_status batch_upload(lbm_batch* b, int64_t todo) {
  lbm_ctx* h0 = b->ctx[0];
  const size_t n = b->ctx.size();
  long long c = b->clock;
  if (b->precision == LBM_FP64) {
    std::vector<InstDesc<double>> tab;
    fill_table(b, tab, todo);
    HIP_OR_FAIL(h0, hipMemcpyAsync(b->d_table, tab.data(), n * sizeof(tab[0]), hipMemcpyHostToDevice, b->stream));
    HIP_OR_FAIL(h0, hipMemcpyAsync(b->d_clock, &c, sizeof(c), hipMemcpyHostToDevice, b->stream));
    HIP_OR_FAIL(h0, hipStreamSynchronize(b->stream));
  } else {
    std::vector<InstDesc<float>> tab;
    fill_table(b, tab, todo);
    HIP_OR_FAIL(h0, hipMemcpyAsync(b->d_table, tab.data(), n * sizeof(tab[0]), hipMemcpyHostToDevice, b->stream));
    HIP_OR_FAIL(h0, hipMemcpyAsync(b->d_clock, &c, sizeof(c), hipMemcpyHostToDevice, b->stream));
    HIP_OR_FAIL(h0, hipStreamSynchronize(b->stream));
  }
  // the captured launches depend only on the table address, the instance count, the grid size
  // (total tiles of the active instances in table order) and the shape; keep the graph while
  // these are unchanged
  std::vector<lbm_ctx*> layout;
  for (size_t i = 0; i < n; ++i)
    if (b->remaining[i] > 0) layout.push_back(b->ctx[i]);
  if (b->graph && (layout != b->graph_layout || b->shape != b->graph_shape)) {
    (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
  }
  b->graph_layout = layout;
  b->graph_shape = b->shape;
  return LBM_OK;
}

// Workgroups of the batch's persistent kernel: as many as are resident at once on the device
// (a multiple of the 8 XCDs), and no more than the tiles need.
static lbm_status persistent_grid(lbm_batch* b, int* grid) {
  if (b->pgrid_shape != b->shape) {
    int cus = 0;
    HIP_OR_FAIL(b->ctx[0], hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->ctx[0]->device));
    const int per_cu = persist_step(b->precision, b->qg, b->shape, 0, nullptr, nullptr, 0, nullptr, 0, 0, 0, nullptr, 0);
    b->pgrid = per_cu * cus / NXCD * NXCD;
    b->pgrid_shape = b->shape;
    if (b->pgrid < NXCD) return fail(b->ctx[0], LBM_E_DEVICE, "persistent kernel: no resident workgroups");
  }
  *grid = std::min(b->pgrid, (b->total_tiles + NXCD - 1) / NXCD * NXCD);
  return LBM_OK;
}

// nl launches of the batch's step kernel (or one persistent kernel doing them), then the clock
// advance by the steps they span
static lbm_status batch_launch(lbm_batch* b, int nl) {
  const int n = (int)b->ctx.size();
  const int d = shape_def(b->precision, b->shape).depth;
  bool open = false;
  for (const lbm_ctx* h : b->ctx) open = open || (h->prm.y_walls && h->prm.open_top);
  if (b->persistent) {
    int grid = 0;
    lbm_status st = persistent_grid(b, &grid);
    if (st != LBM_OK) return st;
    grid_bar_reset_kernel<<<1, 64, 0, b->stream>>>(b->d_bar);
    persist_step(b->precision, b->qg, b->shape, grid, b->stream, b->d_table, n, b->d_clock, b->total_tiles, nl,
                 open ? 1 : 0, b->d_bar, b->spin_limit);
    clock_advance_kernel<<<1, 64, 0, b->stream>>>(b->d_clock, (long long)nl * d);
    HIP_OR_FAIL(b->ctx[0], hipGetLastError());
    b->persistent_used = true;
    return LBM_OK;
  }
  for (int s = 0; s < nl; ++s) {
    launch_step(b->precision, b->qg, b->shape, b->total_tiles, b->stream, b->d_table, n, b->d_clock, s, FROM_CLOCK);
    if (open) launch_open_top(b->precision, n, b->stream, b->d_table, b->d_clock, s, FROM_CLOCK);
  }
  clock_advance_kernel<<<1, 64, 0, b->stream>>>(b->d_clock, (long long)nl * d);
  HIP_OR_FAIL(b->ctx[0], hipGetLastError());
  return LBM_OK;
}

// Up to k steps of every instance with budget left (each stops at its own budget); *advanced
// receives the batch steps taken (0 once no instance has budget left).
static lbm_status batch_advance(lbm_batch* b, int64_t k, int64_t* advanced) {
  *advanced = 0;
  lbm_ctx* h0 = b->ctx[0];
  // a member that failed was parked by lbm_batch_sync (budget 0): the others go on
  int64_t maxrem = 0;
  for (int64_t r : b->remaining) maxrem = std::max(maxrem, r);
  const int64_t todo = std::min(k, maxrem);
  if (todo == 0) return LBM_OK;
  *advanced = todo;
  lbm_status st = batch_upload(b, todo);  // every call: the step window of each instance
  if (st != LBM_OK) return st;
  if (b->total_tiles == 0) return LBM_OK;
  const int d = shape_def(b->precision, b->shape).depth;
  const int64_t launches = (todo + d - 1) / d;
  const int64_t per_graph = GRAPH_STEPS / d;
  int64_t left = launches;
  while (left >= per_graph && b->stream != nullptr) {
    if (!b->graph) {
      hipGraph_t g = nullptr;
      HIP_OR_FAIL(h0, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
      lbm_status s = batch_launch(b, (int)per_graph);
      hipError_t e = hipStreamEndCapture(b->stream, &g);
      if (s != LBM_OK) return s;
      if (e != hipSuccess) return fail(h0, LBM_E_DEVICE, "hipStreamEndCapture failed");
      e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) {
        b->graph = nullptr;
        return fail(h0, LBM_E_DEVICE, "hipGraphInstantiate failed");
      }
    }
    HIP_OR_FAIL(h0, hipGraphLaunch(b->graph, b->stream));
    left -= per_graph;
  }
  if (left > 0) {
    lbm_status s = batch_launch(b, (int)left);
    if (s != LBM_OK) return s;
  }
  b->clock += launches * d;
  for (size_t i = 0; i < b->ctx.size(); ++i) {
    const int64_t ran = std::min<int64_t>(todo, b->remaining[i]);
    b->pending[i] += ran;
    b->ctx[i]->batch_unsynced += ran;
    b->pending_launches[i] += (ran + d - 1) / d;
    b->pending_hmoves[i] += history_moves(ran, d);
    b->remaining[i] -= ran;
    if (ran > 0) b->moved[i] = 1;
  }
  return LBM_OK;
}

// The FP64 mass and energy of member i after the launches enqueued so far, as the next record of
// its diagnostics log, on the batch's stream (its buffers are those after its pending launches).
static lbm_status enqueue_member_diagnostics(lbm_batch* b, size_t i) {
  lbm_ctx* h = b->ctx[i];
  const bool odd = ((h->gen ^ (int)(b->pending_launches[i] & 1)) & 1) != 0;
  const void* f = odd ? h->fB : h->fA;
  const void* g = odd ? h->gB : h->gA;
  lbm_status s = enqueue_diagnostics_of(h, b->stream, f, g, h->d_ring + h->diag_enqueued % DIAG_RING,
                                        (long long)(h->steps + b->pending[i]));
  if (s == LBM_OK) ++h->diag_enqueued;
  return s;
}

lbm_status lbm_batch_step(lbm_batch* b, int64_t k) {
  lbm::HostRange range_("lbm_batch_step");
  if (!b || k < 0) return LBM_E_INVAL;
  if (k == 0) return LBM_OK;
  int64_t adv = 0;
  if (b->diag_every <= 0) return batch_advance(b, k, &adv);
  // diagnostics every diag_every batch steps: the launches are split there and each member that
  // advanced since its last record gets one
  while (k > 0) {
    const int64_t seg = std::min(k, b->diag_every - b->diag_since);
    lbm_status st = batch_advance(b, seg, &adv);
    if (st != LBM_OK) return st;
    if (adv == 0) break;
    k -= seg;
    b->diag_since += adv;
    // a record at every k-th batch step, and where the last budget ran out inside an interval
    if (b->diag_since >= b->diag_every || adv < seg) {
      for (size_t i = 0; i < b->ctx.size(); ++i)
        if (b->moved[i]) {
          st = enqueue_member_diagnostics(b, i);
          if (st != LBM_OK) return st;
          b->moved[i] = 0;
        }
      b->diag_since = 0;
    }
  }
  return LBM_OK;
}

lbm_status lbm_batch_set_diagnostics_interval(lbm_batch* b, int64_t k) {
  if (!b || k < 0) return LBM_E_INVAL;
  b->diag_every = k;
  b->diag_since = 0;
  std::fill(b->moved.begin(), b->moved.end(), (char)0);
  return LBM_OK;
}

lbm_status lbm_batch_sync(lbm_batch* b, lbm_status* status) {
  lbm::HostRange range_("lbm_batch_sync");
  if (!b) return LBM_E_INVAL;
  const size_t n = b->ctx.size();
  // The launches already enqueued have advanced the members (their buffer parities and step
  // counts follow them whatever the outcome of the wait).
  for (size_t i = 0; i < n; ++i) {
    lbm_ctx* h = b->ctx[i];
    h->steps += b->pending[i];
    h->batch_unsynced = 0;
    h->gen ^= (int)(b->pending_launches[i] & 1);
    h->hgen ^= (int)(b->pending_hmoves[i] & 1);
    b->pending[i] = 0;
    b->pending_launches[i] = 0;
    b->pending_hmoves[i] = 0;
  }
  // A device error leaves every member's state unknown: each is marked failed (LBM_E_DEVICE in
  // status[]) and parked.
  auto device_failure = [&](lbm_ctx* h, const char* call, hipError_t e) {
    const std::string msg = std::string(call) + ": " + hipGetErrorString(e);
    for (size_t i = 0; i < n; ++i) {
      b->ctx[i]->failed = true;
      b->ctx[i]->last_error = "batched run: " + msg;
      b->remaining[i] = 0;
      if (status) status[i] = LBM_E_DEVICE;
    }
    return fail(h, LBM_E_DEVICE, msg);
  };
  hipError_t e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return device_failure(b->ctx[0], "hipStreamSynchronize", e);
  if (b->persistent_used) {
    GridBar bar{};
    e = hipMemcpy(&bar, b->d_bar, sizeof(bar), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return device_failure(b->ctx[0], "hipMemcpy", e);
    b->persistent_used = false;
    if (bar.abort) {
      for (size_t i = 0; i < n; ++i) {
        b->ctx[i]->failed = true;
        b->ctx[i]->last_error = "batched run: a grid barrier wait of the persistent kernel timed out";
        b->remaining[i] = 0;
        if (status) status[i] = LBM_E_DEVICE;
      }
      return fail(b->ctx[0], LBM_E_DEVICE, "persistent kernel: a grid barrier wait timed out");
    }
  }
  lbm_status worst = LBM_OK;
  for (size_t i = 0; i < n; ++i) {
    lbm_ctx* h = b->ctx[i];
    unsigned err = 0;
    e = hipMemcpy(&err, h->d_err, sizeof(unsigned), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return device_failure(h, "hipMemcpy", e);
    if (err && !h->failed) {
      h->failed = true;
      h->last_error = "numerical failure on the device (batched run)";
    }
    if (h->failed) {
      b->remaining[i] = 0;
      worst = LBM_E_NUMERIC;
    }
  }
  if (status)
    for (size_t i = 0; i < n; ++i) status[i] = b->ctx[i]->failed ? LBM_E_NUMERIC : LBM_OK;
  return worst;
}

lbm_status lbm_batch_destroy(lbm_batch* b) {
  if (!b) return LBM_E_INVAL;
  // the members are not touched: they may already be destroyed
  if (b->graph) (void)hipGraphExecDestroy(b->graph);
  lbm_status s = LBM_OK;
  if (b->noalloc_device >= 0) s = release_static_area(b);
  delete b;
  return s;
}

lbm_status lbm_batch_create_noalloc(lbm_ctx* const* ctxs, int n, void* hip_stream, lbm_batch** out) {
  if (!out || !ctxs || n <= 0 || n > LBM_BATCH_NOALLOC_MAX) return LBM_E_INVAL;
  *out = nullptr;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return LBM_E_DEVICE;
  for (int i = 0; i < n; ++i)
    if (!ctxs[i] || ctxs[i]->device != dev) return LBM_E_INVAL;
  std::lock_guard<std::mutex> lock(g_area_mu);
  if (g_area_busy[dev]) return LBM_E_STATE;
  void* area = nullptr;
  const lbm_status a = static_area(dev, &area);
  if (a != LBM_OK) return a;
  const lbm_status s = lbm_batch_create(ctxs, n, area, STATIC_AREA_BYTES, hip_stream, out);
  if (s != LBM_OK) return s;
  (*out)->noalloc_device = dev;
  g_area_busy[dev] = true;
  return LBM_OK;
}

}  // extern "C"
