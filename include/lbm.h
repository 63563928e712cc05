/*
 * lbm.h -- C ABI of the MI355X (gfx950) library for the thermal pseudopotential lattice
 * Boltzmann model of L. Wang, J. Huang, K. He, "A new thermal lattice Boltzmann model for
 * liquid-vapor phase change" (arXiv:2205.00686).
 *
 * One time step is the fused D2Q9 MRT pseudopotential flow step (Section 2, Eqs. 1-11:
 * Peng-Robinson pressure, pseudopotential, interaction/wetting/buoyancy forces, Li et al.'s
 * forcing in moment space, streaming) coupled to the D2Q5 MRT temperature step with the
 * rho*c_v-modified collision and linear equilibrium (Section 3.2, Eqs. 20-26 and 39-53).
 *
 * Conventions shared by every entry point:
 *   - Lattice units, dx = dt = 1.  Grid nx x ny nodes; host fields are FP64, row-major
 *     [ny][nx] with x fastest, owned by the caller.
 *   - Device memory is owned by the caller: one allocation of lbm_footprint_bytes() bytes
 *     (any 256-byte aligned device pointer, e.g. a torch uint8 tensor), which must outlive
 *     the context.  The library allocates no device memory of its own.
 *   - Work is enqueued on the HIP stream given at creation (hipStream_t passed as void*;
 *     NULL = the null stream).  lbm_step is asynchronous; calls that return host data
 *     synchronise the stream.
 *   - Every call returns an lbm_status; lbm_last_error() gives the text of the last error on
 *     a context.  A numerical failure detected on the device (density <= 0, temperature
 *     <= 0, a pseudopotential argument < 0, NaN/Inf) is sticky: it is reported as
 *     LBM_E_NUMERIC by the next synchronising call and every later call on the context.
 *   - One context per stream; calls on one context are not thread-safe.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;
typedef struct lbm_batch lbm_batch;

typedef enum {
  LBM_OK = 0,
  LBM_E_INVAL = -1,   /* invalid argument or parameter set */
  LBM_E_NOMEM = -2,   /* device buffer smaller than the footprint */
  LBM_E_DEVICE = -3,  /* a HIP runtime call failed */
  LBM_E_NUMERIC = -4, /* the device flagged a numerical failure (sticky) */
  LBM_E_STATE = -5    /* call out of order (step before init) or context already failed */
} lbm_status;

enum { LBM_FP32 = 0, LBM_FP64 = 1 };

/* Flags.  LBM_FREEZE_FLOW and LBM_NO_S are for tests: they zero terms inside the one step
   kernel and add no code path.  LBM_BGK selects the BGK model of Eq. (21) for the D2Q5 thermal
   lattice: every D2Q5 rate is set to 1/tau_g (vs3 and vs4 are then ignored), which is the MRT
   step of Eq. (39) with Lambda = I / tau_g. */
enum {
  LBM_FREEZE_FLOW = 1u, /* populations f are not updated; u = (sum c_i f_i)/rho, no force */
  LBM_NO_S = 2u,        /* correction term S_i of Eq. (24) switched off */
  LBM_BGK = 8u          /* D2Q5 thermal populations with the BGK collision of Eq. (21) */
};

/* Parameters of the problem statement.  lbm_params_default() fills the paper's values. */
typedef struct {
  int32_t nx, ny;        /* grid size, each >= 3 */
  int32_t precision;     /* LBM_FP32: populations stored and collided in FP32; LBM_FP64 */
  /* thermal lattice: 5 (D2Q5 with the MRT of Eq. 39, the paper's model; 0 also means 5) or 9
     (D2Q9 with the BGK collision of Eq. 21, the linear equilibrium of Eq. 22 with the D2Q9
     weights, chat_s^2 = 1/3, grad T from the first moment as in Eqs. 49-50).  D2Q9 ignores
     wdot, vs3 and vs4; it runs on the one-step tile shapes only. */
  int32_t thermal_q;
  /* Peng-Robinson EOS (Eq. 10): a = 3/49, b = 2/21, R = 1, acentric factor 0.344;
     interaction strength G = -1 (Eq. 9) */
  double a, b, R, acentric, G;
  /* D2Q9 MRT (Eq. 5): kinematic viscosity nu gives s_p = 1/(3 nu + 1/2); s_e, s_eps, s_q;
     sigma of Li et al.'s forcing (Eq. 8); all rates not tied to nu are 1 (Section 4) */
  double nu, s_e, s_eps, s_q, sigma;
  /* D2Q5 MRT (Eqs. 26, 39, 53): conductivity lambda gives varsigma_1 = varsigma_2 =
     1/(lambda/chat_s^2 + 1/2) with chat_s^2 = wdot/2; heat capacity c_v; weight parameter
     wdot in (0,1); relaxation rates varsigma_3, varsigma_4 */
  double lambda, cv, wdot, vs3, vs4;
  /* buoyancy F_b = (rho - rho_ave) g (Section 4.3, rho_ave the mean density of the whole domain).
     rho_ave = NaN: that mean, in FP64.  On closed and periodic domains mass is conserved and the
     mean of the initial density is used throughout; with an open top the device tracks the mass
     that crosses the top in each step (FP64, added by the boundary pass after the step), so
     rho_ave is the mean density of the current state at every step.  A finite rho_ave is used as
     a constant. */
  double gx, gy, rho_ave;
  int32_t y_walls;       /* 0: periodic in y; 1: no-slip halfway walls at y=-1/2 and ny-1/2 */
  int32_t thermal_box;   /* 1: Dirichlet T = T_box on all four edges (flow stays periodic) */
  /* wall temperatures (y_walls = 1): T_bot(x) = T_bot + hot_dT exp(-(x-hot_x0)^2/(2 hot_sigma^2)),
     T_top; applied by halfway anti-bounce-back */
  double T_box, T_top, T_bot, hot_dT, hot_x0, hot_sigma;
  double theta_bot_deg, theta_top_deg; /* contact angles of the geometric wetting rule (Eq. 54) */
  uint32_t flags;        /* LBM_FREEZE_FLOW | LBM_NO_S (tests only) | LBM_BGK */
  /* with y_walls = 1: the top is an open boundary (the outflow condition the paper uses for
     its open-top problems, Sections 4.2-4.3, read as the convective outflow condition of the
     populations entering the top row: f_i(x,N,t+1) = [f_i(x,N,t) + U f_i(x,N-1,t+1)]/(1+U),
     U = j_y/rho of the top node at time t clipped to [0,1]; zero-gradient pseudopotential and
     velocity above it; the temperature stays T_top).  Runs on the one-step tile shapes; mass
     leaves and enters through the top. */
  int32_t open_top;
} lbm_params;

/* Fill *p with the paper's parameter values (Sections 2 and 4) for an nx x ny FP32 grid. */
void lbm_params_default(lbm_params* p, int32_t nx, int32_t ny);

/* Check a parameter set without touching the device.  LBM_E_INVAL if nx or ny < 3, one
   population plane (nx * ny values) exceeds 2^32 - 1 bytes (about 1.07e9 nodes in FP32,
   5.4e8 in FP64), a relaxation rate is outside (0, 2), wdot outside (0, 1), c_v <= 0, nu <= 0,
   lambda <= 0, thermal_q is not 0, 5 or 9, flags holds an unknown bit, or open_top is set
   without y_walls. */
lbm_status lbm_validate(const lbm_params* p);

/* Exact device bytes a context needs (populations f and g and the temperature history, each
   in two copies, and a small control block: 128 B per node in FP32 with the D2Q5 thermal
   lattice, 160 B with D2Q9; twice that in FP64; plus 48 KiB); 0 if lbm_validate fails. */
size_t lbm_footprint_bytes(const lbm_params* p);

/* Create a context on the current HIP device over caller-owned device memory dev_mem of
   `bytes` bytes (256-byte aligned), enqueueing on hip_stream.  *out receives the handle.
   LBM_E_INVAL on bad parameters or a misaligned pointer, LBM_E_NOMEM if bytes is smaller than
   lbm_footprint_bytes(p). */
lbm_status lbm_create(const lbm_params* p, void* dev_mem, size_t bytes, void* hip_stream, lbm_ctx** out);

/* Initial state from host FP64 fields (each nx*ny): f_i = f_i^eq(rho, u) (Eq. 3),
   g_i = what_i T (Eq. 22), temperature history = T.  Computes rho_ave if it is NaN.
   LBM_E_INVAL if rho or T is not positive and finite, or min(rho) * c_v < 1 (the modified
   collision of Eq. 39 weights the old population by 1 - 1/(rho c_v), which must not be
   negative).  Synchronises the stream. */
lbm_status lbm_init(lbm_ctx* h, const double* rho, const double* ux, const double* uy, const double* T);

/* Enqueue n time steps (Eqs. 1-11 then 20-53, one fused kernel per step).  Asynchronous.
   LBM_E_STATE before lbm_init or after a failure. */
lbm_status lbm_step(lbm_ctx* h, int64_t n);

/* Number of steps taken since lbm_init (or the count restored by lbm_load_state). */
int64_t lbm_steps_done(const lbm_ctx* h);

/* Tile shapes of the step kernel.  A workgroup of `waves` wavefronts updates a tile_x x tile_y
   block of nodes, steps_per_launch (1 or 2) time steps per kernel launch; the library holds
   lbm_shape_count(precision) shapes, numbered from 0.  The shape decides only how the work is
   grouped into workgroups and launches: every shape gives bit-identical results.
   lbm_shape_info: LBM_E_INVAL for an unknown precision or k; NULL outputs are skipped.
   A two-step shape keeps the first step's result for the tile and its halo in LDS, which needs
   a grid larger than that halo region, the D2Q5 thermal lattice (the D2Q9 populations do not
   fit in LDS twice) and no open top (its boundary pass runs between steps): lbm_shape_fits
   tells whether shape k can run the simulation of *p (1) or not (0, also for invalid
   parameters). */
int lbm_shape_count(int32_t precision);
lbm_status lbm_shape_info(int32_t precision, int k, int* tile_x, int* tile_y, int* waves, int* steps_per_launch);
int lbm_shape_fits(const lbm_params* p, int k);

/* Use shape k for the context's later steps (k = -1: the library's choice from the grid size,
   the default).  Ordered on the context's stream after the steps already enqueued; waits for
   that stream.  LBM_E_INVAL for k outside [-1, lbm_shape_count) or a shape that does not fit
   the grid (lbm_shape_fits). */
lbm_status lbm_set_shape(lbm_ctx* h, int k);

/* The shape in use (never -1); -1 for a NULL context. */
int lbm_get_shape(const lbm_ctx* h);

/* Order in which a launch's workgroups take the tiles of the context (results do not depend on it):
   order = 0, the default: strips of 8 tile columns, each walked from the bottom tile row to the
   top, where the context's state exceeds the 256 MB Infinity Cache (the halo rows a tile reads are
   then still in the L2 of its XCD), whole tile rows in order otherwise; 1: whole rows; k >= 2:
   strips of k tile columns.  Applies to later steps, also in batches.  Waits for the stream.
   LBM_E_INVAL for order < 0.  lbm_get_tile_order: the strip width in use, in tiles (the number of
   tile columns for whole rows); -1 for a NULL context. */
lbm_status lbm_set_tile_order(lbm_ctx* h, int order);
int lbm_get_tile_order(const lbm_ctx* h);

/* Wait for the stream and report any device-side numerical failure. */
lbm_status lbm_sync(lbm_ctx* h);

/* Current macroscopic fields to host FP64 arrays (each nx*ny, any may be NULL):
   rho = sum f_i, u = (sum c_i f_i + F_n/2)/rho with the force of the current state (Eq. 11),
   T = sum g_i (Eq. 25).  Synchronises. */
lbm_status lbm_read_fields(lbm_ctx* h, double* rho, double* ux, double* uy, double* T);

/* Mass sum(rho) and thermal energy sum(rho c_v T) of the current state, accumulated in FP64
   in a fixed order (deterministic; the reduction of lbm_set_diagnostics_interval).  Synchronises. */
lbm_status lbm_diagnostics(lbm_ctx* h, double* mass, double* energy);

/* Diagnostics every k steps, off the step kernel: with k > 0 every later lbm_step enqueues, after
   each step whose count since lbm_init is a multiple of k, the FP64 reduction of lbm_diagnostics
   (a thread's nodes, then the 64 lanes of a wavefront by cross-lane shuffles, then the wavefronts,
   then the per-workgroup partials, each in a fixed order, so the values are deterministic and
   equal to lbm_diagnostics at that step) as its own kernels on the context's stream; the record
   (step count, mass, energy) goes to a ring of LBM_DIAG_RING records in the context's device
   memory, where the oldest are overwritten.  k = 0 stops it.  Either value of k clears the log.
   LBM_E_INVAL for k < 0. */
#define LBM_DIAG_RING 256
lbm_status lbm_set_diagnostics_interval(lbm_ctx* h, int64_t k);

/* The records enqueued since the last call (at most the last LBM_DIAG_RING of them), oldest first,
   up to max of them, into caller-owned host arrays steps[max], mass[max], energy[max]; *count
   receives how many.  Synchronises (a numerical failure is reported as by lbm_sync).  LBM_E_INVAL
   for NULL outputs or max < 0, LBM_E_STATE before lbm_init. */
lbm_status lbm_read_diagnostics_log(lbm_ctx* h, int64_t* steps, double* mass, double* energy, int max, int* count);

/* Vapour profile of the current state, for the bubble-departure readout of Section 4.3
   (departure diameter against gravity): counts[y] = number of columns x in [x_lo, x_hi)
   (taken modulo nx, so the window may wrap) whose density is below rho_threshold, for every
   row y of the grid.  The density is summed in the working precision as in lbm_read_fields and
   compared with rho_threshold rounded to that precision.  counts: caller-owned host array of ny
   ints.  Computed on the device; synchronising.  LBM_E_INVAL for a window wider than nx or
   empty, a non-finite threshold or NULL pointers; LBM_E_STATE before lbm_init. */
lbm_status lbm_vapour_rows(lbm_ctx* h, double rho_threshold, int x_lo, int x_hi, int32_t* counts);

/* One vapour component of lbm_vapour_components: a connected set of vapour nodes (8-connected,
   periodic in x).  root is the smallest node index y*nx + x of the component, area its number of
   nodes, [y_min, y_max] and [x_min, x_max] the rows and columns it occupies (column indices as
   stored, so a component that wraps around x spans from near 0 to near nx - 1), and y_sum the sum
   of its nodes' rows (centroid row = y_sum / area). */
typedef struct lbm_component {
  int32_t root, area, y_min, y_max, x_min, x_max;
  int64_t y_sum;
} lbm_component;

#define LBM_MAX_COMPONENTS 4096

/* Vapour components of the current state, for the bubble-departure readout of Section 4.3: a
   departed bubble is a component that touches neither the heated wall nor the vapour above the
   pool.  The vapour nodes are those of rows [y_lo, y_hi) whose density, summed in the working
   precision as in lbm_read_fields, is below rho_threshold when compared in FP64 (so exactly the
   nodes where the density lbm_read_fields returns is below it).  Labelled on the device by
   union-find; the result does not depend on the order of execution.  *n_total receives the
   number of components; the first min(n_total, max_out) of them in increasing root order are
   written to the caller-owned host array out[max_out].  The labels use the buffers the next step
   overwrites before reading them, so the state is not changed.  Synchronising.
   LBM_E_INVAL for an empty or out-of-grid row range, a non-finite threshold, max_out < 0 or NULL
   pointers, and for more than LBM_MAX_COMPONENTS components (possible only where the rows hold
   more than about 16 000 nodes; *n_total is still set); LBM_E_STATE before lbm_init
   or for a batch member whose steps lbm_batch_sync has not yet brought up to date. */
lbm_status lbm_vapour_components(lbm_ctx* h, double rho_threshold, int y_lo, int y_hi, lbm_component* out,
                                 int max_out, int* n_total);

/* Raw state to / from a caller-owned host buffer of lbm_state_bytes() bytes: f[9][ny][nx],
   g[Q][ny][nx] (Q = 5 or 9, the thermal lattice), history[2][ny][nx] in the context's precision,
   then a 64-byte trailer: magic "LBM2D", format version, precision, nx, ny, Q, the step count
   (int64), rho_ave, T_ref and the tracked mass (FP64).  The temperature populations are stored
   relative to T_ref (the mean initial temperature): the buffer holds g_i - what_i T_ref and
   T - T_ref for the history.  Resuming from a saved state reproduces an uninterrupted run bit for
   bit.  lbm_save_state: LBM_E_STATE before lbm_init, LBM_E_INVAL for a smaller buffer; synchronises.
   lbm_load_state: LBM_E_INVAL unless bytes equals lbm_state_bytes() and the trailer names this
   format, the context's precision, grid and thermal lattice; then the context is initialised from
   the buffer (it need not have been initialised before); synchronises. */
size_t lbm_state_bytes(const lbm_ctx* h);
lbm_status lbm_save_state(lbm_ctx* h, void* host, size_t bytes);
lbm_status lbm_load_state(lbm_ctx* h, const void* host, size_t bytes);

/* The current populations as FP64 host arrays with the storage offset undone (any may be NULL):
   f[9][ny][nx], g[Q][ny][nx] = the thermal populations g_i of Eq. (22)'s lattice (Q = 5 or 9),
   hist[2][ny][nx] = T(t-1), T(t-2).  For checks and inspection; synchronises.  LBM_E_STATE before
   lbm_init, LBM_E_NOMEM if the host staging buffer cannot be allocated. */
lbm_status lbm_read_state(lbm_ctx* h, double* f, double* g, double* hist);

/* Maxwell equal-area coexistence of the Peng-Robinson EOS at temperature T (host, FP64):
   rho_l, rho_g, p_sat.  LBM_E_INVAL if T is at or above the critical temperature. */
lbm_status lbm_eos_coexistence(const lbm_params* p, double T, double* rho_l, double* rho_g, double* p_sat);

/* Critical temperature 0.0778 a / (0.45724 b R) implied by a and b (text after Eq. 10). */
double lbm_critical_temperature(const lbm_params* p);

/* Release the context (host metadata only; the caller frees the device memory). */
lbm_status lbm_destroy(lbm_ctx* h);

const char* lbm_strerror(lbm_status s);
const char* lbm_last_error(const lbm_ctx* h);

/* Device-to-device copy of `bytes` bytes (a multiple of 16; both pointers 16-byte aligned device
   memory owned by the caller) by a streaming kernel with 16-byte lanes, enqueued on hip_stream
   (asynchronous).  Not part of the method: it gives the practical HBM ceiling the step kernels are
   measured against, and a kernel of known traffic (bytes read plus bytes written) that calibrates
   hardware byte counters in profiles.  LBM_E_INVAL for NULL or misaligned pointers or a size that
   is not a multiple of 16; LBM_E_DEVICE if the launch fails. */
lbm_status lbm_device_copy(const void* src, void* dst, size_t bytes, void* hip_stream);

/* ------------------------------------------------------------------------------------
 * Batched execution: many initialised contexts (uneven grids and parameters, same precision and
 * same device) advanced together, each step one kernel launch over the tiles of every
 * active instance; launches are captured in a HIP graph and replayed.  Each instance's
 * arithmetic is exactly that of its own lbm_step, so results are bit-identical to running it
 * alone.  A batch needs lbm_batch_footprint_bytes(n) bytes of caller-owned device memory.
 */
size_t lbm_batch_footprint_bytes(int n);

/* Build a batch over ctxs[0..n) (all initialised, same precision and thermal lattice),
   enqueueing on hip_stream.
   The batch's work is ordered after everything already enqueued on the contexts' own streams
   (their lbm_init, for instance), so a context may be initialised on a stream of its own.
   While the batch exists its members are advanced only through it.  Once lbm_batch_sync has
   returned, a member may be used on its own stream (lbm_read_fields, lbm_step, ...) or
   destroyed.  Between an lbm_batch_step that advanced a member and the next lbm_batch_sync, the
   calls that read, write or advance that member's state on its own (lbm_init, lbm_step,
   lbm_read_fields, lbm_read_state, lbm_diagnostics, lbm_read_diagnostics_log, lbm_vapour_rows,
   lbm_vapour_components, lbm_save_state, lbm_load_state, and lbm_batch_create with it as a
   member) return LBM_E_STATE.
   LBM_E_DEVICE if the stream ordering cannot be set up. */
lbm_status lbm_batch_create(lbm_ctx* const* ctxs, int n, void* dev_mem, size_t bytes, void* hip_stream,
                            lbm_batch** out);

/* Give instance i a budget of `steps` more steps (0 parks it).  Takes effect at the next
   lbm_batch_step.  LBM_E_STATE for an instance that has failed. */
lbm_status lbm_batch_set_budget(lbm_batch* b, int i, int64_t steps);

/* Advance every instance with budget left by up to k steps (each stops at its own budget).
   An instance whose failure lbm_batch_sync has reported stays parked; the others go on. */
lbm_status lbm_batch_step(lbm_batch* b, int64_t k);

/* Steps still budgeted for instance i. */
int64_t lbm_batch_remaining(const lbm_batch* b, int i);

/* Tile shape of the batched launches (k = -1: chosen from the batch's total size, the
   default); the members' own shapes are not used by the batch.  LBM_E_INVAL for k outside
   [-1, lbm_shape_count) or a shape that does not fit every member's grid. */
lbm_status lbm_batch_set_shape(lbm_batch* b, int k);
int lbm_batch_get_shape(const lbm_batch* b);

/* Persistent launches (on = 1): each group of launches of the batch (up to the steps captured in one
   graph replay) becomes one kernel whose workgroups, as many as are resident on the device at once,
   loop over the tiles of every active instance launch after launch, with a grid barrier between
   launches (and around the open-top pass of members that have one).  Results are bit-identical to
   the launch-per-step form (on = 0, the default).  The barrier's wait is bounded by spin_limit
   polls with a short sleep in between (0: 2^24): a workgroup that waits longer, which can happen
   when other work keeps part of the grid from being resident, flags the batch and every workgroup
   leaves the kernel; lbm_batch_sync then marks every member failed with LBM_E_DEVICE.
   LBM_E_INVAL for on other than 0 or 1. */
lbm_status lbm_batch_set_persistent(lbm_batch* b, int on, uint32_t spin_limit);

/* Diagnostics of the members every k steps of the batch (the A12 reduction of lbm_diagnostics,
   Section 4: FP64 mass and thermal energy), counted over lbm_batch_step calls from this call on:
   lbm_batch_step splits its launches at every k-th batch step and enqueues, on the batch's stream,
   the reduction of each member that advanced since its previous record into that member's
   diagnostics log, tagged with the member's own step count (a member whose budget ended inside
   the interval is recorded at the step where it stopped).  When every budget runs out inside an
   interval, the members that advanced are recorded there and the count starts again.  The records are read with
   lbm_read_diagnostics_log on the member once lbm_batch_sync has returned; they equal
   lbm_diagnostics of the member at that step bit for bit, and the simulations' results do not
   change.  k = 0 stops.  LBM_E_INVAL for k < 0. */
lbm_status lbm_batch_set_diagnostics_interval(lbm_batch* b, int64_t k);

/* Wait for the batch's stream; report per-instance failures in status[n] (may be NULL):
   LBM_E_NUMERIC for a member whose device error word is set (it is parked; returns LBM_E_NUMERIC),
   LBM_OK for the others.  The contexts' step counters and buffer parities are brought up to date.
   If the wait or a read-back fails, or a persistent launch's barrier wait timed out, every member
   is marked failed and parked, status[] holds LBM_E_DEVICE for all of them and the call returns
   LBM_E_DEVICE. */
lbm_status lbm_batch_sync(lbm_batch* b, lbm_status* status);

/* Release the batch.  The caller-owned memory stays in use until the batch's stream has
   drained.  The members are not touched, so they may be destroyed before the batch.  A batch made
   by lbm_batch_create_noalloc first waits for its stream (LBM_E_DEVICE if that wait fails), then
   frees its device's static area for the next such batch. */
lbm_status lbm_batch_destroy(lbm_batch* b);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
   loops, harnesses that forbid allocation): lbm_batch_create without the caller's table memory.
   The batch's instance table and clock live in a static device array of the library instead, one
   per device, sized for LBM_BATCH_NOALLOC_MAX instances (about 130 KiB, held by each device the
   library runs on until the process ends).  Everything else is as lbm_batch_create, and the batch
   gives the same results.  The members must be on the current device.  One such batch may exist
   per device at a time: LBM_E_STATE while another one does (lbm_batch_destroy releases it).  The
   area keeps the last batch's table; every lbm_batch_step rewrites it before its launches, so
   nothing has to be cleared, but work on one device that reaches the area by other means while a
   batch uses it races.  LBM_E_INVAL for n outside [1, LBM_BATCH_NOALLOC_MAX], a NULL or
   foreign-device member; LBM_E_DEVICE if the area's device address cannot be obtained.  Allocates
   no device memory (host metadata only, as lbm_batch_create). */
#define LBM_BATCH_NOALLOC_MAX 256
lbm_status lbm_batch_create_noalloc(lbm_ctx* const* ctxs, int n, void* hip_stream, lbm_batch** out);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
