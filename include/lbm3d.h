/*
 * C ABI of the three-dimensional extension of the thermal pseudopotential lattice Boltzmann
 * model of Wang, Huang & He (arXiv:2205.00686): D3Q19 MRT pseudopotential flow coupled to the
 * paper's temperature model on the D3Q7 lattice, which its introduction names as the
 * three-dimensional form of its linear-equilibrium thermal model (no three-dimensional formulas
 * are printed; the lattice choices follow the two-dimensional model):
 *   - flow: d'Humieres' orthogonal D3Q19 moment basis, MRT collision with Li et al.'s forcing
 *     (Eq. 8; the sigma term adds to each diagonal component of the second-moment source what it
 *     adds in two dimensions, so sigma carries over), interaction force of Eq. (9) with the D3Q19
 *     weights 1/6 (axes) and 1/12 (face diagonals), Peng-Robinson EOS (Eq. 10);
 *   - temperature: D3Q7 populations, what_0 = 1 - wdot, what_{1..6} = wdot/6 (chat_s^2 = wdot/3),
 *     non-orthogonal MRT (rows 1, c_x, c_y, c_z, c^2, c_x^2 - c_y^2, c_x^2 - c_z^2; Eqs. 39-40,
 *     47), source Q (Eq. 20) with grad T from the first moments (Eqs. 49-50), correction S
 *     (Eq. 24), the rho c_v-modified collision term (Eq. 39), anti-bounce-back at Dirichlet faces.
 * Domains: periodic in x, y and z; optionally a Dirichlet temperature T_box on all six faces
 * (the flow stays periodic).  Status codes and their meaning are those of lbm.h.
 *
 * Layout in the caller's device memory: f[19][nz][ny][nx], g[7][nz][ny][nx], the temperature
 * history [2][nz][ny][nx] (x fastest), the populations in two copies, plus per-node fields of
 * the current step (15 planes) and a small control block.
 *
 * Two step paths give the same results up to the summation order of div u:
 *   LBM3D_PATH_FUSED (default): one kernel per step; 64 x 8 column tiles, each workgroup marching
 *     through a chunk of z planes with psi, u and the streaming-destination values in LDS;
 *   LBM3D_PATH_PER_NODE: three kernels per step, per-node fields in HBM between them.
 */
#ifndef LBM3D_H
#define LBM3D_H
#include <stddef.h>
#include <stdint.h>

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm3d_ctx lbm3d_ctx;

typedef struct {
  int32_t nx, ny, nz;       /* grid, each >= 3 */
  int32_t precision;        /* LBM_FP32 or LBM_FP64 */
  double a, b, R, acentric, G; /* Peng-Robinson EOS (Eq. 10), interaction strength (Eq. 9) */
  /* D3Q19 MRT: kinematic viscosity nu gives the rate of the five second-order stress moments,
     1/(3 nu + 1/2); s_e, s_eps the energy rates; every other rate is 1; sigma of Eq. (8) */
  double nu, s_e, s_eps, sigma;
  /* D3Q7: conductivity lambda gives varsigma = 1/(lambda/chat_s^2 + 1/2) for the first moments,
     chat_s^2 = wdot/3; heat capacity c_v; vs3 the rate of the three second-order moments */
  double lambda, cv, wdot, vs3;
  int32_t thermal_box;      /* 1: T = T_box on all six faces */
  int32_t z_chunk;          /* fused path: z planes per workgroup; 0 = about one workgroup per CU */
  double T_box;
  uint32_t flags;           /* LBM_FREEZE_FLOW | LBM_NO_S, tests only */
  uint32_t path;            /* LBM3D_PATH_FUSED or LBM3D_PATH_PER_NODE */
} lbm3d_params;

#define LBM3D_PATH_FUSED 0u
#define LBM3D_PATH_PER_NODE 1u

/* The paper's values (as in two dimensions) for an nx x ny x nz FP32 grid. */
void lbm3d_params_default(lbm3d_params* p, int32_t nx, int32_t ny, int32_t nz);

/* LBM_E_INVAL if a size is < 3, a population plane exceeds 2^32 - 1 bytes, a rate is outside
   (0, 2), wdot outside (0, 1), c_v, nu or lambda <= 0, an unknown flag is set, the box
   temperature is not positive and finite, z_chunk < 0 or the path is unknown. */
lbm_status lbm3d_validate(const lbm3d_params* p);

/* Exact device bytes a context needs: 276 B per node in FP32 (f 19 and g 7 in two copies, the
   history, 15 planes of per-step fields), 552 B in FP64, plus 48 KiB; 0 if invalid. */
size_t lbm3d_footprint_bytes(const lbm3d_params* p);

/* Create a context over caller-owned device memory (256-byte aligned, at least the footprint)
   on the current device, enqueueing on hip_stream.  LBM_E_INVAL / LBM_E_NOMEM as lbm_create. */
lbm_status lbm3d_create(const lbm3d_params* p, void* dev_mem, size_t bytes, void* hip_stream, lbm3d_ctx** out);

/* Initial state from host FP64 fields (each nx*ny*nz, x fastest): f = f_eq(rho, u) (Eq. 3 on
   D3Q19), g_i = what_i T (Eq. 22), history = T.  LBM_E_INVAL for non-positive or non-finite
   rho or T, or min(rho) c_v < 1.  Synchronises. */
lbm_status lbm3d_init(lbm3d_ctx* h, const double* rho, const double* ux, const double* uy, const double* uz,
                      const double* T);

/* Enqueue n time steps (the fused path: one kernel per step; the per-node path: per-node fields,
   forces and velocity, collision and streaming).  Asynchronous.  LBM_E_STATE before init or after
   a failure. */
lbm_status lbm3d_step(lbm3d_ctx* h, int64_t n);

/* Wait for the stream; report a device-side numerical failure (sticky). */
lbm_status lbm3d_sync(lbm3d_ctx* h);

/* rho, u (with half the force of the current state), T of the current state to host FP64
   arrays (any may be NULL).  Synchronises. */
lbm_status lbm3d_read_fields(lbm3d_ctx* h, double* rho, double* ux, double* uy, double* uz, double* T);

/* FP64 sums of rho and rho c_v T over the grid (fixed order).  Synchronises. */
lbm_status lbm3d_diagnostics(lbm3d_ctx* h, double* mass, double* energy);

int64_t lbm3d_steps_done(const lbm3d_ctx* h);

/* Raw state to / from a caller-owned host buffer of lbm3d_state_bytes() bytes: f[19][nz][ny][nx],
   g[7][nz][ny][nx], history[2][nz][ny][nx] in the context's precision, then a 48-byte trailer:
   magic "LBM3D", format version, precision, nx, ny, nz, the step count (int64) and T_ref (FP64;
   g and the history are stored relative to it).  Loading restores the step count and T_ref and
   clears a failure; resuming reproduces an uninterrupted run bit for bit.  lbm3d_save_state:
   LBM_E_STATE before init, LBM_E_INVAL for a smaller buffer.  lbm3d_load_state: LBM_E_INVAL
   unless bytes equals lbm3d_state_bytes() and the trailer names this format, the context's
   precision and grid (or for a negative stored step count).  Both synchronise. */
size_t lbm3d_state_bytes(const lbm3d_ctx* h);
lbm_status lbm3d_save_state(lbm3d_ctx* h, void* host, size_t bytes);
lbm_status lbm3d_load_state(lbm3d_ctx* h, const void* host, size_t bytes);
lbm_status lbm3d_destroy(lbm3d_ctx* h);

#ifdef __cplusplus
}
#endif
#endif
