/*
 * Plain FP64 CPU oracle of the three-dimensional extension of the thermal pseudopotential
 * lattice Boltzmann model of L. Wang, J. Huang, K. He, "A new thermal lattice Boltzmann model
 * for liquid-vapor phase change" (arXiv:2205.00686): D3Q19 MRT pseudopotential flow coupled to
 * the paper's temperature model on the D3Q7 lattice (the extension the paper names in its
 * introduction; it gives no three-dimensional formulas, so every lattice-specific choice below
 * is a reading).
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/ and the cpu_baseline leg of bench.py may load this
 * library.  It shares no code with the GPU library; it is written the slow, obvious way:
 * explicit 19x19 and 7x7 transformation matrices inverted by Gauss-Jordan at set-up, moment
 * equilibria and forcing obtained by transforming the velocity-space expressions, whole-grid
 * arrays for every field of time t before anything of time t+1 is written.
 *
 * Arrays are [component][z][y][x], x fastest.  Lattice units.  Domains: periodic in all three
 * directions; optionally a Dirichlet temperature box on all six faces (flow stays periodic).
 *
 * Readings (three-dimensional counterparts of the two-dimensional ones):
 *   R3-M   D3Q19 moments of d'Humieres et al. (2002), orthogonal basis:
 *          1, 19c^2-30, (21c^4-53c^2+24)/2, c_a, (5c^2-9)c_a (a = x, y, z), 3c_x^2-c^2,
 *          (3c^2-5)(3c_x^2-c^2), c_y^2-c_z^2, (3c^2-5)(c_y^2-c_z^2), c_xc_y, c_yc_z, c_xc_z,
 *          (c_y^2-c_z^2)c_x, (c_z^2-c_x^2)c_y, (c_x^2-c_y^2)c_z.
 *          m_eq = M f_eq with the second-order equilibrium (Eq. 3 on D3Q19).
 *          Rates: 1 for every moment not tied to nu (as Section 4 for D2Q9), s_e, s_eps given,
 *          s = 1/(3 nu + 1/2) for the five second-order stress moments.
 *   R3-F   Interaction force F_m = -G psi(x) sum_i w(|c_i|^2) psi(x + c_i) c_i, w(1) = 1/6,
 *          w(2) = 1/12 (the D3Q19 counterpart of Eq. 9's 1/3, 1/12: both give the same force on a
 *          profile that varies along one axis).
 *   R3-LI  Li et al.'s forcing (Eq. 8) in moment space: F~ = M G with G the second-order
 *          (Guo) forcing term in velocity space, plus a sigma term in the two energy moments that
 *          adds to every diagonal component of the second-moment source the same amount as the
 *          two-dimensional Eq. (8) does: sigma Phi / 6 per component, Phi = |F_m|^2 / (psi^2
 *          (1/s - 1/2)).  In D2Q9 the e-moment source is 3 x (trace source) and Eq. (8) puts sigma
 *          Phi there, i.e. sigma Phi / 3 on the trace of two components; in D3Q19 the e-moment
 *          source is 19 x (trace source), the trace holds three components, so e gets
 *          19 * 3 * sigma Phi / 6 = (19/2) sigma Phi and eps, by its rho u^2 coefficient (-11/2
 *          against -3 in D2Q9), -(11/4) sigma Phi.  With this the sigma of the two-dimensional
 *          model carries over: sigma = 1.25 puts a flat interface at the Maxwell densities.
 *   R3-T   D3Q7 temperature lattice: what_0 = 1 - wdot, what_{1..6} = wdot/6, chat_s^2 = wdot/3;
 *          non-orthogonal matrix with rows 1, c_x, c_y, c_z, c^2, c_x^2 - c_y^2, c_x^2 - c_z^2
 *          (the counterpart of Eq. 40), m_eq = [T, 0, 0, 0, wdot T, 0, 0] (Eq. 47); rates
 *          1 (conserved), varsigma = 1/(lambda/chat_s^2 + 1/2) for the three first moments,
 *          vs3 for the other three.  grad T from the first moments as Eqs. (49)-(50); div u by
 *          the isotropic central difference with the D3Q19 weights; Q, S, the modified
 *          collision and anti-bounce-back as in two dimensions.
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define O3_FREEZE_FLOW 1u
#define O3_NO_S 2u
#define O3_FREEZE_THERMAL 4u /* test-only: populations g frozen (isothermal flow) */

typedef struct {
  int32_t nx, ny, nz;
  double a, b, R, acentric, G;
  double nu, s_e, s_eps, sigma;
  double lambda, cv, wdot, vs3;
  int32_t thermal_box;
  double T_box;
  uint32_t flags;
} o3_params;

/* D3Q19 velocities and weights */
static const int C19[19][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},   {0, 0, -1},
                               {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1},
                               {-1, 0, 1}, {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
static double w19(int i) {
  int c2 = C19[i][0] * C19[i][0] + C19[i][1] * C19[i][1] + C19[i][2] * C19[i][2];
  return c2 == 0 ? 1.0 / 3.0 : (c2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
}
/* D3Q7 velocities */
static const int C7[7][3] = {{0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
static double w7(const o3_params* p, int i) { return i == 0 ? 1.0 - p->wdot : p->wdot / 6.0; }
static double chat2(const o3_params* p) { return p->wdot / 3.0; }
static int opp7(int i) { return i == 0 ? 0 : (i % 2 ? i + 1 : i - 1); }

/* R3-M: the d'Humieres moment polynomials */
static void build_M19(double M[19][19]) {
  for (int i = 0; i < 19; ++i) {
    double cx = C19[i][0], cy = C19[i][1], cz = C19[i][2];
    double c2 = cx * cx + cy * cy + cz * cz;
    double row[19] = {1.0,
                      19.0 * c2 - 30.0,
                      (21.0 * c2 * c2 - 53.0 * c2 + 24.0) / 2.0,
                      cx,
                      (5.0 * c2 - 9.0) * cx,
                      cy,
                      (5.0 * c2 - 9.0) * cy,
                      cz,
                      (5.0 * c2 - 9.0) * cz,
                      3.0 * cx * cx - c2,
                      (3.0 * c2 - 5.0) * (3.0 * cx * cx - c2),
                      cy * cy - cz * cz,
                      (3.0 * c2 - 5.0) * (cy * cy - cz * cz),
                      cx * cy,
                      cy * cz,
                      cx * cz,
                      (cy * cy - cz * cz) * cx,
                      (cz * cz - cx * cx) * cy,
                      (cx * cx - cy * cy) * cz};
    for (int k = 0; k < 19; ++k) M[k][i] = row[k];
  }
}
/* R3-T: the non-orthogonal D3Q7 matrix */
static void build_M7(double M[7][7]) {
  for (int i = 0; i < 7; ++i) {
    double cx = C7[i][0], cy = C7[i][1], cz = C7[i][2];
    double row[7] = {1.0, cx, cy, cz, cx * cx + cy * cy + cz * cz, cx * cx - cy * cy, cx * cx - cz * cz};
    for (int k = 0; k < 7; ++k) M[k][i] = row[k];
  }
}
static int invert(int n, const double* A, double* Ainv) {
  double aug[19][38];
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < 2 * n; ++c) aug[r][c] = c < n ? A[r * n + c] : (c - n == r ? 1.0 : 0.0);
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (fabs(aug[r][col]) > fabs(aug[piv][col])) piv = r;
    if (fabs(aug[piv][col]) < 1e-300) return -1;
    if (piv != col)
      for (int c = 0; c < 2 * n; ++c) {
        double t = aug[col][c];
        aug[col][c] = aug[piv][c];
        aug[piv][c] = t;
      }
    double d = aug[col][col];
    for (int c = 0; c < 2 * n; ++c) aug[col][c] /= d;
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      double m = aug[r][col];
      for (int c = 0; c < 2 * n; ++c) aug[r][c] -= m * aug[col][c];
    }
  }
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < n; ++c) Ainv[r * n + c] = aug[r][n + c];
  return 0;
}

/* Peng-Robinson EOS (Eq. 10), as in two dimensions */
double o3_eos_Tc(const o3_params* p) { return 0.0778 * p->a / (0.45724 * p->b * p->R); }
static double pr_kappa(const o3_params* p) {
  double w = p->acentric;
  return 0.37464 + 1.54226 * w - 0.26992 * w * w;
}
double o3_eos_p(const o3_params* p, double rho, double T) {
  double s = 1.0 + pr_kappa(p) * (1.0 - sqrt(T / o3_eos_Tc(p)));
  double b = p->b;
  return rho * p->R * T / (1.0 - b * rho) - p->a * s * s * rho * rho / (1.0 + 2.0 * b * rho - b * b * rho * rho);
}
static double eos_dpdT(const o3_params* p, double rho, double T) {
  double Tc = o3_eos_Tc(p), k = pr_kappa(p);
  double s = 1.0 + k * (1.0 - sqrt(T / Tc));
  double dphi = 2.0 * s * k * (-0.5 / sqrt(T * Tc));
  double b = p->b;
  return rho * p->R / (1.0 - b * rho) - p->a * dphi * rho * rho / (1.0 + 2.0 * b * rho - b * b * rho * rho);
}

/* Eq. (3) on D3Q19 */
void o3_feq(double rho, double ux, double uy, double uz, double fe[19]) {
  double uu = ux * ux + uy * uy + uz * uz;
  for (int i = 0; i < 19; ++i) {
    double cu = C19[i][0] * ux + C19[i][1] * uy + C19[i][2] * uz;
    fe[i] = w19(i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
  }
}
/* second-order (Guo) forcing term in velocity space: w_i [3 (c - u) + 9 (c.u) c] . F */
static void guo(double ux, double uy, double uz, double Fx, double Fy, double Fz, double G[19]) {
  for (int i = 0; i < 19; ++i) {
    double cx = C19[i][0], cy = C19[i][1], cz = C19[i][2];
    double cu = cx * ux + cy * uy + cz * uz;
    G[i] = w19(i) * (3.0 * ((cx - ux) * Fx + (cy - uy) * Fy + (cz - uz) * Fz) + 9.0 * cu * (cx * Fx + cy * Fy + cz * Fz));
  }
}

typedef struct {
  o3_params p;
  int nx, ny, nz;
  size_t n;
  double *f, *fn, *fs, *g, *gn, *gs, *T1, *T2;
  double *rho, *T, *jx, *jy, *jz, *psi, *dpdT, *Fx, *Fy, *Fz, *S2, *ux, *uy, *uz, *Q, *Sc;
  double M[19][19], Minv[19][19], M7[7][7], M7inv[7][7];
  double S[19], Lam[7];
  long steps;
  double last_sumQ, last_sumS;
  int err;
} o3_state;

static size_t id3(const o3_state* s, int x, int y, int z) {
  x = ((x % s->nx) + s->nx) % s->nx;
  y = ((y % s->ny) + s->ny) % s->ny;
  z = ((z % s->nz) + s->nz) % s->nz;
  return ((size_t)z * s->ny + y) * s->nx + x;
}

void o3_free(o3_state* s);

o3_state* o3_new(const o3_params* prm) {
  if (prm->nx < 3 || prm->ny < 3 || prm->nz < 3) return NULL;
  o3_state* s = (o3_state*)calloc(1, sizeof(o3_state));
  s->p = *prm;
  s->nx = prm->nx;
  s->ny = prm->ny;
  s->nz = prm->nz;
  s->n = (size_t)prm->nx * prm->ny * prm->nz;
  size_t n = s->n;
  s->f = calloc(19 * n, sizeof(double));
  s->fn = calloc(19 * n, sizeof(double));
  s->fs = calloc(19 * n, sizeof(double));
  s->g = calloc(7 * n, sizeof(double));
  s->gn = calloc(7 * n, sizeof(double));
  s->gs = calloc(7 * n, sizeof(double));
  double** fl[] = {&s->T1, &s->T2, &s->rho, &s->T,  &s->jx, &s->jy, &s->jz, &s->psi, &s->dpdT, &s->Fx,
                   &s->Fy, &s->Fz, &s->S2,  &s->ux, &s->uy, &s->uz, &s->Q,  &s->Sc};
  for (size_t k = 0; k < sizeof(fl) / sizeof(fl[0]); ++k) *fl[k] = calloc(n, sizeof(double));
  build_M19(s->M);
  build_M7(s->M7);
  if (invert(19, &s->M[0][0], &s->Minv[0][0]) || invert(7, &s->M7[0][0], &s->M7inv[0][0])) {
    o3_free(s);
    return NULL;
  }
  double sv = 1.0 / (3.0 * prm->nu + 0.5);
  double Sd[19] = {1, prm->s_e, prm->s_eps, 1, 1, 1, 1, 1, 1, sv, 1, sv, 1, sv, sv, sv, 1, 1, 1};
  memcpy(s->S, Sd, sizeof(Sd));
  double vs1 = 1.0 / (prm->lambda / chat2(prm) + 0.5);
  double L[7] = {1, vs1, vs1, vs1, prm->vs3, prm->vs3, prm->vs3};
  memcpy(s->Lam, L, sizeof(L));
  return s;
}

void o3_free(o3_state* s) {
  if (!s) return;
  double* ptrs[] = {s->f,  s->fn, s->fs, s->g,  s->gn,   s->gs, s->T1, s->T2, s->rho, s->T,  s->jx, s->jy,
                    s->jz, s->psi, s->dpdT, s->Fx, s->Fy, s->Fz, s->S2, s->ux, s->uy,  s->uz, s->Q,  s->Sc};
  for (size_t k = 0; k < sizeof(ptrs) / sizeof(ptrs[0]); ++k) free(ptrs[k]);
  free(s);
}

void o3_init(o3_state* s, const double* rho, const double* ux, const double* uy, const double* uz, const double* T) {
  size_t n = s->n;
  for (size_t k = 0; k < n; ++k) {
    double fe[19];
    o3_feq(rho[k], ux[k], uy[k], uz[k], fe);
    for (int i = 0; i < 19; ++i) s->f[i * n + k] = fe[i];
    for (int i = 0; i < 7; ++i) s->g[i * n + k] = w7(&s->p, i) * T[k];
    s->T1[k] = s->T2[k] = T[k];
  }
  s->steps = 0;
  s->err = 0;
}

/* fields of time t: rho, j, T, psi, dp/dT; forces and velocity */
static int macro(o3_state* s) {
  const o3_params* p = &s->p;
  size_t n = s->n;
  int err = 0;
#pragma omp parallel for reduction(max : err)
  for (long k = 0; k < (long)n; ++k) {
    double r = 0, jx = 0, jy = 0, jz = 0, T = 0;
    for (int i = 0; i < 19; ++i) {
      double fi = s->f[i * n + k];
      r += fi;
      jx += C19[i][0] * fi;
      jy += C19[i][1] * fi;
      jz += C19[i][2] * fi;
    }
    for (int i = 0; i < 7; ++i) T += s->g[i * n + k];
    s->rho[k] = r;
    s->jx[k] = jx;
    s->jy[k] = jy;
    s->jz[k] = jz;
    s->T[k] = T;
    if (!(r > 0.0) || !isfinite(r) || !(T > 0.0) || !isfinite(T)) {
      err = err > 1 ? err : 1;
      continue;
    }
    double arg = 2.0 * (o3_eos_p(p, r, T) - r / 3.0) / p->G;
    if (!(arg >= 0.0)) err = 2;
    s->psi[k] = arg >= 0.0 ? sqrt(arg) : 0.0;
    s->dpdT[k] = eos_dpdT(p, r, T);
  }
  if (err) return err;
  const int freeze = (p->flags & O3_FREEZE_FLOW) != 0;
#pragma omp parallel for collapse(2)
  for (int z = 0; z < s->nz; ++z)
    for (int y = 0; y < s->ny; ++y)
      for (int x = 0; x < s->nx; ++x) {
        size_t k = id3(s, x, y, z);
        double sx = 0, sy = 0, sz = 0;
        if (!freeze)
          for (int i = 1; i < 19; ++i) {
            int c2 = C19[i][0] * C19[i][0] + C19[i][1] * C19[i][1] + C19[i][2] * C19[i][2];
            double wv = c2 == 1 ? 1.0 / 6.0 : 1.0 / 12.0; /* R3-F */
            double pn = s->psi[id3(s, x + C19[i][0], y + C19[i][1], z + C19[i][2])];
            sx += wv * pn * C19[i][0];
            sy += wv * pn * C19[i][1];
            sz += wv * pn * C19[i][2];
          }
        double c = -p->G * s->psi[k];
        s->Fx[k] = c * sx;
        s->Fy[k] = c * sy;
        s->Fz[k] = c * sz;
        s->S2[k] = p->G * p->G * (sx * sx + sy * sy + sz * sz); /* |F_m|^2 / psi^2 */
        s->ux[k] = (s->jx[k] + 0.5 * s->Fx[k]) / s->rho[k];
        s->uy[k] = (s->jy[k] + 0.5 * s->Fy[k]) / s->rho[k];
        s->uz[k] = (s->jz[k] + 0.5 * s->Fz[k]) / s->rho[k];
      }
  return 0;
}

static int step_once(o3_state* s) {
  const o3_params* p = &s->p;
  const size_t n = s->n;
  const int freeze = (p->flags & O3_FREEZE_FLOW) != 0;
  const int noS = (p->flags & O3_NO_S) != 0;
  int e = macro(s);
  if (e) return e;
  const double cs2h = chat2(p);
  /* thermal sources: div u (isotropic, D3Q19 weights), grad T from the D3Q7 first moments */
#pragma omp parallel for collapse(2)
  for (int z = 0; z < s->nz; ++z)
    for (int y = 0; y < s->ny; ++y)
      for (int x = 0; x < s->nx; ++x) {
        size_t k = id3(s, x, y, z);
        double dv = 0.0;
        for (int i = 1; i < 19; ++i) {
          size_t q = id3(s, x + C19[i][0], y + C19[i][1], z + C19[i][2]);
          dv += w19(i) * (C19[i][0] * s->ux[q] + C19[i][1] * s->uy[q] + C19[i][2] * s->uz[q]);
        }
        dv *= 3.0;
        double m[7];
        for (int r = 0; r < 7; ++r) {
          m[r] = 0.0;
          for (int c = 0; c < 7; ++c) m[r] += s->M7[r][c] * s->g[c * n + k];
        }
        double dTx = -s->Lam[1] * m[1] / cs2h, dTy = -s->Lam[2] * m[2] / cs2h, dTz = -s->Lam[3] * m[3] / cs2h;
        double rcv = s->rho[k] * p->cv;
        s->Q[k] = -(rcv * (s->ux[k] * dTx + s->uy[k] * dTy + s->uz[k] * dTz) + s->T[k] * s->dpdT[k] * dv);
        s->Sc[k] = noS ? 0.0 : rcv * 0.5 * (s->T[k] - 2.0 * s->T1[k] + s->T2[k]);
      }
  /* D3Q19 MRT collision with Li's forcing (R3-M, R3-LI) */
  if (!freeze) {
#pragma omp parallel for
    for (long k = 0; k < (long)n; ++k) {
      double fe[19], G[19], m[19], me[19], F[19];
      o3_feq(s->rho[k], s->ux[k], s->uy[k], s->uz[k], fe);
      guo(s->ux[k], s->uy[k], s->uz[k], s->Fx[k], s->Fy[k], s->Fz[k], G);
      for (int r = 0; r < 19; ++r) {
        m[r] = me[r] = F[r] = 0.0;
        for (int c = 0; c < 19; ++c) {
          m[r] += s->M[r][c] * s->f[c * n + k];
          me[r] += s->M[r][c] * fe[c];
          F[r] += s->M[r][c] * G[c];
        }
      }
      F[1] += (19.0 / 2.0) * p->sigma * s->S2[k] / (1.0 / p->s_e - 0.5);
      F[2] += (-11.0 / 4.0) * p->sigma * s->S2[k] / (1.0 / p->s_eps - 0.5);
      double ms[19];
      for (int r = 0; r < 19; ++r) ms[r] = m[r] - s->S[r] * (m[r] - me[r]) + (1.0 - 0.5 * s->S[r]) * F[r];
      for (int r = 0; r < 19; ++r) {
        double v = 0.0;
        for (int c = 0; c < 19; ++c) v += s->Minv[r][c] * ms[c];
        s->fs[r * n + k] = v;
      }
    }
  }
  /* D3Q7 MRT collision (R3-T, Eq. 39) */
#pragma omp parallel for
  for (long k = 0; k < (long)n; ++k) {
    double m[7], d[7];
    double Tk = s->T[k];
    double meq[7] = {Tk, 0, 0, 0, p->wdot * Tk, 0, 0};
    for (int r = 0; r < 7; ++r) {
      m[r] = 0.0;
      for (int c = 0; c < 7; ++c) m[r] += s->M7[r][c] * s->g[c * n + k];
      d[r] = s->Lam[r] * (m[r] - meq[r]);
    }
    for (int i = 0; i < 7; ++i) {
      double coll = 0.0;
      for (int c = 0; c < 7; ++c) coll += s->M7inv[i][c] * d[c];
      s->gs[i * n + k] = s->g[i * n + k] - coll + w7(p, i) * (s->Q[k] + s->Sc[k]);
    }
  }
  /* streaming of f: periodic */
  if (freeze) {
    memcpy(s->fn, s->f, 19 * n * sizeof(double));
  } else {
#pragma omp parallel for collapse(2)
    for (int z = 0; z < s->nz; ++z)
      for (int y = 0; y < s->ny; ++y)
        for (int x = 0; x < s->nx; ++x) {
          size_t k = id3(s, x, y, z);
          for (int i = 0; i < 19; ++i)
            s->fn[i * n + id3(s, x + C19[i][0], y + C19[i][1], z + C19[i][2])] = s->fs[i * n + k];
        }
  }
  /* streaming of g with the modified collision term (Eq. 39), anti-bounce-back at the faces of a
     Dirichlet temperature box */
  if (p->flags & O3_FREEZE_THERMAL) memcpy(s->gn, s->g, 7 * n * sizeof(double));
  else
#pragma omp parallel for collapse(2)
  for (int z = 0; z < s->nz; ++z)
    for (int y = 0; y < s->ny; ++y)
      for (int x = 0; x < s->nx; ++x) {
        size_t k = id3(s, x, y, z);
        double rcv = s->rho[k] * p->cv;
        for (int i = 0; i < 7; ++i) {
          int xu = x - C7[i][0], yu = y - C7[i][1], zu = z - C7[i][2];
          int out = p->thermal_box && (xu < 0 || xu >= s->nx || yu < 0 || yu >= s->ny || zu < 0 || zu >= s->nz);
          double up = out ? -s->gs[opp7(i) * n + k] + 2.0 * w7(p, i) * p->T_box : s->gs[i * n + id3(s, xu, yu, zu)];
          s->gn[i * n + k] = (up + (rcv - 1.0) * s->g[i * n + k]) / rcv;
        }
      }
  double sq = 0.0, ss = 0.0;
  for (size_t k = 0; k < n; ++k) {
    sq += s->Q[k];
    ss += s->Sc[k];
  }
  s->last_sumQ = sq;
  s->last_sumS = ss;
  for (size_t k = 0; k < n; ++k) {
    s->T2[k] = s->T1[k];
    s->T1[k] = s->T[k];
  }
  double* t;
  t = s->f; s->f = s->fn; s->fn = t;
  t = s->g; s->g = s->gn; s->gn = t;
  s->steps += 1;
  return 0;
}

int o3_step(o3_state* s, long nsteps) {
  if (s->err) return s->err;
  for (long k = 0; k < nsteps; ++k) {
    int e = step_once(s);
    if (e) {
      s->err = e;
      return e;
    }
  }
  return 0;
}

int o3_fields(o3_state* s, double* rho, double* ux, double* uy, double* uz, double* T) {
  int e = macro(s);
  if (e) return e;
  size_t b = s->n * sizeof(double);
  memcpy(rho, s->rho, b);
  memcpy(ux, s->ux, b);
  memcpy(uy, s->uy, b);
  memcpy(uz, s->uz, b);
  memcpy(T, s->T, b);
  return 0;
}
void o3_get_state(const o3_state* s, double* f, double* g, double* hist) {
  memcpy(f, s->f, 19 * s->n * sizeof(double));
  memcpy(g, s->g, 7 * s->n * sizeof(double));
  memcpy(hist, s->T1, s->n * sizeof(double));
  memcpy(hist + s->n, s->T2, s->n * sizeof(double));
}
void o3_diagnostics(const o3_state* s, double* mass, double* energy, double* sumQ, double* sumS) {
  double m = 0.0, en = 0.0;
  for (size_t k = 0; k < s->n; ++k) {
    double r = 0, T = 0;
    for (int i = 0; i < 19; ++i) r += s->f[i * s->n + k];
    for (int i = 0; i < 7; ++i) T += s->g[i * s->n + k];
    m += r;
    en += r * s->p.cv * T;
  }
  *mass = m;
  *energy = en;
  *sumQ = s->last_sumQ;
  *sumS = s->last_sumS;
}
void o3_matrices(const o3_state* s, double* M, double* M7) {
  memcpy(M, s->M, sizeof(s->M));
  memcpy(M7, s->M7, sizeof(s->M7));
}
long o3_steps(const o3_state* s) { return s->steps; }
