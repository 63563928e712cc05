/*
 * Plain FP64 CPU oracle for the thermal pseudopotential lattice Boltzmann model of
 * L. Wang, J. Huang, K. He, "A new thermal lattice Boltzmann model for liquid-vapor
 * phase change" (arXiv:2205.00686).
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the cpu_baseline
 * leg of bench.py may load this library.  It shares no code, header, table or constant
 * with the GPU library; it is deliberately written the slow, obvious way:
 *   - explicit 9x9 (D2Q9) and 5x5 (D2Q5) transformation matrices, inverted numerically
 *     by Gauss-Jordan elimination at set-up;
 *   - every macroscopic field of time t is computed over the whole grid into its own
 *     array before any value of time t+1 is written (two full population arrays);
 *   - the steps run in the order in which the paper introduces them.
 *
 * Lattice units dx = dt = 1 throughout.  Arrays are [component][y][x], x fastest.
 *
 * Readings of passages where the paper is silent or garbled (each is listed with its
 * justification in the design notes of the repository):
 *   R-M   Row 3 of the D2Q9 matrix (Eq. 4) is printed with a 1 in column 5; the
 *         Lallemand-Luo matrix the paper cites has -2 there.  With -2 the rows are
 *         orthogonal and M f_eq = m_eq (Eq. 7) holds exactly; with 1 neither holds.
 *   R-BLEND  rho*c_v in Eqs. (21)/(39) is taken at the destination node y = x + c_i and
 *         time t:  g_i(y,t+1) = [g*_i(y-c_i) + (rho(y,t) c_v - 1) g_i(y,t)] / (rho(y,t) c_v).
 *         Summed over the grid this gives sum rho c_v (T^{t+1}-T^t) = sum (Q + S) exactly,
 *         the discrete form of rho c_v dT/dt = div(lambda grad T) + Q (Eq. 20).
 *   R-GRADT  grad T from the non-equilibrium first moments, Eqs. (49)-(50), with the
 *         lattice sound speed of the D2Q5 set (the unhatted c_s there is a misprint).
 *   R-DIVU  div u is not specified; the isotropic central difference
 *         3 sum_i w_i c_i . u(x + c_i) with the D2Q9 weights is used.  At a wall the ghost
 *         velocity is the mirror image -u of the first fluid row (u = 0 on the halfway wall
 *         plane); a zero ghost velocity lets a wall-bounded liquid at c_v = 5 grow a
 *         thermo-acoustic mode until psi becomes undefined.
 *   R-D2T  d^2T/dt^2 in Eq. (24) is not specified; the backward difference
 *         T(t) - 2 T(t-1) + T(t-2) is used, with both history levels set to T(0) at start.
 *   R-WALL Walls are halfway (at y = -1/2 and y = ny - 1/2); the ghost rows y = -1 and
 *         y = ny carry the wetting density of Eq. (54) (first fluid layer = row 0, second
 *         = row 1), the wall temperature, and the mirrored velocity of R-DIVU.
 *   R-DIR  Dirichlet temperature "by halfway bounce-back" is the anti-bounce-back rule
 *         g_i(y,t+1) upstream term = -g*_ibar(y,t) + 2 what_i T_w, blended like any other
 *         upstream population.
 *   R-AVE  rho_ave of the buoyancy force F_b = (rho - rho_ave) g (Section 4.3) is the mean
 *         density over the whole domain at the time level of the step: it is recomputed from the
 *         density field of time t at every step (a fixed-order FP64 sum), so that the buoyancy
 *         adds no net force to the domain also when mass leaves or enters through an open top.
 *         A finite rho_ave given in the parameters is used as a constant instead.
 *   R-Q9   The D2Q9 thermal lattice the paper compares against (Sections 1 and 3.1): the BGK
 *         equation of Eq. (21) with the linear equilibrium what_i T of Eq. (22) on the D2Q9
 *         velocities, what_i = the D2Q9 weights (chat_s^2 = 1/3), G_i and S_i of Eqs. (23)-(24)
 *         with the same weights, lambda = chat_s^2 (tau_g - 1/2) as after Eq. (53), and grad T
 *         from the non-equilibrium first moment as in Eqs. (49)-(50):
 *         chat_s^2 dT/dx = -(1/tau_g) sum_i c_ix g_i (the equilibrium part of that sum is 0).
 *   R-OPEN The open top boundary the paper takes from Lou et al. (Section 4.2, 4.3) is not written
 *         out.  Reading: the convective outflow condition for the populations that enter the top
 *         row from outside (c_y = -1),
 *           f_i(x, N, t+1) = [f_i(x, N, t) + U f_i(x, N-1, t+1)] / (1 + U),
 *         with U = the local normal velocity j_y / rho of the top node at time t, clipped to
 *         [0, 1]; populations leaving through the top are dropped; the ghost row above carries the
 *         pseudopotential and the velocity of the top row (zero gradient); the temperature keeps
 *         the Dirichlet value T_top (R-DIR).  The bottom stays a wall (R-WALL).
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_FREEZE_FLOW 1u /* test-only: populations f frozen, u = j/rho, no force */
#define ORC_NO_S 2u        /* test-only: correction term S_i of Eq. (24) switched off */
#define ORC_FREEZE_THERMAL 4u /* test-only: populations g frozen (isothermal flow) */
#define ORC_BGK 8u            /* D2Q5 with the BGK collision of Eq. (21) instead of Eq. (39) */

/* Parameters of the problem statement (Sections 2-4 of the paper). */
typedef struct {
  int32_t nx, ny;
  double a, b, R, acentric, G;  /* Peng-Robinson EOS (Eq. 10) and interaction strength (Eq. 9) */
  double nu, s_e, s_eps, s_q, sigma; /* D2Q9 MRT rates (Eq. 5) and Li's sigma (Eq. 8) */
  double lambda, cv, wdot, vs3, vs4; /* conductivity, c_v, D2Q5 weight parameter, varsigma_3,4 */
  double gx, gy, rho_ave;       /* body-force acceleration and rho_ave of F_b (NaN: current mean, R-AVE) */
  int32_t y_walls;              /* 0: periodic in y; 1: no-slip walls at y=-1/2 and y=ny-1/2 */
  int32_t thermal_box;          /* 1: Dirichlet T = T_box on all four edges (flow periodic) */
  double T_box, T_top, T_bot, hot_dT, hot_x0, hot_sigma;
  double theta_bot_deg, theta_top_deg;
  uint32_t flags;
  int32_t thermal_q;            /* thermal lattice: 5 (D2Q5, Eqs. 26 and 39; 0 means 5) or 9 (R-Q9) */
  int32_t open_top;             /* with y_walls: the top is the open boundary of R-OPEN */
} orc_params;

/* ---------------------------------------------------------------- lattices (Eqs. 2, 3, 26) */
static const int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double W9[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                             1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
static const int HX[5] = {0, 1, 0, -1, 0};
static const int HY[5] = {0, 0, 1, 0, -1};
static const double CS2 = 1.0 / 3.0; /* c_s^2 of the D2Q9 set, c = 1 */

static int opposite9(int i) {
  for (int k = 0; k < 9; ++k)
    if (CX[k] == -CX[i] && CY[k] == -CY[i]) return k;
  return -1;
}
static int opposite5(int i) {
  for (int k = 0; k < 5; ++k)
    if (HX[k] == -HX[i] && HY[k] == -HY[i]) return k;
  return -1;
}

/* D2Q5 weights: what_0 = 1 - wdot, what_{1..4} = wdot/4, chat_s^2 = wdot/2 (Eq. 26). */
static double what5(const orc_params* p, int i) { return i == 0 ? 1.0 - p->wdot : p->wdot / 4.0; }
static double chat_s2_5(const orc_params* p) { return p->wdot / 2.0; }

/* The thermal lattice in use: number of velocities, velocities, weights, chat_s^2 (R-Q9). */
static int qg(const orc_params* p) { return p->thermal_q == 9 ? 9 : 5; }
static int gcx(const orc_params* p, int i) { return qg(p) == 9 ? CX[i] : HX[i]; }
static int gcy(const orc_params* p, int i) { return qg(p) == 9 ? CY[i] : HY[i]; }
static double gw(const orc_params* p, int i) { return qg(p) == 9 ? W9[i] : what5(p, i); }
static double chat_s2(const orc_params* p) { return qg(p) == 9 ? CS2 : chat_s2_5(p); }
static int gopp(const orc_params* p, int i) { return qg(p) == 9 ? opposite9(i) : opposite5(i); }
/* BGK collision (Eq. 21) for D2Q9, or for D2Q5 when asked for */
static int bgk(const orc_params* p) { return qg(p) == 9 || (p->flags & ORC_BGK) != 0; }

/* ------------------------------------------------------------ transformation matrices */
/* Eq. (4), with row 3 read as the Lallemand-Luo epsilon row (reading R-M). */
static void build_M(double M[9][9]) {
  static const double rows[9][9] = {
      {1, 1, 1, 1, 1, 1, 1, 1, 1},
      {-4, -1, -1, -1, -1, 2, 2, 2, 2},
      {4, -2, -2, -2, -2, 1, 1, 1, 1},
      {0, 1, 0, -1, 0, 1, -1, -1, 1},
      {0, -2, 0, 2, 0, 1, -1, -1, 1},
      {0, 0, 1, 0, -1, 1, 1, -1, -1},
      {0, 0, -2, 0, 2, 1, 1, -1, -1},
      {0, 1, -1, 1, -1, 0, 0, 0, 0},
      {0, 0, 0, 0, 0, 1, -1, 1, -1}};
  memcpy(M, rows, sizeof(rows));
}
/* Eq. (40): non-orthogonal D2Q5 matrix. */
static void build_Mhat(double Mh[5][5]) {
  static const double rows[5][5] = {
      {1, 1, 1, 1, 1}, {0, 1, 0, -1, 0}, {0, 0, 1, 0, -1}, {0, 1, 1, 1, 1}, {0, 1, -1, 1, -1}};
  memcpy(Mh, rows, sizeof(rows));
}
/* Gauss-Jordan inverse with partial pivoting of an n x n row-major matrix. */
static int invert(int n, const double* A, double* Ainv) {
  double aug[9][18];
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < 2 * n; ++c)
      aug[r][c] = c < n ? A[r * n + c] : (c - n == r ? 1.0 : 0.0);
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

/* ------------------------------------------------------------ thermodynamics (Eq. 10) */
/* a = 0.45724 R^2 Tc^2 / pc and b = 0.0778 R Tc / pc give Tc = 0.0778 a / (0.45724 b R). */
double orc_eos_Tc(const orc_params* p) { return 0.0778 * p->a / (0.45724 * p->b * p->R); }
static double pr_kappa(const orc_params* p) {
  double w = p->acentric;
  return 0.37464 + 1.54226 * w - 0.26992 * w * w;
}
double orc_eos_p(const orc_params* p, double rho, double T) {
  double Tc = orc_eos_Tc(p);
  double s = 1.0 + pr_kappa(p) * (1.0 - sqrt(T / Tc));
  double phi = s * s;
  double b = p->b;
  return rho * p->R * T / (1.0 - b * rho) - p->a * phi * rho * rho / (1.0 + 2.0 * b * rho - b * b * rho * rho);
}
/* (d p_EOS / dT) at constant rho: only the two T-dependent factors RT and phi(T) vary. */
double orc_eos_dpdT(const orc_params* p, double rho, double T) {
  double Tc = orc_eos_Tc(p);
  double k = pr_kappa(p);
  double s = 1.0 + k * (1.0 - sqrt(T / Tc));
  double dphi = 2.0 * s * k * (-0.5 / sqrt(T * Tc)); /* d/dT of s^2 */
  double b = p->b;
  return rho * p->R / (1.0 - b * rho) - p->a * dphi * rho * rho / (1.0 + 2.0 * b * rho - b * b * rho * rho);
}
/* psi = sqrt(2 (p_EOS - rho c_s^2) / (G dx^2)) (text after Eq. 9). Returns -1 if undefined. */
double orc_psi(const orc_params* p, double rho, double T) {
  double arg = 2.0 * (orc_eos_p(p, rho, T) - rho * CS2) / p->G;
  if (!(arg >= 0.0)) return -1.0;
  return sqrt(arg);
}

/* Maxwell equal-area construction for the EOS at temperature T:
 *   p(rho_g) = p(rho_l) = p_sat  and  integral_{v_l}^{v_g} (p - p_sat) dv = 0, v = 1/rho,
 * i.e. integral_{rho_g}^{rho_l} (p(rho) - p_sat) / rho^2 drho = 0.
 * Spinodal points are bracketed on a fine density scan, roots and p_sat by bisection,
 * the integral by composite Simpson on 20000 panels.  Returns 0 on success. */
static double simpson_area(const orc_params* p, double T, double psat, double r0, double r1) {
  const int N = 20000;
  double h = (r1 - r0) / N, s = 0.0;
  for (int k = 0; k <= N; ++k) {
    double r = r0 + k * h;
    double v = (orc_eos_p(p, r, T) - psat) / (r * r);
    s += (k == 0 || k == N) ? v : (k % 2 ? 4.0 * v : 2.0 * v);
  }
  return s * h / 3.0;
}
static double root_increasing(const orc_params* p, double T, double target, double lo, double hi) {
  for (int it = 0; it < 200; ++it) {
    double mid = 0.5 * (lo + hi);
    if (orc_eos_p(p, mid, T) < target) lo = mid; else hi = mid;
  }
  return 0.5 * (lo + hi);
}
int orc_maxwell(const orc_params* p, double T, double* rho_l, double* rho_g, double* p_sat) {
  double rmax = (1.0 / p->b) * (1.0 - 1e-9);
  /* scan for the local maximum (end of the vapour branch) and local minimum of p(rho) */
  const int NS = 200000;
  double h = rmax / NS;
  double rs_max = -1, rs_min = -1;
  double prev = orc_eos_p(p, h, T);
  int rising = 1;
  for (int k = 2; k < NS; ++k) {
    double cur = orc_eos_p(p, k * h, T);
    if (rising && cur < prev) { rs_max = (k - 1) * h; rising = 0; }
    else if (!rising && cur > prev) { rs_min = (k - 1) * h; break; }
    prev = cur;
  }
  if (rs_max < 0 || rs_min < 0) return -1; /* supercritical: no coexistence */
  double p_hi = orc_eos_p(p, rs_max, T);
  double p_lo = orc_eos_p(p, rs_min, T);
  if (p_lo < 1e-14) p_lo = 1e-14;
  double lo = p_lo, hi = p_hi, rl = 0, rg = 0;
  for (int it = 0; it < 200; ++it) {
    double ps = 0.5 * (lo + hi);
    rg = root_increasing(p, T, ps, 1e-12, rs_max);
    rl = root_increasing(p, T, ps, rs_min, rmax);
    double A = simpson_area(p, T, ps, rg, rl);
    if (A > 0) lo = ps; else hi = ps; /* A decreases as p_sat rises */
  }
  *p_sat = 0.5 * (lo + hi);
  *rho_g = root_increasing(p, T, *p_sat, 1e-12, rs_max);
  *rho_l = root_increasing(p, T, *p_sat, rs_min, rmax);
  return 0;
}

/* -------------------------------------------------------------- equilibria and forcing */
/* Eq. (3) */
void orc_feq(double rho, double ux, double uy, double feq[9]) {
  double uu = ux * ux + uy * uy;
  for (int i = 0; i < 9; ++i) {
    double cu = CX[i] * ux + CY[i] * uy;
    feq[i] = W9[i] * rho * (1.0 + cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
  }
}
/* Eq. (7) */
void orc_meq(double rho, double ux, double uy, double meq[9]) {
  double uu = ux * ux + uy * uy;
  double v[9] = {1.0, -2.0 + 3.0 * uu, 1.0 - 3.0 * uu, ux, -ux, uy, -uy, ux * ux - uy * uy, ux * uy};
  for (int k = 0; k < 9; ++k) meq[k] = rho * v[k];
}
/* Eq. (8): Li et al.'s forcing term in moment space. */
void orc_force_moments(double ux, double uy, double Fnx, double Fny, double Fmx, double Fmy,
                       double psi, double sigma, double s_e, double s_eps, double F[9]) {
  double uF = ux * Fnx + uy * Fny;
  double Fm2 = Fmx * Fmx + Fmy * Fmy;
  double corr_e = sigma * Fm2 / (psi * psi * (1.0 / s_e - 0.5));
  double corr_eps = sigma * Fm2 / (psi * psi * (1.0 / s_eps - 0.5));
  F[0] = 0.0;
  F[1] = 6.0 * uF + corr_e;
  F[2] = -6.0 * uF - corr_eps;
  F[3] = Fnx;
  F[4] = -Fnx;
  F[5] = Fny;
  F[6] = -Fny;
  F[7] = 2.0 * (ux * Fnx - uy * Fny);
  F[8] = ux * Fny + uy * Fnx;
}

/* ---------------------------------------------------------------------------- state */
typedef struct orc_state {
  orc_params p;
  int nx, ny;
  size_t n;
  double *f, *fn, *g, *gn, *T1, *T2;
  /* per-step fields of time t */
  double *rho, *T, *jx, *jy, *psi, *dpdT, *Fmx, *Fmy, *Fnx, *Fny, *ux, *uy, *divu, *Q, *Sc;
  double *fs, *gs; /* post-collision populations */
  double *ghost_rho_b, *ghost_rho_t, *ghost_psi_b, *ghost_psi_t;
  double M[9][9], Minv[9][9], Mh[5][5], Mhinv[5][5];
  double Sdiag[9], Lam[5];
  double rho_ave;
  long steps;
  double last_sumQ, last_sumS;
  int err; /* 0 ok; 1 rho<=0 or non-finite; 2 psi undefined */
} orc_state;

static size_t idx(const orc_state* s, int x, int y) { return (size_t)y * s->nx + x; }
static int wrap(int v, int n) { return ((v % n) + n) % n; }

/* wall temperature seen by the link crossing the bottom (side<0) or top (side>0) wall at column x */
static double wall_T(const orc_state* s, int side, int x) {
  const orc_params* p = &s->p;
  if (p->thermal_box) return p->T_box;
  if (side < 0) {
    double d = x - p->hot_x0;
    double bump = p->hot_sigma > 0 ? p->hot_dT * exp(-d * d / (2.0 * p->hot_sigma * p->hot_sigma)) : 0.0;
    return p->T_bot + bump;
  }
  return p->T_top;
}

void orc_free(orc_state* s);

orc_state* orc_new(const orc_params* prm) {
  if (prm->nx < 3 || prm->ny < 3) return NULL;
  if (prm->open_top && !prm->y_walls) return NULL;
  if (prm->thermal_q != 0 && prm->thermal_q != 5 && prm->thermal_q != 9) return NULL;
  orc_state* s = (orc_state*)calloc(1, sizeof(orc_state));
  s->p = *prm;
  s->nx = prm->nx;
  s->ny = prm->ny;
  s->n = (size_t)prm->nx * prm->ny;
  size_t n = s->n;
  s->f = calloc(9 * n, sizeof(double));
  s->fn = calloc(9 * n, sizeof(double));
  s->fs = calloc(9 * n, sizeof(double));
  s->g = calloc(9 * n, sizeof(double)); /* room for either thermal lattice */
  s->gn = calloc(9 * n, sizeof(double));
  s->gs = calloc(9 * n, sizeof(double));
  double** fields[] = {&s->T1, &s->T2, &s->rho, &s->T, &s->jx, &s->jy, &s->psi, &s->dpdT, &s->Fmx,
                       &s->Fmy, &s->Fnx, &s->Fny, &s->ux, &s->uy, &s->divu, &s->Q, &s->Sc};
  for (size_t k = 0; k < sizeof(fields) / sizeof(fields[0]); ++k) *fields[k] = calloc(n, sizeof(double));
  s->ghost_rho_b = calloc(s->nx, sizeof(double));
  s->ghost_rho_t = calloc(s->nx, sizeof(double));
  s->ghost_psi_b = calloc(s->nx, sizeof(double));
  s->ghost_psi_t = calloc(s->nx, sizeof(double));
  build_M(s->M);
  build_Mhat(s->Mh);
  if (invert(9, &s->M[0][0], &s->Minv[0][0]) || invert(5, &s->Mh[0][0], &s->Mhinv[0][0])) {
    orc_free(s);
    return NULL;
  }
  /* S = diag(s0, s_e, s_eps, s_j, s_q, s_j, s_q, s_p, s_p); the rates of conserved moments
     (s0, s_j) and every rate not tied to a physical parameter are 1 (Section 4). */
  double sp = 1.0 / (3.0 * prm->nu + 0.5); /* nu = c_s^2 (1/s_p - 1/2) */
  double Sd[9] = {1.0, prm->s_e, prm->s_eps, 1.0, prm->s_q, 1.0, prm->s_q, sp, sp};
  memcpy(s->Sdiag, Sd, sizeof(Sd));
  /* lambda = (1/varsigma_1 - 1/2) chat_s^2 (Eq. 53 and the relation after it) */
  double vs1 = 1.0 / (prm->lambda / chat_s2(prm) + 0.5);
  double L[5] = {1.0, vs1, vs1, prm->vs3, prm->vs4};
  memcpy(s->Lam, L, sizeof(L));
  return s;
}

void orc_free(orc_state* s) {
  if (!s) return;
  double* ptrs[] = {s->f, s->fn, s->fs, s->g, s->gn, s->gs, s->T1, s->T2, s->rho, s->T, s->jx, s->jy,
                    s->psi, s->dpdT, s->Fmx, s->Fmy, s->Fnx, s->Fny, s->ux, s->uy, s->divu, s->Q, s->Sc,
                    s->ghost_rho_b, s->ghost_rho_t, s->ghost_psi_b, s->ghost_psi_t};
  for (size_t k = 0; k < sizeof(ptrs) / sizeof(ptrs[0]); ++k) free(ptrs[k]);
  free(s);
}

/* Initial state: f = f_eq(rho, u) (Eq. 3), g = what_i T (Eq. 22), both history levels = T. */
void orc_init(orc_state* s, const double* rho, const double* ux, const double* uy, const double* T) {
  size_t n = s->n;
  double sum = 0.0;
  for (size_t k = 0; k < n; ++k) {
    double fe[9];
    orc_feq(rho[k], ux[k], uy[k], fe);
    for (int i = 0; i < 9; ++i) s->f[i * n + k] = fe[i];
    for (int i = 0; i < qg(&s->p); ++i) s->g[i * n + k] = gw(&s->p, i) * T[k];
    s->T1[k] = T[k];
    s->T2[k] = T[k];
    sum += rho[k];
  }
  s->rho_ave = isnan(s->p.rho_ave) ? sum / (double)n : s->p.rho_ave;
  s->steps = 0;
  s->err = 0;
}

/* psi at (x, y) including the wall ghost rows */
static double psi_at(const orc_state* s, int x, int y) {
  x = wrap(x, s->nx);
  if (s->p.y_walls) {
    if (y == -1) return s->ghost_psi_b[x];
    if (y == s->ny) return s->ghost_psi_t[x];
  } else {
    y = wrap(y, s->ny);
  }
  return s->psi[idx(s, x, y)];
}
/* velocity at (x, y); a ghost row carries the mirror image -u of the adjacent fluid row, so
   that u vanishes on the halfway wall plane (no-slip) */
static void u_at(const orc_state* s, int x, int y, double* ux, double* uy) {
  x = wrap(x, s->nx);
  if (s->p.y_walls) {
    if (y < 0 || y >= s->ny) {
      int yf = y < 0 ? 0 : s->ny - 1;
      double sign = (y >= s->ny && s->p.open_top) ? 1.0 : -1.0; /* R-OPEN above the top, R-DIVU at walls */
      *ux = sign * s->ux[idx(s, x, yf)];
      *uy = sign * s->uy[idx(s, x, yf)];
      return;
    }
  } else {
    y = wrap(y, s->ny);
  }
  *ux = s->ux[idx(s, x, y)];
  *uy = s->uy[idx(s, x, y)];
}

/* Macroscopic fields of time t: rho, j, T (Eqs. 11, 25); p, psi, dp/dT (Eq. 10, text after
 * Eq. 9); ghost rows (Eq. 54); F_m (Eq. 9), F_b, F_n, u (Eq. 11). Returns 0 or an error code. */
static int compute_macro(orc_state* s) {
  const orc_params* p = &s->p;
  const int nx = s->nx, ny = s->ny;
  const size_t n = s->n;
  int err = 0;
#pragma omp parallel for reduction(max : err)
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      size_t k = idx(s, x, y);
      double r = 0, jx = 0, jy = 0, T = 0;
      for (int i = 0; i < 9; ++i) {
        double fi = s->f[i * n + k];
        r += fi;
        jx += CX[i] * fi;
        jy += CY[i] * fi;
      }
      for (int i = 0; i < qg(p); ++i) T += s->g[i * n + k];
      s->rho[k] = r;
      s->jx[k] = jx;
      s->jy[k] = jy;
      s->T[k] = T;
      if (!(r > 0.0) || !isfinite(r) || !isfinite(T) || !(T > 0.0)) { err = err > 1 ? err : 1; continue; }
      double ps = orc_psi(p, r, T);
      if (ps < 0) err = 2;
      s->psi[k] = ps;
      s->dpdT[k] = orc_eos_dpdT(p, r, T);
    }
  if (err) return err;
  /* rho_ave of the buoyancy force: the mean density of the domain at time t (R-AVE), summed
     row by row in a fixed order */
  if (isnan(p->rho_ave)) {
    double total = 0.0;
    for (int y = 0; y < ny; ++y) {
      double row = 0.0;
      for (int x = 0; x < nx; ++x) row += s->rho[idx(s, x, y)];
      total += row;
    }
    s->rho_ave = total / (double)n;
  }
  if (p->y_walls) {
    /* Eq. (54): rho_ghost(x) = rho(x, 2nd layer) + tan(pi/2 - theta) |rho(x+1, 1st) - rho(x-1, 1st)| */
    double tb = tan(M_PI / 2.0 - p->theta_bot_deg * M_PI / 180.0);
    double tt = tan(M_PI / 2.0 - p->theta_top_deg * M_PI / 180.0);
    for (int x = 0; x < nx; ++x) {
      double rb = s->rho[idx(s, x, 1)] +
                  tb * fabs(s->rho[idx(s, wrap(x + 1, nx), 0)] - s->rho[idx(s, wrap(x - 1, nx), 0)]);
      double rt = s->rho[idx(s, x, ny - 2)] +
                  tt * fabs(s->rho[idx(s, wrap(x + 1, nx), ny - 1)] - s->rho[idx(s, wrap(x - 1, nx), ny - 1)]);
      s->ghost_rho_b[x] = rb;
      s->ghost_rho_t[x] = rt;
      s->ghost_psi_b[x] = orc_psi(p, rb, wall_T(s, -1, x));
      s->ghost_psi_t[x] = orc_psi(p, rt, wall_T(s, +1, x));
      if (p->open_top) { /* R-OPEN: zero gradient above the open top */
        s->ghost_rho_t[x] = s->rho[idx(s, x, ny - 1)];
        s->ghost_psi_t[x] = s->psi[idx(s, x, ny - 1)];
      }
      if (s->ghost_psi_b[x] < 0 || s->ghost_psi_t[x] < 0) return 2;
    }
  }
  const int freeze = (p->flags & ORC_FREEZE_FLOW) != 0;
#pragma omp parallel for
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      size_t k = idx(s, x, y);
      double fmx = 0, fmy = 0;
      if (!freeze) {
        /* Eq. (9): F_m = -G psi(x) sum_i varpi(|c_i|^2) psi(x + c_i) c_i, varpi(1)=1/3, varpi(2)=1/12 */
        double sx = 0, sy = 0;
        for (int i = 1; i < 9; ++i) {
          double wv = (CX[i] * CX[i] + CY[i] * CY[i]) == 1 ? 1.0 / 3.0 : 1.0 / 12.0;
          double pn = psi_at(s, x + CX[i], y + CY[i]);
          sx += wv * pn * CX[i];
          sy += wv * pn * CY[i];
        }
        fmx = -p->G * s->psi[k] * sx;
        fmy = -p->G * s->psi[k] * sy;
      }
      s->Fmx[k] = fmx;
      s->Fmy[k] = fmy;
      /* F_b = (rho - rho_ave) g (Section 4.3) ; F_n = F_m + F_b (text after Eq. 8) */
      double fbx = freeze ? 0.0 : (s->rho[k] - s->rho_ave) * p->gx;
      double fby = freeze ? 0.0 : (s->rho[k] - s->rho_ave) * p->gy;
      s->Fnx[k] = fmx + fbx;
      s->Fny[k] = fmy + fby;
      /* Eq. (11): rho u = sum_i c_i f_i + (dt/2) F_n */
      s->ux[k] = (s->jx[k] + 0.5 * s->Fnx[k]) / s->rho[k];
      s->uy[k] = (s->jy[k] + 0.5 * s->Fny[k]) / s->rho[k];
    }
  return 0;
}

/* One time step.  Returns 0, or an error code (state then left unchanged). */
static int step_once(orc_state* s) {
  const orc_params* p = &s->p;
  const int nx = s->nx, ny = s->ny;
  const size_t n = s->n;
  const int freeze = (p->flags & ORC_FREEZE_FLOW) != 0;
  const int noS = (p->flags & ORC_NO_S) != 0;
  int e = compute_macro(s);
  if (e) return e;

  /* Thermal source terms (Eqs. 20, 23, 24, 49, 50). */
  const double cs2h = chat_s2(p);
#pragma omp parallel for
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      size_t k = idx(s, x, y);
      /* div u by the isotropic central difference (reading R-DIVU) */
      double dv = 0.0;
      for (int i = 1; i < 9; ++i) {
        double ux, uy;
        u_at(s, x + CX[i], y + CY[i], &ux, &uy);
        dv += W9[i] * (CX[i] * ux + CY[i] * uy);
      }
      dv *= 1.0 / CS2;
      s->divu[k] = dv;
      /* grad T from the non-equilibrium moments m_1, m_2 (Eqs. 49, 50); m_eq_1 = m_eq_2 = 0 (Eq. 47).
         D2Q9 (R-Q9): the first moment sum_i c_i g_i with the single rate 1/tau_g. */
      double dTx, dTy;
      if (qg(p) == 9) {
        double mx = 0.0, my = 0.0;
        for (int i = 0; i < 9; ++i) {
          mx += CX[i] * s->g[i * n + k];
          my += CY[i] * s->g[i * n + k];
        }
        dTx = -s->Lam[1] * mx / cs2h;
        dTy = -s->Lam[1] * my / cs2h;
      } else {
        double mh[5];
        for (int r = 0; r < 5; ++r) {
          mh[r] = 0.0;
          for (int c = 0; c < 5; ++c) mh[r] += s->Mh[r][c] * s->g[c * n + k];
        }
        dTx = -s->Lam[1] * mh[1] / cs2h;
        dTy = -s->Lam[2] * mh[2] / cs2h;
      }
      double rcv = s->rho[k] * p->cv;
      /* Q = -[rho c_v u . grad T + T (dp/dT)_rho div u] (Eq. 20) */
      s->Q[k] = -(rcv * (s->ux[k] * dTx + s->uy[k] * dTy) + s->T[k] * s->dpdT[k] * dv);
      /* sum_i S_i = rho c_v (dt/2) d^2T/dt^2 (Eq. 24), backward difference (reading R-D2T) */
      s->Sc[k] = noS ? 0.0 : rcv * 0.5 * (s->T[k] - 2.0 * s->T1[k] + s->T2[k]);
    }

  /* D2Q9 MRT collision with Li's forcing (Eqs. 5, 7, 8) */
  if (!freeze) {
#pragma omp parallel for
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        size_t k = idx(s, x, y);
        double m[9], meq[9], F[9], ms[9];
        for (int r = 0; r < 9; ++r) {
          m[r] = 0.0;
          for (int c = 0; c < 9; ++c) m[r] += s->M[r][c] * s->f[c * n + k];
        }
        orc_meq(s->rho[k], s->ux[k], s->uy[k], meq);
        orc_force_moments(s->ux[k], s->uy[k], s->Fnx[k], s->Fny[k], s->Fmx[k], s->Fmy[k], s->psi[k],
                          p->sigma, p->s_e, p->s_eps, F);
        for (int r = 0; r < 9; ++r)
          ms[r] = m[r] - s->Sdiag[r] * (m[r] - meq[r]) + (1.0 - 0.5 * s->Sdiag[r]) * F[r];
        for (int r = 0; r < 9; ++r) {
          double v = 0.0;
          for (int c = 0; c < 9; ++c) v += s->Minv[r][c] * ms[c];
          s->fs[r * n + k] = v;
        }
      }
  }

  /* BGK collision (Eq. 21): g* = g - (g - what T) / tau_g + G + S, for the D2Q9 thermal
     lattice (R-Q9) or the BGK variant of the D2Q5 model */
  if (bgk(p)) {
    const double itau = s->Lam[1];
#pragma omp parallel for
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        size_t k = idx(s, x, y);
        double Tk = s->T[k];
        for (int i = 0; i < qg(p); ++i) {
          double gi = s->g[i * n + k];
          double geq = gw(p, i) * Tk;                          /* Eq. (22) */
          double Gi = gw(p, i) * s->Q[k];                      /* Eq. (23) */
          double Si = gw(p, i) * s->Sc[k];                     /* Eq. (24) */
          s->gs[i * n + k] = gi - itau * (gi - geq) + Gi + Si;
        }
      }
  } else
  /* D2Q5 MRT collision (Eq. 39): g* = g - Mh^-1 Lambda (Mh g - m_eq) + G + S */
#pragma omp parallel for
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      size_t k = idx(s, x, y);
      double mh[5], d[5];
      double Tk = s->T[k];
      double mheq[5] = {Tk, 0.0, 0.0, p->wdot * Tk, 0.0}; /* Eq. (47) */
      for (int r = 0; r < 5; ++r) {
        mh[r] = 0.0;
        for (int c = 0; c < 5; ++c) mh[r] += s->Mh[r][c] * s->g[c * n + k];
        d[r] = s->Lam[r] * (mh[r] - mheq[r]);
      }
      for (int i = 0; i < 5; ++i) {
        double coll = 0.0;
        for (int c = 0; c < 5; ++c) coll += s->Mhinv[i][c] * d[c];
        double Gi = what5(p, i) * s->Q[k];  /* Eq. (23) */
        double Si = what5(p, i) * s->Sc[k]; /* Eq. (24) */
        s->gs[i * n + k] = s->g[i * n + k] - coll + Gi + Si;
      }
    }

  /* Streaming of f (Eq. 6) with periodic wrap or halfway bounce-back at the y walls. */
  if (freeze) {
    memcpy(s->fn, s->f, 9 * n * sizeof(double));
  } else {
#pragma omp parallel for
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        size_t k = idx(s, x, y);
        for (int i = 0; i < 9; ++i) {
          int xd = x + CX[i], yd = y + CY[i];
          if (p->y_walls && yd >= ny && p->open_top) continue; /* leaves through the open top */
          if (p->y_walls && (yd < 0 || yd >= ny)) {
            s->fn[opposite9(i) * n + k] = s->fs[i * n + k];
          } else {
            s->fn[i * n + idx(s, wrap(xd, nx), wrap(yd, ny))] = s->fs[i * n + k];
          }
        }
      }
    if (p->y_walls && p->open_top) {
      /* R-OPEN: the populations entering the top row from outside */
      for (int x = 0; x < nx; ++x) {
        size_t k = idx(s, x, ny - 1), kb = idx(s, x, ny - 2);
        double r = 0.0, jy = 0.0;
        for (int i = 0; i < 9; ++i) {
          r += s->f[i * n + k];
          jy += CY[i] * s->f[i * n + k];
        }
        double U = jy / r;
        U = U < 0.0 ? 0.0 : (U > 1.0 ? 1.0 : U);
        for (int i = 0; i < 9; ++i)
          if (CY[i] == -1) s->fn[i * n + k] = (s->f[i * n + k] + U * s->fn[i * n + kb]) / (1.0 + U);
      }
    }
  }

  /* Streaming of g with the modified collision term (Eq. 39, reading R-BLEND), the
     upstream population replaced by anti-bounce-back at Dirichlet edges (reading R-DIR). */
  if (p->flags & ORC_FREEZE_THERMAL) memcpy(s->gn, s->g, 9 * n * sizeof(double));
  else
#pragma omp parallel for
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      size_t k = idx(s, x, y);
      double rcv = s->rho[k] * p->cv;
      for (int i = 0; i < qg(p); ++i) {
        int xu = x - gcx(p, i), yu = y - gcy(p, i);
        int outside_y = (p->y_walls || p->thermal_box) && (yu < 0 || yu >= ny);
        int outside_x = p->thermal_box && (xu < 0 || xu >= nx);
        double up;
        if (outside_x || outside_y) {
          double Tw = p->thermal_box ? p->T_box : wall_T(s, yu < 0 ? -1 : +1, x);
          up = -s->gs[gopp(p, i) * n + k] + 2.0 * gw(p, i) * Tw;
        } else {
          up = s->gs[i * n + idx(s, wrap(xu, nx), wrap(yu, ny))];
        }
        s->gn[i * n + k] = (up + (rcv - 1.0) * s->g[i * n + k]) / rcv;
      }
    }

  double sq = 0.0, ss = 0.0;
  for (int y = 0; y < ny; ++y) {
    double rq = 0.0, rs = 0.0;
    for (int x = 0; x < nx; ++x) {
      rq += s->Q[idx(s, x, y)];
      rs += s->Sc[idx(s, x, y)];
    }
    sq += rq;
    ss += rs;
  }
  s->last_sumQ = sq;
  s->last_sumS = ss;

  /* history of T for the next step's d^2T/dt^2 */
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

int orc_step(orc_state* s, long nsteps) {
  if (s->err) return s->err;
  for (long k = 0; k < nsteps; ++k) {
    int e = step_once(s);
    if (e) { s->err = e; return e; }
  }
  return 0;
}

/* rho, u (Eq. 11 with the force of time t), T (Eq. 25) of the current state. */
int orc_fields(orc_state* s, double* rho, double* ux, double* uy, double* T) {
  int e = compute_macro(s);
  if (e) return e;
  memcpy(rho, s->rho, s->n * sizeof(double));
  memcpy(ux, s->ux, s->n * sizeof(double));
  memcpy(uy, s->uy, s->n * sizeof(double));
  memcpy(T, s->T, s->n * sizeof(double));
  return 0;
}

/* Raw state: f[9][ny][nx], g[Q][ny][nx] (Q = 5 or 9), history[2][ny][nx] (T(t-1), T(t-2)). */
void orc_get_state(const orc_state* s, double* f, double* g, double* hist) {
  memcpy(f, s->f, 9 * s->n * sizeof(double));
  memcpy(g, s->g, qg(&s->p) * s->n * sizeof(double));
  memcpy(hist, s->T1, s->n * sizeof(double));
  memcpy(hist + s->n, s->T2, s->n * sizeof(double));
}
void orc_set_state(orc_state* s, const double* f, const double* g, const double* hist) {
  memcpy(s->f, f, 9 * s->n * sizeof(double));
  memcpy(s->g, g, qg(&s->p) * s->n * sizeof(double));
  memcpy(s->T1, hist, s->n * sizeof(double));
  memcpy(s->T2, hist + s->n, s->n * sizeof(double));
  s->err = 0;
}

/* mass = sum rho, energy = sum rho c_v T of the current state; sums of Q and S of the last step. */
void orc_diagnostics(const orc_state* s, double* mass, double* energy, double* sumQ, double* sumS) {
  double m = 0.0, en = 0.0;
  for (int y = 0; y < s->ny; ++y) {
    double rm = 0.0, re = 0.0;
    for (int x = 0; x < s->nx; ++x) {
      size_t k = idx(s, x, y);
      double r = 0, T = 0;
      for (int i = 0; i < 9; ++i) r += s->f[i * s->n + k];
      for (int i = 0; i < qg(&s->p); ++i) T += s->g[i * s->n + k];
      rm += r;
      re += r * s->p.cv * T;
    }
    m += rm;
    en += re;
  }
  *mass = m;
  *energy = en;
  *sumQ = s->last_sumQ;
  *sumS = s->last_sumS;
}

double orc_rho_ave(const orc_state* s) { return s->rho_ave; }

/* post-collision populations f* of the last step (for bookkeeping checks in the tests) */
void orc_get_post(const orc_state* s, double* fs) { memcpy(fs, s->fs, 9 * s->n * sizeof(double)); }

/* threads the grid loops run on */
int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
/* threads for the following grid loops (n >= 1; without OpenMP a no-op) */
void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
long orc_steps(const orc_state* s) { return s->steps; }

/* The matrices in use (for the identity checks of the tests). */
void orc_matrices(const orc_state* s, double* M, double* Minv, double* Mh, double* Mhinv) {
  memcpy(M, s->M, sizeof(s->M));
  memcpy(Minv, s->Minv, sizeof(s->Minv));
  memcpy(Mh, s->Mh, sizeof(s->Mh));
  memcpy(Mhinv, s->Mhinv, sizeof(s->Mhinv));
}
void orc_relaxation(const orc_state* s, double* Sdiag, double* Lam) {
  memcpy(Sdiag, s->Sdiag, sizeof(s->Sdiag));
  memcpy(Lam, s->Lam, sizeof(s->Lam));
}
