// Test driver of the library's host runtime built with AddressSanitizer and
// UndefinedBehaviorSanitizer (host code only; no GPU is used).  Calls every entry point that runs
// without a device: parameter checks (also on randomly corrupted parameter sets), footprints, tile
// shapes, the equation-of-state solves, error strings, and every context and batch call given
// invalid arguments.  Prints "coexistence <T/Tc> <rho_l> <rho_g> <p_sat>" lines for the caller to
// compare with the regular build, then "ok".  Exit status 1 on a broken expectation (a sanitizer
// finding aborts the program).
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <limits>
#include <random>

#include "lbm.h"
#include "lbm3d.h"

static int failures = 0;

#define EXPECT(cond)                                                  \
  do {                                                                \
    if (!(cond)) {                                                    \
      std::fprintf(stderr, "expectation failed at line %d: %s\n", __LINE__, #cond); \
      ++failures;                                                     \
    }                                                                 \
  } while (0)

template <typename P>
static void corrupt(P& p, std::mt19937_64& rng) {
  // overwrite one random 4- or 8-byte field of the struct with a special value
  const double dvals[] = {0.0, -1.0, 1e300, -1e300, std::numeric_limits<double>::quiet_NaN(),
                          std::numeric_limits<double>::infinity(), 1e-300, 0.5, 2.0, 1e6};
  const int32_t ivals[] = {0, -1, 1, 2, 3, 4, 5, 9, 64, 65, 1 << 30, INT32_MIN, INT32_MAX, 7};
  unsigned char* b = reinterpret_cast<unsigned char*>(&p);
  const size_t off4 = (rng() % (sizeof(P) / 4)) * 4;
  if (rng() % 2 && off4 % 8 == 0 && off4 + 8 <= sizeof(P)) {
    const double v = dvals[rng() % (sizeof(dvals) / sizeof(dvals[0]))];
    std::memcpy(b + off4, &v, 8);
  } else {
    const int32_t v = ivals[rng() % (sizeof(ivals) / sizeof(ivals[0]))];
    std::memcpy(b + off4, &v, 4);
  }
}

int main() {
  std::mt19937_64 rng(12345);

  // ---- parameters, footprints, shapes (two dimensions)
  lbm_params p;
  lbm_params_default(&p, 64, 48);
  EXPECT(lbm_validate(&p) == LBM_OK);
  EXPECT(lbm_footprint_bytes(&p) > 0);
  EXPECT(lbm_validate(nullptr) == LBM_E_INVAL);
  EXPECT(lbm_footprint_bytes(nullptr) == 0);
  for (int prec : {LBM_FP32, LBM_FP64}) {
    const int n = lbm_shape_count(prec);
    EXPECT(n > 0);
    for (int k = -2; k < n + 2; ++k) {
      int tx = 0, ty = 0, w = 0, d = 0;
      const lbm_status s = lbm_shape_info(prec, k, &tx, &ty, &w, &d);
      EXPECT((k >= 0 && k < n) == (s == LBM_OK));
      EXPECT(lbm_shape_info(prec, k, nullptr, nullptr, nullptr, nullptr) == s);
      for (int nx : {3, 7, 64, 65, 71, 200}) {
        for (int ny : {3, 5, 16, 17, 40}) {
          lbm_params q;
          lbm_params_default(&q, nx, ny);
          q.precision = prec;
          const int fits = lbm_shape_fits(&q, k);
          EXPECT(fits == 0 || fits == 1);
          if (k < 0 || k >= n) EXPECT(fits == 0);
        }
      }
    }
  }
  EXPECT(lbm_shape_count(7) == 0);
  for (int it = 0; it < 3000; ++it) {
    lbm_params q;
    lbm_params_default(&q, 3 + (int)(rng() % 300), 3 + (int)(rng() % 300));
    const int nbad = 1 + (int)(rng() % 3);
    for (int j = 0; j < nbad; ++j) corrupt(q, rng);
    const lbm_status s = lbm_validate(&q);
    EXPECT(s == LBM_OK || s == LBM_E_INVAL);
    const size_t fb = lbm_footprint_bytes(&q);
    EXPECT((s == LBM_OK) == (fb > 0));
    for (int k = -1; k < 10; ++k) (void)lbm_shape_fits(&q, k);
    double rl = 0, rg = 0, ps = 0;
    (void)lbm_eos_coexistence(&q, 0.86 * 0.0729, &rl, &rg, &ps);
    (void)lbm_critical_temperature(&q);
  }

  // ---- equation of state
  const double Tc = lbm_critical_temperature(&p);
  EXPECT(Tc > 0 && std::isfinite(Tc));
  for (double r : {0.5, 0.6, 0.7, 0.8, 0.86, 0.9, 0.95, 0.98}) {
    double rl = 0, rg = 0, ps = 0;
    EXPECT(lbm_eos_coexistence(&p, r * Tc, &rl, &rg, &ps) == LBM_OK);
    EXPECT(rl > rg && rg > 0 && ps > 0);
    std::printf("coexistence %.17g %.17g %.17g %.17g\n", r, rl, rg, ps);
  }
  for (double r : {-1.0, 0.0, 1.0, 1.5, std::numeric_limits<double>::quiet_NaN()}) {
    double rl = 0, rg = 0, ps = 0;
    EXPECT(lbm_eos_coexistence(&p, r * Tc, &rl, &rg, &ps) != LBM_OK);
  }
  EXPECT(lbm_eos_coexistence(nullptr, 0.86 * Tc, nullptr, nullptr, nullptr) == LBM_E_INVAL);

  // ---- error strings
  for (int s = LBM_E_STATE; s <= LBM_OK; ++s) {
    const char* t = lbm_strerror((lbm_status)s);
    EXPECT(t != nullptr && std::strlen(t) > 0);
  }
  EXPECT(lbm_last_error(nullptr) != nullptr);

  // ---- context and batch calls with invalid arguments (no device needed to reject them)
  lbm_ctx* h = nullptr;
  EXPECT(lbm_create(nullptr, nullptr, 0, nullptr, &h) == LBM_E_INVAL);
  EXPECT(lbm_create(&p, nullptr, 0, nullptr, nullptr) == LBM_E_INVAL);
  EXPECT(lbm_init(nullptr, nullptr, nullptr, nullptr, nullptr) == LBM_E_INVAL);
  EXPECT(lbm_step(nullptr, 1) == LBM_E_INVAL);
  EXPECT(lbm_steps_done(nullptr) == -1);
  EXPECT(lbm_set_shape(nullptr, 0) == LBM_E_INVAL);
  EXPECT(lbm_get_shape(nullptr) < 0);
  EXPECT(lbm_set_tile_order(nullptr, 0) == LBM_E_INVAL);
  EXPECT(lbm_sync(nullptr) == LBM_E_INVAL);
  EXPECT(lbm_read_fields(nullptr, nullptr, nullptr, nullptr, nullptr) == LBM_E_INVAL);
  EXPECT(lbm_diagnostics(nullptr, nullptr, nullptr) == LBM_E_INVAL);
  EXPECT(lbm_set_diagnostics_interval(nullptr, 1) == LBM_E_INVAL);
  int cnt = 0;
  EXPECT(lbm_read_diagnostics_log(nullptr, nullptr, nullptr, nullptr, 0, &cnt) == LBM_E_INVAL);
  int32_t rows[4];
  EXPECT(lbm_vapour_rows(nullptr, 1.0, 0, 1, rows) == LBM_E_INVAL);
  lbm_component comp[2];
  int ncomp = -1;
  EXPECT(lbm_vapour_components(nullptr, 1.0, 0, 1, comp, 2, &ncomp) == LBM_E_INVAL);
  EXPECT(lbm_state_bytes(nullptr) == 0);
  EXPECT(lbm_save_state(nullptr, nullptr, 0) == LBM_E_INVAL);
  EXPECT(lbm_load_state(nullptr, nullptr, 0) == LBM_E_INVAL);
  EXPECT(lbm_read_state(nullptr, nullptr, nullptr, nullptr) == LBM_E_INVAL);
  EXPECT(lbm_destroy(nullptr) == LBM_E_INVAL);
  EXPECT(lbm_device_copy(nullptr, nullptr, 16, nullptr) == LBM_E_INVAL);
  for (int n : {-1, 0, 1, 64, 4096}) {
    const size_t b = lbm_batch_footprint_bytes(n);
    EXPECT((n > 0) == (b > 0));
  }
  lbm_batch* bt = nullptr;
  EXPECT(lbm_batch_create(nullptr, 1, nullptr, 0, nullptr, &bt) == LBM_E_INVAL);
  EXPECT(lbm_batch_create_noalloc(nullptr, 1, nullptr, &bt) == LBM_E_INVAL);
  EXPECT(lbm_batch_set_budget(nullptr, 0, 1) == LBM_E_INVAL);
  EXPECT(lbm_batch_step(nullptr, 1) == LBM_E_INVAL);
  EXPECT(lbm_batch_remaining(nullptr, 0) < 0);
  EXPECT(lbm_batch_set_shape(nullptr, 0) == LBM_E_INVAL);
  EXPECT(lbm_batch_set_persistent(nullptr, 1, 0) == LBM_E_INVAL);
  EXPECT(lbm_batch_set_diagnostics_interval(nullptr, 10) == LBM_E_INVAL);
  EXPECT(lbm_batch_sync(nullptr, nullptr) == LBM_E_INVAL);
  EXPECT(lbm_batch_destroy(nullptr) == LBM_E_INVAL);

  // ---- three dimensions
  lbm3d_params p3;
  lbm3d_params_default(&p3, 32, 24, 16);
  EXPECT(lbm3d_validate(&p3) == LBM_OK);
  EXPECT(lbm3d_footprint_bytes(&p3) > 0);
  EXPECT(lbm3d_validate(nullptr) == LBM_E_INVAL);
  for (int it = 0; it < 3000; ++it) {
    lbm3d_params q;
    lbm3d_params_default(&q, 3 + (int)(rng() % 100), 3 + (int)(rng() % 100), 3 + (int)(rng() % 100));
    const int nbad = 1 + (int)(rng() % 3);
    for (int j = 0; j < nbad; ++j) corrupt(q, rng);
    const lbm_status s = lbm3d_validate(&q);
    EXPECT(s == LBM_OK || s == LBM_E_INVAL);
    EXPECT((s == LBM_OK) == (lbm3d_footprint_bytes(&q) > 0));
  }
  lbm3d_ctx* h3 = nullptr;
  EXPECT(lbm3d_create(nullptr, nullptr, 0, nullptr, &h3) == LBM_E_INVAL);
  EXPECT(lbm3d_init(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) == LBM_E_INVAL);
  EXPECT(lbm3d_step(nullptr, 1) == LBM_E_INVAL);
  EXPECT(lbm3d_sync(nullptr) == LBM_E_INVAL);
  EXPECT(lbm3d_read_fields(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) == LBM_E_INVAL);
  EXPECT(lbm3d_diagnostics(nullptr, nullptr, nullptr) == LBM_E_INVAL);
  EXPECT(lbm3d_state_bytes(nullptr) == 0);
  EXPECT(lbm3d_save_state(nullptr, nullptr, 0) == LBM_E_INVAL);
  EXPECT(lbm3d_load_state(nullptr, nullptr, 0) == LBM_E_INVAL);
  EXPECT(lbm3d_destroy(nullptr) == LBM_E_INVAL);

  if (failures) {
    std::fprintf(stderr, "%d expectation(s) failed\n", failures);
    return 1;
  }
  std::printf("ok\n");
  return 0;
}
