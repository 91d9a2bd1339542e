// Host-side checks of the C-ABI under AddressSanitizer and
// UndefinedBehaviorSanitizer (built by tests/test_host_sanitizers.py with
// the sanitizers on the host pass only; the device code is the library's).
// Runs every entry point that needs no GPU: parameter validation and buffer
// layout for many lattice shapes, the rejection paths of create / batch /
// adjoint / state / norms calls, and the host parameter pipeline of the
// refinement rules.  Any sanitizer finding aborts with a report; the exit
// status is the number of failed expectations.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../include/lbm_pp.h"

static int g_fail = 0;
#define EXPECT(cond)                                                      \
  do {                                                                    \
    if (!(cond)) {                                                        \
      std::fprintf(stderr, "expectation failed: %s (line %d)\n", #cond, __LINE__); \
      ++g_fail;                                                           \
    }                                                                     \
  } while (0)

int main() {
  // status strings, including codes outside the enum
  for (int s = -2; s < 10; ++s) EXPECT(lbm_status_string(static_cast<lbm_status>(s)) != nullptr);
  EXPECT(lbm_last_error(nullptr) != nullptr);

  // parameter validation and layout over many shapes
  const int shapes[][2] = {{1, 1}, {1, 6}, {6, 1}, {3, 3}, {61, 5}, {150, 70}, {512, 512},
                           {1024, 2048}, {4096, 4096}, {16384, 16384}, {1, 2560}};
  for (auto& sh : shapes) {
    for (int walls = 0; walls < 2; ++walls)
      for (int prec = 0; prec < 2; ++prec)
        for (int outflow = 0; outflow < 2; ++outflow) {
          lbm_params p;
          lbm_default_params(&p, sh[0], sh[1]);
          p.walls = walls;
          p.precision = prec;
          p.outflow_top = outflow;
          p.thermal = 1;
          size_t n = 0;
          const lbm_status v = lbm_validate(&p);
          const lbm_status b = lbm_buffer_bytes(&p, &n);
          EXPECT(v == b);
          if (v == LBM_OK) {
            const size_t elem = prec ? 4 : 8;
            EXPECT(n >= size_t(20) * size_t(sh[0]) * size_t(sh[1]) * elem);
          }
          for (int ty : {0, 2, 5, 13, 100}) {
            p.tile_y = ty;
            (void)lbm_buffer_bytes(&p, &n);
          }
        }
  }
  {
    lbm_params p;
    lbm_default_params(&p, 16, 16);
    lbm_params bad = p;
    bad.nx = 0;
    EXPECT(lbm_validate(&bad) == LBM_E_INVAL);
    bad = p;
    bad.s_e = 2.0;
    EXPECT(lbm_validate(&bad) == LBM_E_INVAL);
    bad = p;
    bad.rho_l = bad.rho_v;
    EXPECT(lbm_validate(&bad) == LBM_E_INVAL);
    bad = p;
    bad.tile_y = 1;
    EXPECT(lbm_validate(&bad) == LBM_E_INVAL);
    EXPECT(lbm_validate(nullptr) == LBM_E_INVAL);
    size_t n = 0;
    EXPECT(lbm_buffer_bytes(nullptr, &n) == LBM_E_INVAL);

    // create: every rejection path before (and at) the first runtime call
    lbm_ctx* c = nullptr;
    EXPECT(lbm_create(&p, nullptr, 1 << 20, nullptr, &c) == LBM_E_INVAL && c == nullptr);
    EXPECT(lbm_create(&p, reinterpret_cast<void*>(257), size_t(1) << 30, nullptr, &c) == LBM_E_INVAL);
    EXPECT(lbm_create(&p, reinterpret_cast<void*>(256), 16, nullptr, &c) == LBM_E_NOMEM);
    EXPECT(lbm_create(&p, reinterpret_cast<void*>(256), 1 << 20, nullptr, nullptr) == LBM_E_INVAL);
    EXPECT(lbm_create(&bad, reinterpret_cast<void*>(256), 1 << 20, nullptr, &c) != LBM_OK);
    lbm_destroy(nullptr);

    // calls on a null context
    double d = 0;
    int64_t k = 0;
    lbm_norms_t nm;
    EXPECT(lbm_step(nullptr, 1) == LBM_E_INVAL);
    EXPECT(lbm_sync(nullptr) == LBM_E_INVAL);
    EXPECT(lbm_norms(nullptr, &nm) == LBM_E_INVAL);
    EXPECT(lbm_norms_device(nullptr, nullptr) == LBM_E_INVAL);
    EXPECT(lbm_read_fields(nullptr, &d, &d, &d, &d) == LBM_E_INVAL);
    EXPECT(lbm_read_populations(nullptr, &d) == LBM_E_INVAL);
    EXPECT(lbm_init_fields(nullptr, &d, nullptr, nullptr, &d) == LBM_E_INVAL);
    EXPECT(lbm_set_boundary(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) == LBM_E_INVAL);
    EXPECT(lbm_save_state(nullptr, &d, 8) == LBM_E_INVAL);
    EXPECT(lbm_load_state(nullptr, &d, 8) == LBM_E_INVAL);
    EXPECT(lbm_state_bytes(nullptr, &n) == LBM_E_INVAL);
    EXPECT(lbm_set_tile_y(nullptr, 5) == LBM_E_INVAL);
    EXPECT(lbm_get_tile_y(nullptr) < 0 || lbm_get_tile_y(nullptr) == 0);
    EXPECT(lbm_step_count(nullptr) == -1);
    EXPECT(lbm_last_step_time(nullptr, &d) == LBM_E_INVAL);
    EXPECT(lbm_kernel_timing(nullptr, 1) == LBM_E_INVAL);
    EXPECT(lbm_kernel_times(nullptr, &d, &k) == LBM_E_INVAL);
    int32_t cnt = 0;
    EXPECT(lbm_tile_candidates(nullptr, 0, nullptr, 0, &cnt) == LBM_E_INVAL);
    int32_t bt = 0;
    const int32_t cand[] = {4, 8};
    EXPECT(lbm_autotune_tile_y(nullptr, cand, 2, 3, &bt, &d) == LBM_E_INVAL);

    // batches and adjoint: sizes and rejections
    for (int prec = 0; prec < 2; ++prec) {
      EXPECT(lbm_batch_bytes(prec, &n) == LBM_OK && n > 0);
    }
    EXPECT(lbm_batch_bytes(7, &n) == LBM_E_INVAL);
    lbm_batch* bb = nullptr;
    EXPECT(lbm_batch_create(nullptr, 1, reinterpret_cast<void*>(256), 1 << 20, nullptr, &bb) == LBM_E_INVAL);
    lbm_ctx* none[1] = {nullptr};
    EXPECT(lbm_batch_create(none, 1, reinterpret_cast<void*>(256), 1 << 20, nullptr, &bb) == LBM_E_INVAL);
    EXPECT(lbm_batch_create(none, 0, reinterpret_cast<void*>(256), 1 << 20, nullptr, &bb) == LBM_E_INVAL);
    const int64_t steps[1] = {3};
    EXPECT(lbm_batch_run(nullptr, steps, 1) == LBM_E_INVAL);
    EXPECT(lbm_batch_prepare(nullptr, steps, 1) == LBM_E_INVAL);
    EXPECT(lbm_batch_last_time(nullptr, &d, &k, &k) == LBM_E_INVAL);
    lbm_batch_destroy(nullptr);
    EXPECT(lbm_batch_last_error(nullptr) != nullptr);
    lbm_params q = p;
    q.thermal = 1;
    EXPECT(lbm_adjoint_bytes(&q, 500, 50, &n) == LBM_OK && n > 0);
    EXPECT(lbm_adjoint_bytes(&q, 0, 50, &n) == LBM_E_INVAL);
    q.walls = 1;
    EXPECT(lbm_adjoint_bytes(&q, 10, 5, &n) == LBM_E_UNSUPPORTED);
    EXPECT(lbm_adjoint_create(nullptr, 10, 5, 3.0, 1.0, nullptr, 0, nullptr) == LBM_E_INVAL);
    EXPECT(lbm_adjoint_forward(nullptr, &d) == LBM_E_INVAL);
    EXPECT(lbm_adjoint_backward(nullptr, 1.0, &d) == LBM_E_INVAL);
    lbm_adjoint_destroy(nullptr);
  }

  // host parameter pipeline (Sec. 3): Maxwell, sigma, gamma, refinement levels
  const double a = 2.0 / 49.0, b = 2.0 / 21.0;
  const double Tc = lbm_pr_critical_temperature(a, b, 1.0);
  EXPECT(std::isfinite(Tc) && Tc > 0.0);
  double rv = 0, rl = 0, ps = 0, sg = 0, g0 = 0;
  EXPECT(lbm_pr_maxwell(a, b, 1.0, 0.344, 0.86 * Tc, &rv, &rl, &ps) == LBM_OK);
  EXPECT(rv > 0.3 && rv < 0.4 && rl > 6.4 && rl < 6.6);
  EXPECT(lbm_pr_maxwell(a, b, 1.0, 0.344, 1.01 * Tc, &rv, &rl, &ps) != LBM_OK);
  EXPECT(lbm_fit_sigma(a, b, 1.0, 0.344, -1.0, 0.86 * Tc, &sg) == LBM_OK && sg > 0.1 && sg < 0.12);
  EXPECT(lbm_planar_gamma(a, b, 1.0, 0.344, -1.0, 0.86 * Tc, sg, &g0) == LBM_OK && g0 > 0.0);
  double hfg = 0, beta = 0;
  EXPECT(lbm_pr_maxwell(a, b, 1.0, 0.344, 0.86 * Tc, &rv, &rl, &ps) == LBM_OK);
  EXPECT(lbm_pr_latent_heat(a, b, 1.0, 0.344, 0.86 * Tc, rv, rl, &hfg) == LBM_OK && hfg > 0.0);
  EXPECT(lbm_pr_latent_heat(a, b, 1.0, 0.344, 0.86 * Tc, rl, rv, &hfg) == LBM_E_INVAL);
  EXPECT(lbm_pr_latent_heat(a, b, 1.0, 0.344, 0.86 * Tc, rv, rl, nullptr) == LBM_E_INVAL);
  EXPECT(lbm_stefan_beta(0.038, &beta) == LBM_OK && beta > 0.1 && beta < 0.2);
  EXPECT(lbm_stefan_beta(-1.0, &beta) == LBM_E_INVAL);
  EXPECT(lbm_stefan_beta(1e300, &beta) == LBM_OK && beta > 20.0 && beta < 30.0);
  for (int m = 0; m <= 5; ++m) {
    lbm_level lv;
    const double dx = std::ldexp(1.0, -m);
    EXPECT(lbm_refinement_level(a, dx, 0.86, b, 1.0, 0.344, -1.0, 0.0, -3e-5, 800, &lv) == LBM_OK);
    EXPECT(std::fabs(lv.a / (a * dx * dx) - 1.0) < 1e-14);
    EXPECT(lv.steps == int64_t(std::llround(800.0 / (dx * dx))));
  }
  EXPECT(lbm_refinement_level(a, 0.5, 0.86, b, 1.0, 0.344, -1.0, 0.0, -3e-5, 800, nullptr) == LBM_E_INVAL);

  std::printf("host sanitizer harness: %d failed expectations\n", g_fail);
  return g_fail;
}
