// Host-side checks of the C ABI under AddressSanitizer and UndefinedBehaviorSanitizer: every
// validation path that runs before a device call (bad geometry, NULL and out-of-range
// arguments, status strings, plan-free utilities) is exercised; on a host without a GPU a
// valid geometry ends in TOMO_ERR_NO_DEVICE.  Built and run by tests/test_host_sanitizers.py;
// any sanitizer report or failed check ends the program with a non-zero status.
#include <cmath>
#include <cstdio>
#include <cstring>

#include "tomo.h"
#include "tomo_nn.h"
#include "tomo_pipeline.h"

static int failures = 0;
#define CHECK(cond)                                                         \
  do {                                                                      \
    if (!(cond)) {                                                          \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #cond, __LINE__); \
      ++failures;                                                           \
    }                                                                       \
  } while (0)

static tomo_geometry_t geom() {
  tomo_geometry_t g;
  std::memset(&g, 0, sizeof g);
  g.n = 64;
  g.n_slices = 2;
  g.n_angles = 30;
  g.n_det = 92;
  g.center = NAN;
  g.kb_width = 6;
  g.kb_oversamp = 2.0;
  g.beta = 0.01;
  g.p = 1.2;
  g.q = 2.0;
  g.sigma = 0.1;
  g.T = 1.0;
  g.neighbours = 26;
  return g;
}

int main() {
  for (int s = 0; s < 10; ++s) CHECK(std::strlen(tomo_status_string(s)) > 0);
  CHECK(std::strcmp(tomo_status_string(99), "unknown status") == 0);
  CHECK(std::strcmp(tomo_status_string(-1), "unknown status") == 0);
  CHECK(tomo_last_error(nullptr) != nullptr);

  tomo_plan plan = reinterpret_cast<tomo_plan>(0x1);
  CHECK(tomo_plan_create(nullptr, nullptr, &plan) == TOMO_ERR_INVALID_ARG);
  CHECK(tomo_plan_create(nullptr, nullptr, nullptr) == TOMO_ERR_INVALID_ARG);
  const double angles[3] = {0.0, INFINITY, 1.0};
  struct Bad { const char* what; void (*set)(tomo_geometry_t&); };
  const Bad bad[] = {
      {"odd n", [](tomo_geometry_t& g) { g.n = 17; }},
      {"large n", [](tomo_geometry_t& g) { g.n = 4096; }},
      {"no slices", [](tomo_geometry_t& g) { g.n_slices = 0; }},
      {"odd detector", [](tomo_geometry_t& g) { g.n_det = 91; }},
      {"pad", [](tomo_geometry_t& g) { g.pad = 100; }},
      {"levels", [](tomo_geometry_t& g) { g.n_levels = 7; }},
      {"level detector", [](tomo_geometry_t& g) { g.n_levels = 2; g.n_det = 90; }},
      {"kb width", [](tomo_geometry_t& g) { g.kb_width = 17; }},
      {"oversampling", [](tomo_geometry_t& g) { g.kb_oversamp = 1.0; }},
      {"p", [](tomo_geometry_t& g) { g.p = 2.5; }},
      {"q", [](tomo_geometry_t& g) { g.q = 1.5; }},
      {"sigma", [](tomo_geometry_t& g) { g.sigma = 0.0; }},
      {"neighbours", [](tomo_geometry_t& g) { g.neighbours = 6; }},
      {"flags", [](tomo_geometry_t& g) { g.flags = 8; }},
      {"center", [](tomo_geometry_t& g) { g.center = INFINITY; }},
  };
  for (const Bad& b : bad) {
    tomo_geometry_t g = geom();
    b.set(g);
    plan = reinterpret_cast<tomo_plan>(0x1);
    const tomo_status s = tomo_plan_create(&g, nullptr, &plan);
    if (s != TOMO_ERR_INVALID_ARG) std::fprintf(stderr, "geometry '%s' not rejected\n", b.what);
    CHECK(s == TOMO_ERR_INVALID_ARG && plan == nullptr);
    CHECK(std::strlen(tomo_last_error(nullptr)) > 0);
  }
  {
    tomo_geometry_t g = geom();
    g.n_angles = 3;
    g.angles = angles;
    CHECK(tomo_plan_create(&g, nullptr, &plan) == TOMO_ERR_INVALID_ARG);
  }
  {
    tomo_geometry_t g = geom();
    const tomo_status s = tomo_plan_create(&g, nullptr, &plan);
    CHECK(s == TOMO_ERR_NO_DEVICE || s == TOMO_OK);
    if (s == TOMO_OK) tomo_plan_destroy(plan);
  }
  CHECK(tomo_plan_destroy(nullptr) == TOMO_OK);
  size_t bytes = 0;
  CHECK(tomo_plan_workspace_size(nullptr, &bytes) == TOMO_ERR_INVALID_ARG);
  CHECK(tomo_plan_set_workspace(nullptr, nullptr, 0) == TOMO_ERR_INVALID_ARG);
  CHECK(tomo_reconstruct(nullptr, nullptr, nullptr, nullptr, nullptr) == TOMO_ERR_INVALID_ARG);
  CHECK(tomo_gradient(nullptr, nullptr, nullptr, nullptr, nullptr) == TOMO_ERR_INVALID_ARG);
  CHECK(tomo_gradient_direct(nullptr, nullptr, nullptr, nullptr, nullptr) == TOMO_ERR_INVALID_ARG);
  CHECK(tomo_forward_project(nullptr, nullptr, nullptr) == TOMO_ERR_INVALID_ARG);
  CHECK(tomo_lanczos_prolong(nullptr, nullptr, 16, 1, nullptr) == TOMO_ERR_INVALID_ARG);
  tomo_batch batch = nullptr;
  CHECK(tomo_batch_create(nullptr, 0, nullptr, &batch) == TOMO_ERR_INVALID_ARG);
  CHECK(tomo_batch_destroy(nullptr) == TOMO_OK);

  CHECK(tomo_plan_geometry(nullptr, nullptr, nullptr, nullptr) == TOMO_ERR_INVALID_ARG);
  {
    int32_t f = -1, a = -1, b = -1, w = -1;
    CHECK(tomo_pipeline_window(11, 4, 0, 2, &f, &a, &b, &w) == TOMO_OK);
    CHECK(f == 7 && a == 8 && b == 11 && w == 3);
    CHECK(tomo_pipeline_window(13, 6, 2, 0, &f, &a, &b, nullptr) == TOMO_OK && f == 0 && a == 0 && b == 2);
    CHECK(tomo_pipeline_window(3, 4, 0, 0, &f, &a, &b, &w) == TOMO_ERR_INVALID_ARG);
    CHECK(tomo_pipeline_window(10, 4, 2, 0, &f, &a, &b, &w) == TOMO_ERR_INVALID_ARG);
    CHECK(tomo_pipeline_window(10, 4, 0, 3, &f, &a, &b, &w) == TOMO_ERR_INVALID_ARG);
    CHECK(tomo_pipeline_window(10, 4, 0, 0, nullptr, &a, &b, &w) == TOMO_ERR_INVALID_ARG);
    CHECK(std::strlen(tomo_pipeline_last_error(nullptr)) > 0);
    tomo_pipeline pipe = reinterpret_cast<tomo_pipeline>(0x1);
    CHECK(tomo_pipeline_create(nullptr, 16, 0, 2, &pipe) == TOMO_ERR_INVALID_ARG && pipe == nullptr);
    CHECK(tomo_pipeline_create(nullptr, 16, 0, 2, nullptr) == TOMO_ERR_INVALID_ARG);
    CHECK(tomo_pipeline_workspace_size(nullptr, &bytes) == TOMO_ERR_INVALID_ARG);
    CHECK(tomo_pipeline_set_workspace(nullptr, nullptr, 0) == TOMO_ERR_INVALID_ARG);
    CHECK(tomo_pipeline_run(nullptr, nullptr, nullptr, nullptr, nullptr) == TOMO_ERR_INVALID_ARG);
    CHECK(tomo_pipeline_destroy(nullptr) == TOMO_OK);
  }

  tomo_unet net = reinterpret_cast<tomo_unet>(0x1);
  CHECK(tomo_unet_create(0, 32, 1, 64, 64, nullptr, &net) == TOMO_ERR_INVALID_ARG);
  CHECK(tomo_unet_create(2, 40, 1, 64, 64, nullptr, &net) == TOMO_ERR_INVALID_ARG);
  CHECK(tomo_unet_create(3, 32, 1, 66, 64, nullptr, &net) == TOMO_ERR_INVALID_ARG);
  {
    const tomo_status s = tomo_unet_create(2, 32, 1, 64, 64, nullptr, &net);
    CHECK(s == TOMO_ERR_NO_DEVICE || s == TOMO_OK);
    if (s == TOMO_OK) tomo_unet_destroy(net);
  }
  CHECK(tomo_unet_set_domain(nullptr, nullptr) == TOMO_ERR_INVALID_ARG);
  size_t floats = 0;
  CHECK(tomo_nn_wgrad_scratch(64, 96, 4096, &floats) == TOMO_OK && floats > 0);
  CHECK(tomo_nn_wgrad_scratch(48, 96, 4096, &floats) == TOMO_ERR_INVALID_ARG);
  CHECK(tomo_nn_conv3x3(nullptr, 32, nullptr, nullptr, nullptr, 32, nullptr, 0, 32, 32, 1, 8, 8, 0,
                        nullptr) == TOMO_ERR_INVALID_ARG);
  CHECK(tomo_nn_conv3x3_wgrad(nullptr, 32, nullptr, 32, nullptr, nullptr, 32, 32, 1, 8, 8, nullptr, 0,
                              nullptr) == TOMO_ERR_INVALID_ARG);
  CHECK(tomo_nn_conv3x3_wgrad_noalloc(nullptr, 32, nullptr, 32, nullptr, nullptr, 32, 32, 1, 8, 8,
                                      nullptr) == TOMO_ERR_INVALID_ARG);
  if (failures) std::fprintf(stderr, "%d checks failed\n", failures);
  else std::printf("sanitized host checks passed\n");
  return failures ? 1 : 0;
}
