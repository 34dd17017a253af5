// Drives the host-only paths of libcuba's C ABI -- parameter validation,
// workspace sizing, argument checks that return before any device work,
// error strings -- so that a build whose host code runs under
// AddressSanitizer and UndefinedBehaviorSanitizer reports any fault in
// them.  Needs no GPU: no call here reaches the device.  Exits non-zero on
// a failed check.
#include <cmath>
#include <cstdio>
#include <cstring>

#include "cuba.h"

#define CHECK(cond)                                                     \
  do {                                                                  \
    if (!(cond)) {                                                      \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #cond, __LINE__); \
      return 1;                                                         \
    }                                                                   \
  } while (0)

static cuba_params tube() {
  cuba_params p;
  std::memset(&p, 0, sizeof p);
  p.box[0] = 10.0; p.box[1] = 1.0; p.box[2] = 1.0;
  p.cells[0] = 100; p.cells[1] = 1; p.cells[2] = 1;
  p.sigma = 0.4; p.r_test = 100.0; p.dt = 0.02; p.seed = 1; p.cell_capacity = 256;
  return p;
}

int main() {
  const cuba_params p = tube();
  const size_t ws = cuba_workspace_bytes(&p, 10209);
  CHECK(ws > 0 && ws % 256 == 0);
  CHECK(cuba_workspace_bytes(nullptr, 10) == 0);
  CHECK(cuba_workspace_bytes(&p, -1) == 0);

  // every invalid parameter cuba_init rejects, before any device work
  struct Bad { const char *what; void (*edit)(cuba_params &); };
  const Bad bad[] = {
      {"box", [](cuba_params &q) { q.box[1] = 0.0; }},
      {"box nan", [](cuba_params &q) { q.box[2] = NAN; }},
      {"cells", [](cuba_params &q) { q.cells[0] = 0; }},
      {"cells overflow", [](cuba_params &q) { q.cells[0] = q.cells[1] = q.cells[2] = 2000; }},
      {"sigma", [](cuba_params &q) { q.sigma = -1.0; }},
      {"r_test", [](cuba_params &q) { q.r_test = 0.0; }},
      {"dt", [](cuba_params &q) { q.dt = 0.5; }},
      {"dt inf", [](cuba_params &q) { q.dt = INFINITY; }},
      {"2K > 1", [](cuba_params &q) { q.sigma = 1e6; }},
      {"capacity", [](cuba_params &q) { q.cell_capacity = CUBA_MAX_CELL_CAPACITY + 1; }},
  };
  double dummy_arr[4] = {0, 0, 0, 0};
  const double *d = dummy_arr;
  for (const Bad &b : bad) {
    cuba_params q = p;
    b.edit(q);
    CHECK(cuba_workspace_bytes(&q, 100) == 0);
    cuba_ctx *ctx = reinterpret_cast<cuba_ctx *>(0x1);
    const int rc = cuba_init(&ctx, &q, 100, d, d, d, d, d, d, nullptr, 0, nullptr);
    if (rc != CUBA_EINVAL) std::fprintf(stderr, "case %s: rc %d\n", b.what, rc);
    CHECK(rc == CUBA_EINVAL && ctx == nullptr);
    CHECK(std::strlen(cuba_last_error()) > 0);
    CHECK(cuba_init_static(&ctx, &q, 100, d, d, d, d, d, d, nullptr) == CUBA_EINVAL);
  }
  cuba_ctx *ctx = nullptr;
  CHECK(cuba_init(nullptr, &p, 1, d, d, d, d, d, d, nullptr, 0, nullptr) == CUBA_EINVAL);
  CHECK(cuba_init(&ctx, &p, -5, d, d, d, d, d, d, nullptr, 0, nullptr) == CUBA_EINVAL);
  CHECK(cuba_init(&ctx, &p, 10, nullptr, d, d, d, d, d, nullptr, 0, nullptr) == CUBA_EINVAL);
  // workspace: missing, misaligned, too small
  alignas(256) static char small[512];
  CHECK(cuba_init(&ctx, &p, 10, d, d, d, d, d, d, nullptr, ws, nullptr) == CUBA_EINVAL);
  CHECK(cuba_init(&ctx, &p, 10, d, d, d, d, d, d, small + 8, ws, nullptr) == CUBA_EINVAL);
  CHECK(cuba_init(&ctx, &p, 10, d, d, d, d, d, d, small, sizeof small, nullptr) == CUBA_ENOMEM);
  // the library's own workspace is bounded
  cuba_params big = p;
  big.box[1] = big.box[2] = 8.0;
  big.cells[1] = big.cells[2] = 40;
  big.cell_capacity = 1024;
  CHECK(cuba_workspace_bytes(&big, 1000) > CUBA_STATIC_WORKSPACE_BYTES);
  CHECK(cuba_init_static(&ctx, &big, 1000, d, d, d, d, d, d, nullptr) == CUBA_ENOMEM);
  CHECK(ctx == nullptr);

  // calls on a NULL context or with NULL outputs
  uint64_t counters[3];
  double ms[CUBA_NUM_STAGES];
  int64_t launches[CUBA_NUM_STAGES];
  int32_t lanes = 0;
  double dt = 0.0;
  CHECK(cuba_step(nullptr, 1) == CUBA_EINVAL);
  CHECK(cuba_observe(nullptr, nullptr, nullptr) == CUBA_EINVAL);
  CHECK(cuba_observe_moments(nullptr, nullptr) == CUBA_EINVAL);
  CHECK(cuba_get_state(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) ==
        CUBA_EINVAL);
  CHECK(cuba_trace_step(nullptr, nullptr) == CUBA_EINVAL);
  CHECK(cuba_sync(nullptr) == CUBA_EINVAL);
  CHECK(cuba_set_cell_lanes(nullptr, 0) == CUBA_EINVAL);
  CHECK(cuba_get_cell_lanes(nullptr, &lanes) == CUBA_EINVAL);
  CHECK(cuba_set_dt(nullptr, 0.01) == CUBA_EINVAL);
  CHECK(cuba_get_dt(nullptr, &dt) == CUBA_EINVAL);
  CHECK(cuba_info(nullptr, nullptr, nullptr, nullptr) == CUBA_EINVAL);
  CHECK(cuba_counters(nullptr, counters) == CUBA_EINVAL);
  CHECK(cuba_timing_begin(nullptr, 4) == CUBA_EINVAL);
  CHECK(cuba_timing_begin_sampled(nullptr, 4, 10) == CUBA_EINVAL);
  CHECK(cuba_timing_end(nullptr, ms, launches) == CUBA_EINVAL);
  cuba_destroy(nullptr);

  // batches: sizing and argument checks
  CHECK(cuba_batch_workspace_bytes(16) > 0);
  cuba_batch *b = nullptr;
  CHECK(cuba_batch_create(&b, 0, small, sizeof small, nullptr) == CUBA_EINVAL);
  CHECK(cuba_batch_create(&b, 4, nullptr, 0, nullptr) == CUBA_EINVAL);
  CHECK(cuba_batch_create(&b, 4096, small, sizeof small, nullptr) == CUBA_ENOMEM);
  int32_t bad_slot = 0;
  CHECK(cuba_batch_step(nullptr, 1) == CUBA_EINVAL);
  CHECK(cuba_batch_sync(nullptr, &bad_slot) == CUBA_EINVAL);
  CHECK(cuba_batch_slot(nullptr, 0) == nullptr);
  CHECK(cuba_batch_set_observe(nullptr, 0, 7, nullptr, 1) == CUBA_EINVAL);
  cuba_batch_destroy(nullptr);

  // capacity suggestion: scratch sizing and the checks before device work
  CHECK(cuba_capacity_scratch_bytes(&p) > 0);
  CHECK(cuba_capacity_scratch_bytes(nullptr) == 0);
  int32_t cap = 0;
  CHECK(cuba_suggest_cell_capacity(&p, 0, nullptr, nullptr, nullptr, nullptr, 0, nullptr,
                                   nullptr) == CUBA_EINVAL);
  CHECK(cuba_suggest_cell_capacity(&p, 4, nullptr, nullptr, nullptr, small, sizeof small,
                                   nullptr, &cap) == CUBA_EINVAL);
  CHECK(cuba_suggest_cell_capacity(&p, 0, nullptr, nullptr, nullptr, nullptr, 0, nullptr,
                                   &cap) == CUBA_EINVAL);

  for (int code = 1; code >= -5; --code) CHECK(std::strlen(cuba_strerror(code)) > 0);
  CHECK(std::strncmp(cuba_build_info(), "sources ", 8) == 0);
  std::printf("api sanitizer run ok\n");
  return 0;
}
