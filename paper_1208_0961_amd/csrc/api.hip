// api.hip -- the C ABI of libcuba.so (declared in include/cuba.h): parameter
// validation, the workspace layout, the launch order of one step, and
// error reporting.  All device state lives in the caller's workspace.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "cuba.h"
#include "internal.hpp"

using namespace cuba;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string &msg) {
  g_last_error = msg;
  return code;
}

int hip_fail(hipError_t e, const char *where) {
  return fail(CUBA_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

inline size_t align256(size_t v) { return (v + 255u) & ~(size_t)255u; }

// Byte offsets of every array inside the workspace.
struct Layout {
  size_t status;
  size_t soa[2][7];  // x y z px py pz id, for the two buffers: C x cap block
                     // slots, then n spill slots
  size_t count[2];   // per-cell particle counts of the two buffers
  size_t spill_desc[2];      // SpillDesc of each buffer
  size_t spill_cell[2], spill_ocell[2], spill_hdr[2];
  size_t pool_desc, pool, pool_hdr;  // scratch for stepping overflowing cells
  uint64_t pool_words;
  size_t offsets, tile_sums, cell_sums;
  size_t consts;  // device copy of the geometry
  size_t total;
};

// What the kernels read from device memory instead of kernel arguments.
struct DeviceConsts {
  Geometry g;
};

// The spill slots of a buffer hold every particle of the context (so no
// binning can lose one); the pool holds, per overflowing cell of n members,
// its n - cap spilled members' slots and, for a cell larger than the LDS
// holds, n + n / 2 + 1 + (n + 31) / 32 words more: at most 3 n_total plus 3
// words per cell in all.
Layout make_layout(int64_t n_cells, uint32_t cap, int64_t n) {
  Layout L{};
  size_t off = 0;
  auto take = [&off](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  const size_t cc = (size_t)n_cells;
  const size_t slots = cc * cap;
  const size_t sn = n > 0 ? (size_t)n : 1u;
  const size_t tiles = (cc + kScanTile - 1) / kScanTile;
  L.status = take(sizeof(DevStatus));
  // the two buffers are laid out alike (every array of buffer 1 at one
  // distance from its twin in buffer 0)
  for (int b = 0; b < 2; ++b) {
    for (int a = 0; a < 6; ++a) L.soa[b][a] = take((slots + sn) * sizeof(double));
    L.soa[b][6] = take((slots + sn) * sizeof(uint32_t));
    L.count[b] = take(cc * sizeof(uint32_t));
    L.spill_desc[b] = take(sizeof(SpillDesc));
    L.spill_cell[b] = take(sn * sizeof(uint32_t));
    L.spill_ocell[b] = take(cc * sizeof(uint32_t));
    L.spill_hdr[b] = take(kSpillHdrWords * sizeof(uint32_t));
  }
  L.pool_words = (uint64_t)sn * 3u + 3u * cc + 64u;
  L.pool_desc = take(sizeof(OverflowPool));
  L.pool = take((size_t)L.pool_words * sizeof(uint32_t));
  L.pool_hdr = take(2 * sizeof(unsigned long long));
  L.offsets = take((cc + 1) * sizeof(uint32_t));
  L.tile_sums = take(tiles * sizeof(uint32_t));
  L.cell_sums = take(cc * kCellSums * sizeof(double));
  L.consts = take(sizeof(DeviceConsts));
  L.total = off;
  return L;
}

// Validated problem constants (same formulas as the determinism contract).
struct Derived {
  Geometry g;
  double vcell, kfac, vol;
  double sr;  // sigma / r_test
  int64_t n_cells;
  uint32_t cap;
};

// Default slots per cell: twice the mean occupancy plus 32, rounded up to
// 32 (a Poisson cell exceeds it rarely; one that does keeps its surplus in
// spill slots and takes the slower overflow path).
uint32_t default_capacity(int64_t n, int64_t n_cells) {
  const double mean = n_cells > 0 ? (double)n / (double)n_cells : 0.0;
  double cap = std::ceil((2.0 * mean + 32.0) / 32.0) * 32.0;
  if (cap > (double)kCellCap) cap = (double)kCellCap;
  return (uint32_t)cap;
}

int derive(const cuba_params *p, int64_t n, Derived &d) {
  if (!p) return fail(CUBA_EINVAL, "params is NULL");
  int64_t nc = 1;
  for (int k = 0; k < 3; ++k) {
    if (!(std::isfinite(p->box[k]) && p->box[k] > 0.0))
      return fail(CUBA_EINVAL, "box edges must be finite and > 0");
    if (p->cells[k] < 1) return fail(CUBA_EINVAL, "cells must be >= 1");
    nc *= p->cells[k];
  }
  if (nc >= ((int64_t)1 << 31)) return fail(CUBA_EINVAL, "too many cells (>= 2^31)");
  if (!(std::isfinite(p->sigma) && p->sigma >= 0.0))
    return fail(CUBA_EINVAL, "sigma must be finite and >= 0");
  if (!(std::isfinite(p->r_test) && p->r_test > 0.0))
    return fail(CUBA_EINVAL, "r_test must be finite and > 0");
  if (!(std::isfinite(p->dt) && p->dt > 0.0))
    return fail(CUBA_EINVAL, "dt must be finite and > 0");
  for (int k = 0; k < 3; ++k) {
    d.g.L[k] = p->box[k];
    d.g.n[k] = p->cells[k];
    d.g.dx[k] = p->box[k] / (double)p->cells[k];
    // Sec. 5: dt below the cell edge, so a particle moves at most one cell
    if (!(p->dt < d.g.dx[k])) return fail(CUBA_EINVAL, "dt must be below every cell edge");
  }
  d.g.dt = p->dt;
  d.vcell = (d.g.dx[0] * d.g.dx[1]) * d.g.dx[2];
  d.sr = p->sigma / p->r_test;
  d.kfac = (d.sr * p->dt) / d.vcell;
  if (!(2.0 * d.kfac <= 1.0))
    return fail(CUBA_EINVAL, "sigma / r_test * dt / V_cell > 1/2: P22 could exceed 1");
  d.vol = ((p->r_test * d.g.dx[0]) * p->box[1]) * p->box[2];
  d.n_cells = nc;
  if (p->cell_capacity < 0 || p->cell_capacity > (int32_t)kCellCap)
    return fail(CUBA_EINVAL, "cell_capacity must be in [0, " + std::to_string(kCellCap) + "]");
  d.cap = p->cell_capacity == 0 ? default_capacity(n, nc) : (uint32_t)p->cell_capacity;
  // slots (blocks, then spill slots) are addressed with 32-bit indices
  if ((uint64_t)nc * d.cap + (uint64_t)(n > 0 ? n : 1) >= ((uint64_t)1 << 32))
    return fail(CUBA_EINVAL, "cells x cell_capacity + n must stay below 2^32 slots");
  return CUBA_OK;
}

// Lanes per cell from the occupancy at init (over[k] = cells holding more
// than 8 << k particles) and the scattering constant K:
//  * one wave per cell for boxes of fewer cells than a few waves per SIMD,
//    whose steps are bound by launch latency, which the second kernel adds to;
//  * on the plain path (plain: not in a batch), packed cells if at most a
//    small fraction of the cells exceed 64 particles and the mean occupancy
//    is at most 8, or at most 12 with 2K >= 1 % (where most pair-test rounds
//    of the fixed-lane kernels hold a pair that passes the filter, and pay
//    for its exact test in the whole wave);
//  * else the smallest group of 8, 16 or 32 lanes that all but a small
//    fraction of the cells fit (64-lane groups lost to one wave per cell
//    in every measured occupancy mix);
//  * else, on the plain path, packed cells if at least a quarter of the
//    cells hold at most 8 particles and few exceed 64: a box of dense and
//    sparse regions;
//  * else one wave per cell.
// Except: on the plain path, a box of fewer cells than the chip has SIMDs,
// most of them holding more than 32 particles, takes two waves per cell (the
// 1-D tube's 100 cells step in 24 instead of 33 us; at 10 000 cells and
// more the second wave's extra work outweighs its parallelism).
constexpr double kOversizeFraction = 2e-3;
constexpr double kSparseFraction = 0.25;
constexpr int64_t kSmallCellsMinCells = 16384;
constexpr int64_t kTwoWaveMaxCells = 1024;
constexpr double kPackedMean = 8.0, kPackedMeanHighK = 12.0, kHighTwoK = 0.01;
uint32_t default_lanes(const uint32_t over[4], int64_t n_cells, int64_t n, double kfac,
                       bool plain) {
  if (plain && n_cells < kTwoWaveMaxCells && 2 * (int64_t)over[2] >= n_cells)
    return kTwoWavesPerCell;
  if (n_cells < kSmallCellsMinCells) return 0;
  const double limit = kOversizeFraction * (double)n_cells;
  const double mean = (double)n / (double)n_cells;
  const bool packable = plain && (double)over[3] <= limit;
  if (packable && (mean <= kPackedMean || (2.0 * kfac >= kHighTwoK && mean <= kPackedMeanHighK)))
    return kPackedCells;
  for (uint32_t k = 0; k < 3; ++k)
    if ((double)over[k] <= limit) return 8u << k;
  if (packable && (double)(n_cells - over[0]) >= kSparseFraction * (double)n_cells)
    return kPackedCells;
  return 0;
}

void destroy_side(SideStream &sd) {
  if (sd.fork) (void)hipEventDestroy(sd.fork);
  if (sd.join) (void)hipEventDestroy(sd.join);
  if (sd.stream) (void)hipStreamDestroy(sd.stream);
  sd = SideStream{};
}

// A non-blocking stream of default priority and two timing-free events.
hipError_t create_side(SideStream &sd) {
  sd = SideStream{};
  hipError_t e = hipStreamCreateWithFlags(&sd.stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&sd.fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&sd.join, hipEventDisableTiming);
  if (e != hipSuccess) destroy_side(sd);
  return e;
}

// Pairs can only be accepted when the Philox high word w1 is below this:
// u >= w1 2^-32 and P22 <= 2 K (1 + 13 eps) < 2 K (1 + 2^-30).
uint64_t w1_limit(double kfac) {
  const double pmax = (2.0 * kfac) * (1.0 + 0x1p-30);
  const double lim = std::ceil(pmax * 0x1p32);
  if (lim >= 0x1p32) return (uint64_t)1 << 32;
  return (uint64_t)lim;
}

}  // namespace

// One timed stage launch: events recorded just before and after it.
struct TimedLaunch {
  int stage;
  hipEvent_t before, after;
};

struct cuba_ctx {
  Derived d;
  PairArgs pa;
  int64_t n;
  uint32_t next_step;
  uint32_t lanes;  // lanes per cell of the cell kernels (valid_cell_lanes)
  uint32_t over[4];  // cells of the initial state holding > 8, 16, 32, 64 particles
  hipStream_t stream;
  DevStatus *status;
  Cells buf[2];
  int cur;
  uint32_t *offsets, *tile_sums;
  double *cell_sums;
  DeviceConsts *consts;  // in the workspace
  bool in_library = false;  // set up by cuba_init_static: not freed by cuba_destroy
  // stage timing (cuba_timing_begin / cuba_timing_end)
  bool timing = false;
  size_t timing_cap = 0;
  uint32_t timing_step_every = 1;  // time every n-th fused-step launch
  uint64_t step_launches = 0;      // fused-step launches since timing began
  std::vector<hipEvent_t> event_pool;
  std::vector<TimedLaunch> timed;
};

namespace {

int check_launch(const char *where) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, where);
  return CUBA_OK;
}

enum Stage { kStageBin = 0, kStageStep, kStageCollide, kStageObserve, kStageOffsets };
static_assert(kStageOffsets + 1 == CUBA_NUM_STAGES, "stage count");

// Runs launch(events) while timing (fused steps: every
// timing_step_every-th one only), else launch(nullptr).  The binning and
// collision stages take the events into their launch (on the kernel's own
// dispatch where it is one kernel: two event packets between launches
// would delay the next one and read a few microseconds above the kernel's
// duration); the other stages are bracketed here.
template <typename F>
void stage(cuba_ctx *c, int which, F &&launch) {
  bool sampled = true;
  if (c->timing && which == kStageStep)
    sampled = c->step_launches++ % c->timing_step_every == 0;
  if (c->timing && sampled && c->timed.size() < c->timing_cap) {
    const size_t k = c->timed.size();
    TimedLaunch t{which, c->event_pool[2 * k], c->event_pool[2 * k + 1]};
    if (which == kStageBin || which == kStageStep || which == kStageCollide) {
      launch(&t);
    } else {
      (void)hipEventRecord(t.before, c->stream);
      launch(&t);
      (void)hipEventRecord(t.after, c->stream);
    }
    c->timed.push_back(t);
  } else {
    launch(nullptr);
  }
}


void drop_timing(cuba_ctx *c) {
  for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
  c->event_pool.clear();
  c->timed.clear();
  c->timing = false;
  c->timing_cap = 0;
  c->timing_step_every = 1;
  c->step_launches = 0;
}

// Device copy of the geometry.
// The oversize-cell launch takes a wave per cell once such cells average
// more than one in 64 (by the initial histogram), else a wave per 64 cells.
uint32_t over_span(const uint32_t over[4], uint32_t lanes, int64_t n_cells) {
  if (lanes == 0 || lanes == kTwoWavesPerCell) return 64;
  const uint32_t k = lanes == 8 ? 0 : lanes == 16 ? 1 : lanes == 32 ? 2 : 3;
  return (int64_t)over[k] * 64 > n_cells ? 1u : 64u;
}

// A new time step for the steps issued after this call (Sec. 6 names a
// variable dt as the next step of the method): validated as at init, then
// K, the w1 filter bound and the device copy of the geometry follow it.
// Nothing changes on an error.
int apply_dt(cuba_ctx *c, double dt) {
  if (!(std::isfinite(dt) && dt > 0.0)) return fail(CUBA_EINVAL, "dt must be finite and > 0");
  for (int k = 0; k < 3; ++k)
    if (!(dt < c->d.g.dx[k])) return fail(CUBA_EINVAL, "dt must be below every cell edge");
  const double kfac = (c->d.sr * dt) / c->d.vcell;
  if (!(2.0 * kfac <= 1.0))
    return fail(CUBA_EINVAL, "sigma / r_test * dt / V_cell > 1/2: P22 could exceed 1");
  launch_store_f64(&c->consts->g.dt, dt, c->stream);
  const int rc = check_launch("dt update");
  if (rc != CUBA_OK) return rc;
  c->d.g.dt = dt;
  c->d.kfac = kfac;
  c->pa.kfac = kfac;
  const uint64_t lim = w1_limit(kfac);
  c->pa.any = lim > 0 ? 1u : 0u;
  c->pa.w1_max = lim > 0 ? (uint32_t)(lim - 1) : 0u;
  return CUBA_OK;
}

StepDevice step_device(const cuba_ctx *c) {
  return StepDevice{&c->consts->g, over_span(c->over, c->lanes, c->d.n_cells)};
}

// The step launch's device arguments, with the stage's timing events.
StepDevice timed_step_device(const cuba_ctx *c, const TimedLaunch *t) {
  StepDevice dev = step_device(c);
  if (t) {
    dev.ev_start = t->before;
    dev.ev_stop = t->after;
  }
  return dev;
}

// nsteps steps: stream + bin into the other buffer, then nsteps - 1 fused
// steps (collide, then stream + bin into the other buffer), then the last
// collisions in place.  With a trace (nsteps = 1) the binning records cells
// and the compact offsets are built before the collisions.
int run_steps(cuba_ctx *c, int32_t nsteps, const TraceArgs *trace_in) {
  if (nsteps <= 0) return CUBA_OK;
  // the oversize-cell kernel follows the small-cell kernel on the same
  // stream: a fork to a second stream and back costs more per step than
  // the overlap gains for a single event (measured on MI355X)
  const SideStream *side = nullptr;
  stage(c, kStageBin, [&](const TimedLaunch *t) {
    launch_stream_bin(c->buf[c->cur], c->buf[c->cur ^ 1], c->d.n_cells, c->lanes, c->d.g,
                      c->status, trace_in ? trace_in->cell : nullptr, c->next_step,
                      c->stream, t ? t->before : nullptr, t ? t->after : nullptr);
  });
  c->cur ^= 1;
  for (int32_t s = 1; s < nsteps; ++s) {
    stage(c, kStageStep, [&](const TimedLaunch *t) {
      launch_step(c->buf[c->cur], c->buf[c->cur ^ 1], true, c->d.n_cells, c->lanes,
                  c->next_step, c->pa, c->d.g, c->status, nullptr, c->stream, side,
                  timed_step_device(c, t));
    });
    c->cur ^= 1;
    c->next_step += 1;
  }
  TraceArgs tr{};
  if (trace_in) {
    tr = *trace_in;
    stage(c, kStageOffsets, [&](const TimedLaunch *) {
      launch_offsets(c->buf[c->cur], const_cast<uint32_t *>(tr.offsets), c->tile_sums,
                     c->d.n_cells, c->stream);
    });
  }
  stage(c, kStageCollide, [&](const TimedLaunch *t) {
    launch_step(c->buf[c->cur], c->buf[c->cur ^ 1], false, c->d.n_cells, c->lanes,
                c->next_step, c->pa, c->d.g, c->status, trace_in ? &tr : nullptr, c->stream,
                side, timed_step_device(c, t));
  });
  c->next_step += 1;
  return check_launch("step launch");
}

}  // namespace

extern "C" {

size_t cuba_capacity_scratch_bytes(const cuba_params *params) {
  Derived d;
  if (derive(params, 0, d) != CUBA_OK) return 0;
  return ((size_t)(d.n_cells + 1) * sizeof(uint32_t) + 255) / 256 * 256;
}

int cuba_suggest_cell_capacity(const cuba_params *params, int64_t n, const double *x,
                               const double *y, const double *z, void *scratch,
                               size_t scratch_bytes, void *stream, int32_t *cap) {
  if (!cap) return fail(CUBA_EINVAL, "cap is NULL");
  if (n < 0 || n >= 0xFFFFFFFFll) return fail(CUBA_EINVAL, "n must be in [0, 2^32 - 1)");
  Derived d;
  const int rc = derive(params, 0, d);
  if (rc != CUBA_OK) return rc;
  if (n > 0 && !(x && y && z)) return fail(CUBA_EINVAL, "position arrays must not be NULL");
  const size_t need = cuba_capacity_scratch_bytes(params);
  if (!scratch || scratch_bytes < need || ((uintptr_t)scratch & 255u) != 0)
    return fail(CUBA_EINVAL, "scratch must be 256-byte aligned and hold "
                             "cuba_capacity_scratch_bytes(params)");
  hipStream_t s = (hipStream_t)stream;
  uint32_t *count = (uint32_t *)scratch;
  uint32_t *max_count = count + d.n_cells;
  launch_count_cells(x, y, z, n, d.g, d.n_cells, count, max_count, s);
  uint32_t m = 0;
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(&m, max_count, sizeof(m), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "cuba_suggest_cell_capacity");
  if (n == 0 || m == 0) {
    *cap = 64;
    return CUBA_OK;
  }
  const uint64_t want = ((2ull * m + 32ull) + 31ull) / 32ull * 32ull;
  *cap = (int32_t)(want < 64ull ? 64ull : want > kCellCap ? (uint64_t)kCellCap : want);
  return CUBA_OK;
}

size_t cuba_workspace_bytes(const cuba_params *params, int64_t n) {
  Derived d;
  if (n < 0 || n >= 0xFFFFFFFFll || derive(params, n, d) != CUBA_OK) return 0;
  return make_layout(d.n_cells, d.cap, n).total;
}

}  // extern "C"

namespace {

// Checks the arguments of cuba_init / cuba_init_static that do not depend
// on the workspace.
int check_init_args(const cuba_params *params, int64_t n, const double *x, const double *y,
                    const double *z, const double *px, const double *py, const double *pz,
                    Derived &d) {
  if (n < 0 || n >= 0xFFFFFFFFll) return fail(CUBA_EINVAL, "n must be in [0, 2^32 - 1)");
  const int rc = derive(params, n, d);
  if (rc != CUBA_OK) return rc;
  if (n > 0 && !(x && y && z && px && py && pz))
    return fail(CUBA_EINVAL, "particle arrays must not be NULL");
  return CUBA_OK;
}

// Sets up the context c (freshly constructed) on the workspace and bins the
// initial state.  The caller frees c on failure, if it owns it.
int init_context(cuba_ctx *c, const Derived &d, const cuba_params *params, int64_t n,
                 const double *x, const double *y, const double *z, const double *px,
                 const double *py, const double *pz, void *workspace, size_t ws_bytes,
                 void *stream, bool validate = true) {
  int rc = CUBA_OK;
  if (!workspace) return fail(CUBA_EINVAL, "workspace is NULL");
  if (((uintptr_t)workspace & 255u) != 0)
    return fail(CUBA_EINVAL, "workspace must be 256-byte aligned");
  const Layout L = make_layout(d.n_cells, d.cap, n);
  if (ws_bytes < L.total)
    return fail(CUBA_ENOMEM, "workspace too small: need " + std::to_string(L.total) +
                                 " bytes, got " + std::to_string(ws_bytes));
  c->d = d;
  c->pa.kfac = d.kfac;
  const uint64_t lim = w1_limit(d.kfac);
  c->pa.any = lim > 0 ? 1u : 0u;
  c->pa.w1_max = lim > 0 ? (uint32_t)(lim - 1) : 0u;
  c->pa.key0 = (uint32_t)(params->seed & 0xFFFFFFFFu);
  c->pa.key1 = (uint32_t)(params->seed >> 32);
  c->n = n;
  c->next_step = params->step0;
  c->stream = (hipStream_t)stream;
  char *ws = (char *)workspace;
  c->status = (DevStatus *)(ws + L.status);
  for (int b = 0; b < 2; ++b) {
    SoA &st = c->buf[b].st;
    st.x = (double *)(ws + L.soa[b][0]);
    st.y = (double *)(ws + L.soa[b][1]);
    st.z = (double *)(ws + L.soa[b][2]);
    st.px = (double *)(ws + L.soa[b][3]);
    st.py = (double *)(ws + L.soa[b][4]);
    st.pz = (double *)(ws + L.soa[b][5]);
    st.id = (uint32_t *)(ws + L.soa[b][6]);
    c->buf[b].count = (uint32_t *)(ws + L.count[b]);
    c->buf[b].cap = d.cap;
    c->buf[b].sp = (SpillDesc *)(ws + L.spill_desc[b]);
  }
  OverflowPool hpool{};
  hpool.buf = (uint32_t *)(ws + L.pool);
  hpool.hdr = (unsigned long long *)(ws + L.pool_hdr);
  hpool.capacity = L.pool_words;
  SpillDesc hsd[2];
  for (int b = 0; b < 2; ++b) {
    hsd[b].cell = (uint32_t *)(ws + L.spill_cell[b]);
    hsd[b].ocell = (uint32_t *)(ws + L.spill_ocell[b]);
    hsd[b].hdr = (uint32_t *)(ws + L.spill_hdr[b]);
    hsd[b].pool = (OverflowPool *)(ws + L.pool_desc);
    hsd[b].base = (uint64_t)d.n_cells * d.cap;
    hsd[b].capacity = n > 0 ? (uint32_t)n : 1u;
    hsd[b].pad = 0;
  }
  // the kernels derive one buffer's arrays from the other's by a single
  // byte distance: every array of buffer 1 lies that far from its twin
  const ptrdiff_t shift = (char *)c->buf[1].st.x - (char *)c->buf[0].st.x;
  for (int a = 0; a < 7; ++a)
    if ((ptrdiff_t)(L.soa[1][a] - L.soa[0][a]) != shift)
      return fail(CUBA_EINVAL, "internal: buffers not laid out alike");
  if ((ptrdiff_t)(L.count[1] - L.count[0]) != shift ||
      (ptrdiff_t)(L.spill_desc[1] - L.spill_desc[0]) != shift)
    return fail(CUBA_EINVAL, "internal: buffers not laid out alike");
  c->offsets = (uint32_t *)(ws + L.offsets);
  c->tile_sums = (uint32_t *)(ws + L.tile_sums);
  c->cell_sums = (double *)(ws + L.cell_sums);
  c->consts = (DeviceConsts *)(ws + L.consts);
  c->cur = 0;
  DeviceConsts hc{};
  hc.g = d.g;

  // clear status and counts, then check and bin the particles
  launch_fill_u32((uint32_t *)c->status, 0u, sizeof(DevStatus) / sizeof(uint32_t),
                  c->stream);
  launch_fill_u32(c->buf[0].count, 0u, d.n_cells, c->stream);
  launch_fill_u32(c->buf[1].count, 0u, d.n_cells, c->stream);
  for (int b = 0; b < 2; ++b) launch_fill_u32(hsd[b].hdr, 0u, kSpillHdrWords, c->stream);
  launch_fill_u32((uint32_t *)hpool.hdr, 0u, 4, c->stream);
  // the constants and (each in its buffer's region, one buffer's distance
  // apart) the two spill descriptors, written by kernels in stream order
  bool ok = launch_write_bytes(c->consts, &hc, sizeof(hc), c->stream);
  ok = ok && launch_write_bytes(hsd[0].pool, &hpool, sizeof(hpool), c->stream);
  for (int b = 0; b < 2; ++b)
    ok = ok && launch_write_bytes(c->buf[b].sp, &hsd[b], sizeof(SpillDesc), c->stream);
  if (!ok) return fail(CUBA_EDEVICE, "internal: constants do not fit a write launch");
  // the initial binning is consumed by the stream-bin of step step0
  launch_init_bin(x, y, z, px, py, pz, c->buf[0], n, d.g, c->status, c->next_step - 1u,
                  c->stream);
  launch_occupancy_over(c->buf[0], d.n_cells, c->status, c->stream);
  rc = check_launch("init launch");
  if (rc != CUBA_OK) return rc;
  if (!validate) {  // errors of the state surface at the next sync
    c->lanes = 0;
    return CUBA_OK;
  }
  hipError_t e = hipSuccess;
  uint32_t head[5] = {0, 0, 0, 0, 0};  // err, over[4]
  static_assert(offsetof(DevStatus, over) == sizeof(uint32_t), "status layout");
  SpillDesc back[2];
  e = hipMemcpyAsync(head, &c->status->err, sizeof(head), hipMemcpyDeviceToHost, c->stream);
  for (int b = 0; b < 2 && e == hipSuccess; ++b)
    e = hipMemcpyAsync(&back[b], c->buf[b].sp, sizeof(SpillDesc), hipMemcpyDeviceToHost,
                       c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(e, "init check");
  for (int b = 0; b < 2; ++b)
    if (std::memcmp(&back[b], &hsd[b], sizeof(SpillDesc)) != 0)
      return fail(CUBA_EDEVICE, "internal: spill descriptor not in place");
  const uint32_t err = head[0];
  for (int k = 0; k < 4; ++k) c->over[k] = head[1 + k];
  c->lanes = default_lanes(c->over, d.n_cells, n, d.kfac, true);
  if (err & kErrRange)
    return fail(CUBA_ERANGE, "a particle is outside [0, L], non-finite, or has |p| = 0");
  if (err & kErrSpill) return fail(CUBA_EDEVICE, "internal: spill region inconsistent");
  return CUBA_OK;
}

// The library's own workspace for cuba_init_static: one array per device
// (each GPU the library runs on holds its copy until the process ends),
// addressed from the host through hipGetSymbolAddress only.  Every call on a
// device reuses that device's array.
constexpr size_t kStaticWorkspaceBytes = CUBA_STATIC_WORKSPACE_BYTES;

}  // namespace

static __device__ __align__(256) char scratch[kStaticWorkspaceBytes];

namespace {

constexpr int kMaxDevices = 64;
struct StaticSlot {
  void *ptr = nullptr;  // device address of `scratch` on this device
  cuba_ctx ctx;         // the context living on it
};
StaticSlot g_static[kMaxDevices];
std::mutex g_static_mu;

// Device address of the current device's `scratch` (looked up once per
// device, with that device current).
int static_workspace(int &dev, void *&ptr) {
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "static workspace: device");
  if (dev < 0 || dev >= kMaxDevices) return fail(CUBA_EDEVICE, "static workspace: device id");
  if (!g_static[dev].ptr) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "static workspace: symbol address");
    g_static[dev].ptr = p;
  }
  ptr = g_static[dev].ptr;
  return CUBA_OK;
}

}  // namespace

extern "C" {

int cuba_init(cuba_ctx **out, const cuba_params *params, int64_t n, const double *x,
              const double *y, const double *z, const double *px, const double *py,
              const double *pz, void *workspace, size_t ws_bytes, void *stream) {
  if (!out) return fail(CUBA_EINVAL, "out is NULL");
  *out = nullptr;
  Derived d;
  int rc = check_init_args(params, n, x, y, z, px, py, pz, d);
  if (rc != CUBA_OK) return rc;
  cuba_ctx *c = new (std::nothrow) cuba_ctx();
  if (!c) return fail(CUBA_ENOMEM, "host allocation failed");
  rc = init_context(c, d, params, n, x, y, z, px, py, pz, workspace, ws_bytes, stream);
  if (rc != CUBA_OK) {
    delete c;
    return rc;
  }
  *out = c;
  return CUBA_OK;
}

int cuba_init_static(cuba_ctx **out, const cuba_params *params, int64_t n, const double *x,
                     const double *y, const double *z, const double *px, const double *py,
                     const double *pz, void *stream) {
  if (!out) return fail(CUBA_EINVAL, "out is NULL");
  *out = nullptr;
  Derived d;
  int rc = check_init_args(params, n, x, y, z, px, py, pz, d);
  if (rc != CUBA_OK) return rc;
  const size_t need = make_layout(d.n_cells, d.cap, n).total;
  if (need > kStaticWorkspaceBytes)
    return fail(CUBA_ENOMEM, "static workspace too small: need " + std::to_string(need) +
                                 " bytes, the library holds " +
                                 std::to_string(kStaticWorkspaceBytes));
  std::lock_guard<std::mutex> lock(g_static_mu);
  int dev = 0;
  void *ws = nullptr;
  rc = static_workspace(dev, ws);
  if (rc != CUBA_OK) return rc;
  cuba_ctx *c = &g_static[dev].ctx;
  drop_timing(c);
  *c = cuba_ctx{};
  c->in_library = true;
  rc = init_context(c, d, params, n, x, y, z, px, py, pz, ws, kStaticWorkspaceBytes, stream);
  if (rc != CUBA_OK) return rc;
  *out = c;
  return CUBA_OK;
}

int cuba_set_cell_lanes(cuba_ctx *c, int32_t lanes) {
  if (!c) return fail(CUBA_EINVAL, "ctx is NULL");
  if (!valid_plain_cell_lanes(lanes))
    return fail(CUBA_EINVAL, "lanes must be 0, 1, 8, 16, 32, 64 or 128");
  c->lanes = (uint32_t)lanes;
  return CUBA_OK;
}

int cuba_get_cell_lanes(const cuba_ctx *c, int32_t *lanes) {
  if (!c || !lanes) return fail(CUBA_EINVAL, "NULL argument");
  *lanes = (int32_t)c->lanes;
  return CUBA_OK;
}

int cuba_set_dt(cuba_ctx *c, double dt) {
  if (!c) return fail(CUBA_EINVAL, "ctx is NULL");
  return apply_dt(c, dt);
}

int cuba_get_dt(const cuba_ctx *c, double *dt) {
  if (!c || !dt) return fail(CUBA_EINVAL, "NULL argument");
  *dt = c->d.g.dt;
  return CUBA_OK;
}

int cuba_step(cuba_ctx *c, int32_t nsteps) {
  if (!c) return fail(CUBA_EINVAL, "ctx is NULL");
  if (nsteps < 0) return fail(CUBA_EINVAL, "nsteps must be >= 0");
  return run_steps(c, nsteps, nullptr);
}

int cuba_trace_step(cuba_ctx *c, const cuba_trace *t) {
  if (!c || !t) return fail(CUBA_EINVAL, "ctx or trace is NULL");
  if (!t->counts) return fail(CUBA_EINVAL, "trace counts is NULL");
  if (t->cand_cap < 0 || t->claim_cap < 0 || t->cand_cap > 0xFFFFFFFFll ||
      t->claim_cap > 0xFFFFFFFFll)
    return fail(CUBA_EINVAL, "trace capacities out of range");
  TraceArgs tr{};
  tr.cell = t->cell;
  tr.perm = t->perm;
  tr.offsets = t->offsets ? t->offsets : c->offsets;
  tr.cand = t->cand;
  tr.cand_cap = (uint32_t)t->cand_cap;
  tr.claim = t->claim;
  tr.claim_cap = (uint32_t)t->claim_cap;
  tr.counts = t->counts;
  launch_fill_u32(t->counts, 0u, 2, c->stream);
  return run_steps(c, 1, &tr);
}

int cuba_observe(cuba_ctx *c, double *T00, double *T0x) {
  if (!c || !T00 || !T0x) return fail(CUBA_EINVAL, "NULL argument");
  const SlabOut out{T00, T0x, nullptr, nullptr, nullptr, nullptr};
  stage(c, kStageObserve, [&](const TimedLaunch *) {
    launch_observe(c->buf[c->cur], c->d.g, c->d.vol, c->cell_sums, out, c->next_step - 1u,
                   c->stream);
  });
  return check_launch("observe launch");
}

int cuba_observe_moments(cuba_ctx *c, double *out) {
  if (!c || !out) return fail(CUBA_EINVAL, "NULL argument");
  const int64_t nx = c->d.g.n[0];
  const SlabOut o{out, out + nx, out + 2 * nx, out + 3 * nx, out + 4 * nx, out + 5 * nx};
  stage(c, kStageObserve, [&](const TimedLaunch *) {
    launch_observe(c->buf[c->cur], c->d.g, c->d.vol, c->cell_sums, o, c->next_step - 1u,
                   c->stream);
  });
  return check_launch("observe launch");
}

int cuba_get_state(cuba_ctx *c, double *x, double *y, double *z, double *px,
                   double *py, double *pz) {
  if (!c) return fail(CUBA_EINVAL, "ctx is NULL");
  if (c->n > 0 && !(x && y && z && px && py && pz))
    return fail(CUBA_EINVAL, "NULL output array");
  launch_gather_by_id(c->buf[c->cur], c->d.n_cells, x, y, z, px, py, pz, c->next_step - 1u,
                      c->stream);
  return check_launch("get_state launch");
}

int cuba_sync(cuba_ctx *c) {
  if (!c) return fail(CUBA_EINVAL, "ctx is NULL");
  uint32_t err = 0;
  hipError_t e = hipMemcpyAsync(&err, &c->status->err, sizeof(err), hipMemcpyDeviceToHost,
                                c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(e, "sync");
  if (err != 0) {
    launch_fill_u32(&c->status->err, 0u, 1, c->stream);
    e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "sync reset");
    if (err & kErrPairIndex)
      return fail(CUBA_ERANGE, "a cell holds more than " + std::to_string(kMaxPairIndexCell) +
                                   " particles: its pair indices exceed the 32-bit counter "
                                   "word of the random-number contract (its collisions "
                                   "were skipped)");
    if (err & kErrSpill) return fail(CUBA_EDEVICE, "internal: spill region inconsistent");
    if (err & kErrTrace) return fail(CUBA_ENOMEM, "trace buffer too small");
    if (err & kErrRange)
      return fail(CUBA_ERANGE, "a particle of the initial state is outside [0, L], "
                               "non-finite, or has |p| = 0");
    return fail(CUBA_ERANGE, "device reported an invalid state");
  }
  return CUBA_OK;
}

int cuba_info(const cuba_ctx *c, uint32_t *next_step, int64_t *n, int64_t *n_cells) {
  if (!c) return fail(CUBA_EINVAL, "ctx is NULL");
  if (next_step) *next_step = c->next_step;
  if (n) *n = c->n;
  if (n_cells) *n_cells = c->d.n_cells;
  return CUBA_OK;
}

int cuba_counters(cuba_ctx *c, uint64_t out[3]) {
  if (!c || !out) return fail(CUBA_EINVAL, "NULL argument");
  static_assert(sizeof(unsigned long long) == sizeof(uint64_t), "counter width");
  std::vector<unsigned long long> h(3 * kCounterSlots);
  hipError_t e = hipMemcpyAsync(h.data(), c->status->pairs, h.size() * sizeof(h[0]),
                                hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(e, "counters");
  for (int k = 0; k < 3; ++k) {
    uint64_t sum = 0;
    for (uint32_t j = 0; j < kCounterSlots; ++j) sum += h[k * kCounterSlots + j];
    out[k] = sum;
  }
  return CUBA_OK;
}

int cuba_timing_begin(cuba_ctx *c, int32_t max_launches) {
  return cuba_timing_begin_sampled(c, max_launches, 1);
}

int cuba_timing_begin_sampled(cuba_ctx *c, int32_t max_launches, int32_t step_every) {
  if (!c || max_launches < 1 || step_every < 1) return fail(CUBA_EINVAL, "bad timing arguments");
  drop_timing(c);
  c->event_pool.resize(2 * (size_t)max_launches);
  for (size_t k = 0; k < c->event_pool.size(); ++k) {
    const hipError_t e = hipEventCreate(&c->event_pool[k]);
    if (e != hipSuccess) {
      c->event_pool.resize(k);
      drop_timing(c);
      return hip_fail(e, "timing events");
    }
  }
  c->timed.reserve((size_t)max_launches);
  c->timing_cap = (size_t)max_launches;
  c->timing_step_every = (uint32_t)step_every;
  c->timing = true;
  return CUBA_OK;
}

int cuba_timing_end(cuba_ctx *c, double stage_ms[CUBA_NUM_STAGES],
                    int64_t stage_launches[CUBA_NUM_STAGES]) {
  if (!c || !stage_ms || !stage_launches) return fail(CUBA_EINVAL, "NULL argument");
  for (int k = 0; k < CUBA_NUM_STAGES; ++k) {
    stage_ms[k] = 0.0;
    stage_launches[k] = 0;
  }
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    drop_timing(c);
    return hip_fail(e, "timing sync");
  }
  for (const TimedLaunch &t : c->timed) {
    float ms = 0.0f;
    e = hipEventElapsedTime(&ms, t.before, t.after);
    if (e != hipSuccess) {
      drop_timing(c);
      return hip_fail(e, "timing elapsed");
    }
    stage_ms[t.stage] += ms;
    stage_launches[t.stage] += 1;
  }
  drop_timing(c);
  return CUBA_OK;
}

void cuba_destroy(cuba_ctx *c) {
  if (!c) return;
  drop_timing(c);
  if (!c->in_library) delete c;
}

const char *cuba_strerror(int code) {
  switch (code) {
    case CUBA_OK: return "CUBA_OK";
    case CUBA_EINVAL: return "CUBA_EINVAL: invalid parameters or arguments";
    case CUBA_ERANGE: return "CUBA_ERANGE: particle state out of range";
    case CUBA_ENOMEM: return "CUBA_ENOMEM: workspace or buffer too small";
    case CUBA_EDEVICE: return "CUBA_EDEVICE: HIP runtime error";
    default: return "unknown cuba error code";
  }
}

const char *cuba_last_error(void) { return g_last_error.c_str(); }

#ifndef CUBA_SOURCE_HASH
#define CUBA_SOURCE_HASH "unknown"
#endif
const char *cuba_build_info(void) { return "sources " CUBA_SOURCE_HASH "; gfx950"; }

}  // extern "C"

// ---------------------------------------------------------------------------
// Batches of independent events
// ---------------------------------------------------------------------------
struct cuba_batch {
  int32_t max_slots = 0;
  hipStream_t stream = nullptr;
  BatchEvent *dev_table = nullptr;  // in the caller's batch workspace
  uint32_t *dev_begin = nullptr;  // kSpaces x max_slots: first unit per event of each work space
  std::vector<cuba_ctx *> slot_ctx;
  std::vector<int32_t> slot_cpi;
  std::vector<uint8_t> slot_active;  // 0: admitted but held out of the steps
  // observation inside runs (cuba_batch_set_observe): interval (0: off),
  // output rows and the caller's output
  std::vector<int32_t> slot_obs_every, slot_obs_rows;
  std::vector<double *> slot_obs_out;
  std::vector<int32_t> table_slots;  // slots in table order
  BatchSpaces spaces{};  // unit counts of the work spaces (device begins in dev_begin)
  SideStream side{};     // library-owned stream for concurrent kernels of a step
  bool dirty = true;
  uint32_t persistent_waves = 0;
  bool use_graphs = false;
  std::map<int32_t, hipGraphExec_t> graphs;
  // graphs replaced while a launch of them may still run: destroyed at the
  // next sync
  std::vector<hipGraphExec_t> stale_graphs;
  // pinned staging of the table uploads (two, used in turn; an event marks
  // when each one's copies have run), so that an upload does not wait for
  // the stream
  void *staging[2] = {nullptr, nullptr};
  hipEvent_t staged[2] = {nullptr, nullptr};
  bool staged_used[2] = {false, false};
  int next_staging = 0;
  // stage timing of direct (non-graph) runs
  bool timing = false;
  size_t timing_cap = 0;
  std::vector<hipEvent_t> event_pool;
  std::vector<TimedLaunch> timed;
  int pending_stage = -1;
};

namespace {

// The observation kernel takes the events along the grid's y dimension,
// which holds at most 65535 workgroups.
constexpr int32_t kMaxBatchSlots = 65535;

// Work spaces of a batch: binning items, small-cell chunks, oversize scans,
// and the one-wave-per-cell spaces of small and large cell capacity.
constexpr int kSpaces = 5;

// Graphs of the old table: set aside (a launch of them may still be in
// flight) and destroyed once the stream has been synchronized.
void drop_graphs(cuba_batch *b) {
  for (auto &kv : b->graphs) b->stale_graphs.push_back(kv.second);
  b->graphs.clear();
}

void destroy_stale_graphs(cuba_batch *b) {
  for (hipGraphExec_t g : b->stale_graphs) (void)hipGraphExecDestroy(g);
  b->stale_graphs.clear();
}

size_t staging_bytes(int32_t max_slots) {
  return align256((size_t)max_slots * sizeof(BatchEvent)) +
         (size_t)kSpaces * max_slots * sizeof(uint32_t);
}

// Frees the batch's own resources (streams, staging) and the batch.
void release_batch(cuba_batch *b) {
  for (int k = 0; k < 2; ++k) {
    if (b->staged[k]) (void)hipEventDestroy(b->staged[k]);
    if (b->staging[k]) (void)hipHostFree(b->staging[k]);
  }
  destroy_side(b->side);
  delete b;
}

void drop_batch_timing(cuba_batch *b) {
  for (hipEvent_t e : b->event_pool) (void)hipEventDestroy(e);
  b->event_pool.clear();
  b->timed.clear();
  b->timing = false;
  b->timing_cap = 0;
}

// Default cells per binning item: enough cells that an item holds about 64
// particles (a full wave), at most 64 cells; events with lanes per cell > 0
// bin 64 cells per item (in groups of 64 / lanes cells).
int32_t default_cpi(const cuba_ctx *c) {
  if (c->lanes > 0) return 64;
  const double mean = c->d.n_cells > 0 ? (double)c->n / (double)c->d.n_cells : 0.0;
  int32_t cpi = mean > 0.0 ? (int32_t)(64.0 / mean) : 64;
  if (cpi < 1) cpi = 1;
  if (cpi > 64) cpi = 64;
  return cpi;
}


// Rebuilds the device table and the work spaces from the live slots (in
// slot order).
int upload_table(cuba_batch *b) {
  std::vector<BatchEvent> host;
  b->table_slots.clear();
  uint64_t items = 0, chunks = 0, scans = 0, cells[2] = {0, 0};
  bool scan_large = false;
  uint32_t obs_nx = 0;
  std::vector<int> cell_space;
  for (int32_t s = 0; s < b->max_slots; ++s) {
    cuba_ctx *c = b->slot_ctx[s];
    if (!c || c->d.n_cells == 0 || !b->slot_active[s]) continue;
    BatchEvent e{};
    e.buf[0] = c->buf[0];
    e.buf[1] = c->buf[1];
    e.g = c->d.g;
    e.pa = c->pa;
    e.status = c->status;
    e.n_cells = (uint32_t)c->d.n_cells;
    e.cpi = (uint32_t)b->slot_cpi[s];
    e.cur = (uint32_t)c->cur;
    e.t = c->next_step;
    e.lanes = c->lanes;
    if (b->slot_obs_every[s] > 0) {
      e.obs_every = (uint32_t)b->slot_obs_every[s];
      e.obs_rows = (uint32_t)b->slot_obs_rows[s];
      e.obs_sums = c->cell_sums;
      e.obs_out = b->slot_obs_out[s];
      e.obs_vol = c->d.vol;
      if ((uint32_t)c->d.g.n[0] > obs_nx) obs_nx = (uint32_t)c->d.g.n[0];
    }
    const int space = c->d.cap <= kSmallCap ? 0 : 1;
    e.item_begin = (uint32_t)items;
    e.chunk_begin = (uint32_t)chunks;
    e.scan_begin = (uint32_t)scans;
    e.cell_begin = (uint32_t)cells[space];
    items += (e.n_cells + e.cpi - 1) / e.cpi;
    if (c->lanes > 0) {
      const uint64_t per = 64 / c->lanes;
      chunks += (e.n_cells + per - 1) / per;
      scans += (e.n_cells + 63) / 64;
      if (space == 1) scan_large = true;
    } else {
      cells[space] += e.n_cells;
    }
    // grid sizes stay below 2^31 workgroups
    if (items >= 0x80000000ull || chunks >= 0x80000000ull || cells[0] >= 0x80000000ull ||
        cells[1] >= 0x80000000ull)
      return fail(CUBA_EINVAL, "too many cells in the batch for one launch");
    cell_space.push_back(c->lanes > 0 ? -1 : space);
    host.push_back(e);
    b->table_slots.push_back(s);
  }
  const size_t ne = host.size();
  const size_t stride = (size_t)b->max_slots;
  b->spaces.item_begin = b->dev_begin;
  b->spaces.chunk_begin = b->dev_begin + stride;
  b->spaces.scan_begin = b->dev_begin + 2 * stride;
  b->spaces.cell_begin[0] = b->dev_begin + 3 * stride;
  b->spaces.cell_begin[1] = b->dev_begin + 4 * stride;
  b->spaces.n_items = (uint32_t)items;
  b->spaces.n_chunks = (uint32_t)chunks;
  b->spaces.n_scans = (uint32_t)scans;
  b->spaces.n_cells[0] = (uint32_t)cells[0];
  b->spaces.n_cells[1] = (uint32_t)cells[1];
  b->spaces.scan_large = scan_large;
  b->spaces.obs_nx = obs_nx;
  if (ne > 0) {
    // an event outside a cells space gets that space's running total (the
    // next event's begin), so the lookup never lands on it
    std::vector<uint32_t> begins(kSpaces * stride, 0u);
    uint32_t run[2] = {0, 0};
    for (size_t i = 0; i < ne; ++i) {
      begins[i] = host[i].item_begin;
      begins[stride + i] = host[i].chunk_begin;
      begins[2 * stride + i] = host[i].scan_begin;
      for (int sp = 0; sp < 2; ++sp) {
        begins[(3 + sp) * stride + i] = run[sp];
        if (cell_space[i] == sp) run[sp] += host[i].n_cells;
      }
    }
    // through pinned staging, in stream order, without waiting for the
    // stream (only for the staging buffer's previous copies, two uploads ago)
    const int k = b->next_staging;
    b->next_staging ^= 1;
    hipError_t e = b->staged_used[k] ? hipEventSynchronize(b->staged[k]) : hipSuccess;
    if (e != hipSuccess) return hip_fail(e, "batch table staging");
    char *const stage = (char *)b->staging[k];
    const size_t begins_at = align256((size_t)b->max_slots * sizeof(BatchEvent));
    std::memcpy(stage, host.data(), ne * sizeof(BatchEvent));
    std::memcpy(stage + begins_at, begins.data(), begins.size() * sizeof(uint32_t));
    e = hipMemcpyAsync(b->dev_table, stage, ne * sizeof(BatchEvent), hipMemcpyHostToDevice,
                       b->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(b->dev_begin, stage + begins_at, begins.size() * sizeof(uint32_t),
                         hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipEventRecord(b->staged[k], b->stream);
    if (e != hipSuccess) return hip_fail(e, "batch table upload");
    b->staged_used[k] = true;
  }
  drop_graphs(b);
  b->dirty = false;
  return CUBA_OK;
}

void batch_between(void *vb, int next) {
  cuba_batch *b = (cuba_batch *)vb;
  if (!b->timing) return;
  // close the launch bracketed by the previous call
  if (b->pending_stage >= 0) {
    (void)hipEventRecord(b->timed.back().after, b->stream);
    b->pending_stage = -1;
  }
  if (next < 0 || b->timed.size() >= b->timing_cap) return;
  const size_t k = b->timed.size();
  TimedLaunch t{next, b->event_pool[2 * k], b->event_pool[2 * k + 1]};
  (void)hipEventRecord(t.before, b->stream);
  b->timed.push_back(t);
  b->pending_stage = next;
}

}  // namespace

extern "C" {

size_t cuba_batch_workspace_bytes(int32_t max_slots) {
  if (max_slots < 1 || max_slots > kMaxBatchSlots) return 0;
  return align256((size_t)max_slots * sizeof(BatchEvent)) +
         align256((size_t)kSpaces * max_slots * sizeof(uint32_t));
}

int cuba_batch_create(cuba_batch **out, int32_t max_slots, void *workspace,
                      size_t ws_bytes, void *stream) {
  if (!out) return fail(CUBA_EINVAL, "out is NULL");
  *out = nullptr;
  if (max_slots < 1 || max_slots > kMaxBatchSlots)
    return fail(CUBA_EINVAL, "max_slots must be in 1 .. 65535");
  if (!workspace || ((uintptr_t)workspace & 255u) != 0)
    return fail(CUBA_EINVAL, "batch workspace must be non-NULL and 256-byte aligned");
  if (ws_bytes < cuba_batch_workspace_bytes(max_slots))
    return fail(CUBA_ENOMEM, "batch workspace too small");
  cuba_batch *b = new (std::nothrow) cuba_batch();
  if (!b) return fail(CUBA_ENOMEM, "host allocation failed");
  b->max_slots = max_slots;
  b->stream = (hipStream_t)stream;
  b->dev_table = (BatchEvent *)workspace;
  b->dev_begin =
      (uint32_t *)((char *)workspace + align256((size_t)max_slots * sizeof(BatchEvent)));
  b->slot_ctx.assign(max_slots, nullptr);
  b->slot_cpi.assign(max_slots, 1);
  b->slot_active.assign(max_slots, 1);
  b->slot_obs_every.assign(max_slots, 0);
  b->slot_obs_rows.assign(max_slots, 0);
  b->slot_obs_out.assign(max_slots, nullptr);
  hipError_t e = create_side(b->side);
  for (int k = 0; k < 2 && e == hipSuccess; ++k) {
    e = hipHostMalloc(&b->staging[k], staging_bytes(max_slots), hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->staged[k], hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    release_batch(b);
    return hip_fail(e, "batch side stream and staging");
  }
  *out = b;
  return CUBA_OK;
}

int cuba_batch_admit_async(cuba_batch *b, int32_t slot, const cuba_params *params, int64_t n,
                           const double *x, const double *y, const double *z,
                           const double *px, const double *py, const double *pz,
                           void *workspace, size_t ws_bytes, int32_t lanes) {
  if (!b) return fail(CUBA_EINVAL, "batch is NULL");
  if (slot < 0 || slot >= b->max_slots) return fail(CUBA_EINVAL, "slot out of range");
  if (b->slot_ctx[slot]) return fail(CUBA_EINVAL, "slot is occupied");
  if (!valid_cell_lanes(lanes)) return fail(CUBA_EINVAL, "lanes must be 0, 8, 16, 32 or 64");
  Derived d;
  int rc = check_init_args(params, n, x, y, z, px, py, pz, d);
  if (rc != CUBA_OK) return rc;
  cuba_ctx *c = new (std::nothrow) cuba_ctx();
  if (!c) return fail(CUBA_ENOMEM, "host allocation failed");
  rc = init_context(c, d, params, n, x, y, z, px, py, pz, workspace, ws_bytes,
                    (void *)b->stream, false);
  if (rc != CUBA_OK) {
    delete c;
    return rc;
  }
  c->lanes = (uint32_t)lanes;
  b->slot_ctx[slot] = c;
  b->slot_cpi[slot] = default_cpi(c);
  b->slot_active[slot] = 1;
  b->dirty = true;
  return CUBA_OK;
}

int cuba_batch_admit(cuba_batch *b, int32_t slot, const cuba_params *params, int64_t n,
                     const double *x, const double *y, const double *z, const double *px,
                     const double *py, const double *pz, void *workspace,
                     size_t ws_bytes) {
  if (!b) return fail(CUBA_EINVAL, "batch is NULL");
  if (slot < 0 || slot >= b->max_slots) return fail(CUBA_EINVAL, "slot out of range");
  if (b->slot_ctx[slot]) return fail(CUBA_EINVAL, "slot is occupied");
  cuba_ctx *c = nullptr;
  const int rc = cuba_init(&c, params, n, x, y, z, px, py, pz, workspace, ws_bytes,
                           (void *)b->stream);
  if (rc != CUBA_OK) return rc;
  // a batch steps the oversize cells of an event 64 to a wave
  c->lanes = default_lanes(c->over, c->d.n_cells, c->n, c->d.kfac, false);
  b->slot_ctx[slot] = c;
  b->slot_cpi[slot] = default_cpi(c);
  b->slot_active[slot] = 1;
  b->dirty = true;
  return CUBA_OK;
}

int cuba_batch_set_active(cuba_batch *b, int32_t slot, int32_t active) {
  if (!b || slot < 0 || slot >= b->max_slots || !b->slot_ctx[slot])
    return fail(CUBA_EINVAL, "slot is not occupied");
  const uint8_t a = active != 0 ? 1 : 0;
  if (b->slot_active[slot] != a) {
    b->slot_active[slot] = a;
    b->dirty = true;
  }
  return CUBA_OK;
}

int cuba_batch_retire(cuba_batch *b, int32_t slot) {
  if (!b) return fail(CUBA_EINVAL, "batch is NULL");
  if (slot < 0 || slot >= b->max_slots || !b->slot_ctx[slot])
    return fail(CUBA_EINVAL, "slot is not occupied");
  // the event's device state is the caller's workspace; its host context
  // is not read by work already queued on the stream
  cuba_destroy(b->slot_ctx[slot]);
  b->slot_ctx[slot] = nullptr;
  b->slot_obs_every[slot] = 0;
  b->slot_obs_rows[slot] = 0;
  b->slot_obs_out[slot] = nullptr;
  b->dirty = true;
  return CUBA_OK;
}

int cuba_batch_set_observe(cuba_batch *b, int32_t slot, int32_t every, double *out,
                           int32_t rows) {
  if (!b || slot < 0 || slot >= b->max_slots || !b->slot_ctx[slot])
    return fail(CUBA_EINVAL, "slot is not occupied");
  if (every < 0) return fail(CUBA_EINVAL, "every must be >= 0");
  if (every > 0 && (!out || rows < 1))
    return fail(CUBA_EINVAL, "an observing slot needs an output of at least one row");
  b->slot_obs_every[slot] = every;
  b->slot_obs_rows[slot] = every > 0 ? rows : 0;
  b->slot_obs_out[slot] = every > 0 ? out : nullptr;
  b->dirty = true;
  return CUBA_OK;
}

cuba_ctx *cuba_batch_slot(cuba_batch *b, int32_t slot) {
  if (!b || slot < 0 || slot >= b->max_slots) return nullptr;
  return b->slot_ctx[slot];
}

int cuba_batch_set_cells_per_item(cuba_batch *b, int32_t slot, int32_t cells) {
  if (!b || slot < 0 || slot >= b->max_slots || !b->slot_ctx[slot])
    return fail(CUBA_EINVAL, "slot is not occupied");
  if (cells < 1 || cells > 4096) return fail(CUBA_EINVAL, "cells per item out of range");
  b->slot_cpi[slot] = cells;
  b->dirty = true;
  return CUBA_OK;
}

int cuba_batch_observe(cuba_batch *b, int32_t slot, double *T00, double *T0x) {
  if (!b || slot < 0 || slot >= b->max_slots || !b->slot_ctx[slot])
    return fail(CUBA_EINVAL, "slot is not occupied");
  return cuba_observe(b->slot_ctx[slot], T00, T0x);
}

int cuba_batch_observe_moments(cuba_batch *b, int32_t slot, double *out) {
  if (!b || slot < 0 || slot >= b->max_slots || !b->slot_ctx[slot])
    return fail(CUBA_EINVAL, "slot is not occupied");
  return cuba_observe_moments(b->slot_ctx[slot], out);
}

int cuba_batch_set_cell_lanes(cuba_batch *b, int32_t slot, int32_t lanes) {
  if (!b || slot < 0 || slot >= b->max_slots || !b->slot_ctx[slot])
    return fail(CUBA_EINVAL, "slot is not occupied");
  if (!valid_cell_lanes(lanes)) return fail(CUBA_EINVAL, "lanes must be 0, 8, 16, 32 or 64");
  b->slot_ctx[slot]->lanes = (uint32_t)lanes;
  b->dirty = true;
  return CUBA_OK;
}

int cuba_batch_set_dt(cuba_batch *b, int32_t slot, double dt) {
  if (!b || slot < 0 || slot >= b->max_slots || !b->slot_ctx[slot])
    return fail(CUBA_EINVAL, "slot is not occupied");
  const int rc = apply_dt(b->slot_ctx[slot], dt);
  if (rc != CUBA_OK) return rc;
  b->dirty = true;
  return CUBA_OK;
}

int cuba_batch_set_launch(cuba_batch *b, int32_t persistent_waves, int32_t use_graphs) {
  if (!b || persistent_waves < 0) return fail(CUBA_EINVAL, "bad launch settings");
  if (use_graphs && b->stream == nullptr)
    return fail(CUBA_EINVAL, "graph capture needs a non-null stream");
  b->persistent_waves = (uint32_t)persistent_waves;
  b->use_graphs = use_graphs != 0;
  drop_graphs(b);
  return CUBA_OK;
}

int cuba_batch_step(cuba_batch *b, int32_t nsteps) {
  if (!b) return fail(CUBA_EINVAL, "batch is NULL");
  if (nsteps < 0) return fail(CUBA_EINVAL, "nsteps must be >= 0");
  if (nsteps == 0) return CUBA_OK;
  if (b->dirty) {
    const int rc = upload_table(b);
    if (rc != CUBA_OK) return rc;
  }
  const uint32_t n_events = (uint32_t)b->table_slots.size();
  if (n_events > 0) {
    if (b->use_graphs && !b->timing) {
      auto it = b->graphs.find(nsteps);
      if (it == b->graphs.end()) {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "graph capture begin");
        launch_batch_run(b->dev_table, b->spaces, n_events, nsteps, b->persistent_waves,
                         b->stream, &b->side, nullptr, nullptr);
        e = hipStreamEndCapture(b->stream, &graph);
        if (e != hipSuccess) return hip_fail(e, "graph capture end");
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return hip_fail(e, "graph instantiate");
        it = b->graphs.emplace(nsteps, exec).first;
      }
      const hipError_t e = hipGraphLaunch(it->second, b->stream);
      if (e != hipSuccess) return hip_fail(e, "graph launch");
    } else {
      // the launches after which an event observes (direct launches only)
      std::vector<uint8_t> obs_at;
      if (b->spaces.obs_nx > 0) {
        obs_at.assign((size_t)nsteps + 1, 0);
        for (int32_t s : b->table_slots) {
          const int32_t every = b->slot_obs_every[s];
          if (every <= 0) continue;
          const uint32_t t0 = b->slot_ctx[s]->next_step;
          // launch j collides step t0 + j - 1, due when (t0 + j) % every == 0
          for (uint64_t j = every - t0 % (uint32_t)every; j <= (uint64_t)nsteps; j += every)
            obs_at[j] = 1;
        }
      }
      launch_batch_run(b->dev_table, b->spaces, n_events, nsteps, b->persistent_waves,
                       b->stream, &b->side, b->timing ? batch_between : nullptr, b,
                       obs_at.empty() ? nullptr : obs_at.data());
      const int rc = check_launch("batch run launch");
      if (rc != CUBA_OK) return rc;
    }
  }
  for (int32_t s : b->table_slots) {
    cuba_ctx *c = b->slot_ctx[s];
    c->cur ^= (nsteps & 1);
    c->next_step += (uint32_t)nsteps;
  }
  return CUBA_OK;
}

int cuba_batch_sync(cuba_batch *b, int32_t *bad_slot) {
  if (!b) return fail(CUBA_EINVAL, "batch is NULL");
  if (bad_slot) *bad_slot = -1;
  const hipError_t e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return hip_fail(e, "batch sync");
  destroy_stale_graphs(b);
  for (int32_t s = 0; s < b->max_slots; ++s) {
    if (!b->slot_ctx[s]) continue;
    const int rc = cuba_sync(b->slot_ctx[s]);
    if (rc != CUBA_OK) {
      if (bad_slot) *bad_slot = s;
      g_last_error = "slot " + std::to_string(s) + ": " + g_last_error;
      return rc;
    }
  }
  return CUBA_OK;
}

int cuba_batch_timing_begin(cuba_batch *b, int32_t max_launches) {
  if (!b || max_launches < 1) return fail(CUBA_EINVAL, "bad timing arguments");
  drop_batch_timing(b);
  b->event_pool.resize(2 * (size_t)max_launches);
  for (size_t k = 0; k < b->event_pool.size(); ++k) {
    const hipError_t e = hipEventCreate(&b->event_pool[k]);
    if (e != hipSuccess) {
      b->event_pool.resize(k);
      drop_batch_timing(b);
      return hip_fail(e, "timing events");
    }
  }
  b->timing_cap = (size_t)max_launches;
  b->timing = true;
  b->pending_stage = -1;
  return CUBA_OK;
}

int cuba_batch_timing_end(cuba_batch *b, double stage_ms[CUBA_NUM_STAGES],
                          int64_t stage_launches[CUBA_NUM_STAGES]) {
  if (!b || !stage_ms || !stage_launches) return fail(CUBA_EINVAL, "NULL argument");
  for (int k = 0; k < CUBA_NUM_STAGES; ++k) {
    stage_ms[k] = 0.0;
    stage_launches[k] = 0;
  }
  hipError_t e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) {
    drop_batch_timing(b);
    return hip_fail(e, "timing sync");
  }
  for (const TimedLaunch &t : b->timed) {
    float ms = 0.0f;
    e = hipEventElapsedTime(&ms, t.before, t.after);
    if (e != hipSuccess) {
      drop_batch_timing(b);
      return hip_fail(e, "timing elapsed");
    }
    stage_ms[t.stage] += ms;
    stage_launches[t.stage] += 1;
  }
  drop_batch_timing(b);
  return CUBA_OK;
}

void cuba_batch_destroy(cuba_batch *b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  (void)hipStreamSynchronize(b->side.stream);
  drop_graphs(b);
  destroy_stale_graphs(b);
  drop_batch_timing(b);
  for (cuba_ctx *c : b->slot_ctx) cuba_destroy(c);
  release_batch(b);
}

}  // extern "C"
