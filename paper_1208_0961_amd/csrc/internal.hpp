// internal.hpp -- host-side view of the workspace and the kernel launchers
// shared by the C-ABI layer (api.hip) and the kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "device.hpp"

namespace cuba {

constexpr uint32_t kCellCap = 1024;  // = CUBA_MAX_CELL_OCCUPANCY
constexpr uint32_t kScanTile = 2048; // counts per scan tile
constexpr uint32_t kObsChunks = 16;  // partial sums per slab in the observe pass

// Device-side error bits, accumulated until the next cuba_sync.
constexpr uint32_t kErrOccupancy = 1u;  // a cell over kCellCap
constexpr uint32_t kErrTrace = 2u;      // trace buffer too small
constexpr uint32_t kErrRange = 4u;      // invalid initial particle

// Structure-of-arrays particle state (FP64 position and momentum, u32 id).
struct SoA {
  double *x, *y, *z, *px, *py, *pz;
  uint32_t *id;
};

// Device-resident bookkeeping at the head of the workspace.  The work
// counters are spread over kCounterSlots slots (by cell) so that the
// per-cell atomics of the collision kernel do not contend on one address.
constexpr uint32_t kCounterSlots = 256;
struct DevStatus {
  uint32_t err;
  uint32_t pad[63];
  unsigned long long pairs[kCounterSlots];   // pair tests
  unsigned long long cand[kCounterSlots];    // pairs with u < P22
  unsigned long long claims[kCounterSlots];  // scatterings
};

struct TraceArgs {
  uint32_t *cell;     // [n] by id
  uint32_t *perm;     // [n]
  uint32_t *cand;     // [3 cap]
  uint32_t cand_cap;
  uint32_t *claim;    // [3 cap]
  uint32_t claim_cap;
  uint32_t *counts;   // [2]
};

struct PairArgs {
  double kfac;       // K = sigma / r_test * dt / V_cell
  uint32_t w1_max;   // a pair can be accepted only if its Philox word w1 <= w1_max
  uint32_t any;      // 0 when no pair can be accepted (K = 0)
  uint32_t key0, key1;
};

// Launchers (kernels.hip).  All asynchronous on stream s.
void launch_load(const double *x, const double *y, const double *z,
                 const double *px, const double *py, const double *pz, SoA dst,
                 int64_t n, const Geometry &g, DevStatus *st, hipStream_t s);
void launch_fill_u32(uint32_t *p, uint32_t v, int64_t count, hipStream_t s);
void launch_count(const SoA &src, int64_t n, const Geometry &g, bool stream,
                  uint32_t *counts, hipStream_t s);
void launch_scan(uint32_t *counts, uint32_t *offsets, uint32_t *cursor,
                 uint32_t *tile_sums, int64_t n_cells, hipStream_t s);
void launch_scatter(const SoA &src, SoA dst, int64_t n, const Geometry &g,
                    bool stream, uint32_t *cursor, uint32_t *trace_cell,
                    hipStream_t s);
void launch_collide(const uint32_t *offsets, SoA st, int64_t n_cells,
                    uint32_t t, const PairArgs &pa, DevStatus *status,
                    const TraceArgs *trace, hipStream_t s);
void launch_observe(const uint32_t *offsets, const SoA &st, const Geometry &g,
                    double vol, double *partial, double *T00, double *T0x,
                    hipStream_t s);
void launch_gather_by_id(const SoA &st, int64_t n, double *x, double *y,
                         double *z, double *px, double *py, double *pz,
                         hipStream_t s);

}  // namespace cuba
