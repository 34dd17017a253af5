// internal.hpp -- host-side view of the workspace and the kernel launchers
// shared by the C-ABI layer (api.hip) and the kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "device.hpp"

namespace cuba {

constexpr uint32_t kCellCap = 1024;  // = CUBA_MAX_CELL_OCCUPANCY
constexpr uint32_t kSmallCap = 512;  // cell kernels with half the LDS
constexpr uint32_t kScanTile = 2048; // counts per scan tile

// Device-side error bits, accumulated until the next cuba_sync.
constexpr uint32_t kErrSpill = 1u;      // internal: the spill region filled (cannot happen:
                                        // it holds every particle of the context)
constexpr uint32_t kErrTrace = 2u;      // trace buffer too small
constexpr uint32_t kErrRange = 4u;      // invalid initial particle
constexpr uint32_t kErrPairIndex = 8u;  // a cell too full for the 32-bit pair index
                                        // (its collisions were skipped)

// Most particles a cell may hold: its pair indices k < n (n - 1) / 2 must
// fit the 32-bit counter word of the random-number contract (they do up to
// 92 682; the bound is kept one lower, where the oracle puts it).
constexpr uint32_t kMaxPairIndexCell = 92681u;

// Structure-of-arrays particle state (FP64 position and momentum, u32 id).
struct SoA {
  double *x, *y, *z, *px, *py, *pz;
  uint32_t *id;
};

// Where a buffer keeps the particles its cells could not hold.  Every array
// of a buffer has n_cells * cap block slots followed by `capacity` spill
// slots: cell c owns block slots [c cap, c cap + min(count[c], cap)), and a
// cell that receives more (count[c] > cap, an overflowing cell) keeps the
// surplus in spill slots, each tagged with its cell, the cell itself listed
// once in ocell.  The spill slots hold every particle of the context, so no
// binning can lose one.  Counters come in two sets, used by alternate
// binnings of the buffer (set (b >> 1) & 1 for the binning of step b): a
// launch that consumes one set clears the other, which no launch uses then.
// In device memory beside the buffer's arrays (kernels load it only on the
// rare paths that touch it).
struct OverflowPool;
struct SpillDesc {
  uint32_t *cell;   // the cell of each spilled particle
  uint32_t *ocell;  // the overflowing cells, in the order they overflowed
  uint32_t *hdr;    // per set q: [2q] spilled particles, [2q + 1] overflowing cells
  OverflowPool *pool;  // scratch for stepping overflowing cells
  uint64_t base;    // first spill slot: n_cells * cap
  uint32_t capacity;
  uint32_t pad;
};
constexpr uint32_t kSpillHdrWords = 4;
__host__ __device__ inline uint32_t spill_set(uint32_t binning_step) {
  return (binning_step >> 1) & 1u;
}

// A binned state with a fixed capacity per cell (see SpillDesc).
struct Cells {
  SoA st;
  uint32_t *count;
  uint32_t cap;
  SpillDesc *sp;
};

// Scratch of the kernels stepping overflowing cells: the spilled members'
// slots of each such cell, and for cells larger than the LDS holds their
// canonical order, claimed flags and claims, allocated from `buf` by a
// counter: counter t & 1 serves the collisions of step t (the launch of
// step t clears counter (t + 1) & 1, last used two launches before).
struct OverflowPool {
  uint32_t *buf;
  unsigned long long *hdr;  // [2] counters
  uint64_t capacity;        // u32 words
};

// Device-resident bookkeeping at the head of the workspace.  The work
// counters are spread over kCounterSlots slots (by cell) so that the
// per-cell atomics of the collision kernel do not contend on one address.
constexpr uint32_t kCounterSlots = 256;
struct DevStatus {
  uint32_t err;
  uint32_t over[4];  // cells holding more than 8, 16, 32, 64 particles (filled at init)
  uint32_t pad[59];
  unsigned long long pairs[kCounterSlots];   // pair tests
  unsigned long long cand[kCounterSlots];    // pairs with u < P22
  unsigned long long claims[kCounterSlots];  // scatterings
};

struct TraceArgs {
  uint32_t *cell;     // [n] by id
  uint32_t *perm;     // [n]
  const uint32_t *offsets;  // [C+1] compact offsets of the traced binning
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

// One event of a batch as the batched kernels see it (device table).
struct BatchEvent {
  Cells buf[2];
  Geometry g;
  PairArgs pa;
  DevStatus *status;
  uint32_t n_cells;
  uint32_t cpi;         // cells per work item
  uint32_t item_begin;  // first work item of this event
  uint32_t cur;         // buffer holding the state at the start of a run
  uint32_t t;           // step index of the next step
  uint32_t lanes;       // lanes per cell (0: one wave per cell; 8, 16, 32, 64)
  uint32_t chunk_begin; // first small-cell chunk (64 / lanes cells), if lanes > 0
  uint32_t scan_begin;  // first oversize-cell scan unit (64 cells), if lanes > 0
  uint32_t cell_begin;  // first unit in its one-wave-per-cell space, if lanes = 0
                        // (space 0: cell capacity <= kSmallCap, space 1: larger)
  // observation inside runs: after each step s with (s + 1) % obs_every == 0
  // (obs_every > 0), the collision launch writes the per-cell sums into
  // obs_sums and a slab launch writes T00 and T0x into row
  // ((s + 1) / obs_every) % obs_rows of obs_out (rows of 2 nx doubles)
  uint32_t obs_every;
  uint32_t obs_rows;
  uint32_t pad;
  double *obs_sums;
  double *obs_out;
  double obs_vol;       // slab volume
};

// The work spaces of a batch run (see launch_batch_run): unit counts and,
// per event in table order, the first unit of each space (device arrays).
struct BatchSpaces {
  const uint32_t *item_begin, *chunk_begin, *scan_begin, *cell_begin[2];
  uint32_t n_items, n_chunks, n_scans, n_cells[2];
  bool scan_large;  // some small-cell event has a cell capacity > kSmallCap
  uint32_t obs_nx;  // > 0: some event observes inside runs; its largest nx
};

// Lanes per cell of the cell kernels: 0 (one wave per cell), 8, 16, 32, 64
// (64 / lanes cells per wave, one particle per lane; larger cells stepped by
// a whole wave), kPackedCells (whole cells packed into waves of up to 64
// particles, one per lane; plain path only) or kTwoWavesPerCell (a
// workgroup of two waves per cell; plain path only).
constexpr uint32_t kPackedCells = 1;
constexpr uint32_t kTwoWavesPerCell = 128;
inline bool valid_cell_lanes(int32_t v) {
  return v == 0 || v == 8 || v == 16 || v == 32 || v == 64;
}
inline bool valid_plain_cell_lanes(int32_t v) {
  return valid_cell_lanes(v) || v == (int32_t)kTwoWavesPerCell ||
         v == (int32_t)kPackedCells;
}

// A second stream on which a step runs work that is independent of the
// work on the main stream (fork: main -> side, join: side -> main).
struct SideStream {
  hipStream_t stream;
  hipEvent_t fork, join;
};

// Launchers (kernels.hip).  All asynchronous on stream s.
void launch_fill_u32(uint32_t *p, uint32_t v, int64_t count, hipStream_t s);
// *p = v on the device, in stream order.
void launch_store_f64(double *p, double v, hipStream_t s);
// Copies `bytes` (a multiple of 4, at most 256) from host memory to dst on
// the device in stream order, the data travelling as a kernel argument (so
// the call neither waits for the stream nor needs src after it returns).
// False if the size or alignment does not fit.
bool launch_write_bytes(void *dst, const void *src, size_t bytes, hipStream_t s);
// Counts the particles of each cell (count: n_cells words, zeroed here)
// and the largest count into *max_count (zeroed here); non-finite positions
// are skipped.
void launch_count_cells(const double *x, const double *y, const double *z, int64_t n,
                        const Geometry &g, int64_t n_cells, uint32_t *count,
                        uint32_t *max_count, hipStream_t s);
// Validates and bins the id-ordered initial state into dst; the binning is
// that of step `binning_step` (step0 - 1: the stream-bin of step0 consumes
// it).
void launch_init_bin(const double *x, const double *y, const double *z,
                     const double *px, const double *py, const double *pz,
                     const Cells &dst, int64_t n, const Geometry &g, DevStatus *st,
                     uint32_t binning_step, hipStream_t s);
// Stream + bin every particle of src (the binning of step t - 1) into dst
// (the binning of step t), spilled ones included; ev_start / ev_stop: stage
// timing events recorded on the kernel's dispatch, or null.
void launch_stream_bin(const Cells &src, const Cells &dst, int64_t n_cells, uint32_t lanes,
                       const Geometry &g, DevStatus *status, uint32_t *trace_cell,
                       uint32_t t, hipStream_t s, hipEvent_t ev_start = nullptr,
                       hipEvent_t ev_stop = nullptr);
void launch_offsets(const Cells &cur, uint32_t *offsets, uint32_t *tile_sums,
                    int64_t n_cells, hipStream_t s);
// Device copy of the geometry, which the wave-per-cell kernel reads from
// memory where it uses it.
struct StepDevice {
  const Geometry *g;
  // cells per wave of the oversize-cell kernel: 64 (a wave scans 64 cells
  // and steps the oversize ones one after another; few oversize cells) or 1
  // (a wave per cell; many)
  uint32_t over_span;
  // stage timing: events that the launch records at its start and end (on
  // its first kernel's dispatch when it is one kernel), or null
  hipEvent_t ev_start = nullptr, ev_stop = nullptr;
};

// One collision launch (fused: then streaming + binning of the next step).
// lanes > 0: the small-cell kernel on s and, concurrently on side (if not
// NULL; else after it on s), the kernel for the cells it leaves alone
// (overflowing cells among them).
// dev: device copy of g (equal to the host value).  The buffers src and
// dst must be laid out alike (every array at the same distance from its twin).
void launch_step(const Cells &src, const Cells &dst, bool fused, int64_t n_cells,
                 uint32_t lanes, uint32_t t, const PairArgs &pa, const Geometry &g, DevStatus *status,
                 const TraceArgs *trace, hipStream_t s, const SideStream *side,
                 const StepDevice &dev);
// Counts the cells of cur holding more than 8, 16, 32 and 64 particles into
// status->over (which must be zero).
void launch_occupancy_over(const Cells &cur, int64_t n_cells, DevStatus *status, hipStream_t s);
// Per-slab outputs of an observation (each may be NULL): T00, T0x, Txx
// [GeV/fm^3], density n [fm^-3], rest-frame e [GeV/fm^3] and v.
struct SlabOut {
  double *T00, *T0x, *Txx, *n, *e, *v;
};
constexpr uint32_t kCellSums = 4;  // per cell: sum E, sum p_x, sum p_x^2 / E, count
// cell_sums: scratch of kCellSums doubles per cell.  cur holds the binning
// of step binning_step.
void launch_observe(const Cells &cur, const Geometry &g, double vol, double *cell_sums,
                    const SlabOut &out, uint32_t binning_step, hipStream_t s);
// A run of k >= 1 steps of every event in the device table ev (n_events
// live events): stream + bin, k - 1 fused steps, the last collisions, then
// the table advance.  The work spaces: items of cells_per_item cells for the
// binning (every event); for events with lanes per cell > 0, small-cell
// chunks of 64 / lanes cells and scan units of 64 cells for their oversize
// cells; for events with lanes = 0, one unit per cell, in two spaces by cell
// capacity (<= kSmallCap and larger), each stepped by the kernel with the
// LDS for its capacity, so that one large event does not lower the
// occupancy of all the others.  persistent_waves
// > 0 caps the binning grid (persistent waves taking items with a grid
// stride).  Each step runs the small-cell chunks on s and, concurrently on
// side (if not NULL), the one-wave-per-cell events and the oversize cells.
// between (may be NULL) is called before each step of the run with
// its kind (0 stream-bin, 1 fused step, 2 collide) and with -1 after the last
// one: a hook for stage timing.
// obs_at (may be NULL): obs_at[j] != 0 for the launches j after which some
// event of the run is due for an observation inside the run (NULL: the
// observation launch follows every launch while spaces.obs_nx > 0, as a
// graph captured once for many runs needs).
void launch_batch_run(BatchEvent *ev, const BatchSpaces &spaces, uint32_t n_events, int32_t k,
                      uint32_t persistent_waves, hipStream_t s, const SideStream *side,
                      void (*between)(void *, int), void *ctx,
                      const uint8_t *obs_at = nullptr);
void launch_gather_by_id(const Cells &cur, int64_t n_cells, double *x, double *y,
                         double *z, double *px, double *py, double *pz,
                         uint32_t binning_step, hipStream_t s);

}  // namespace cuba
