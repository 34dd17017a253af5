// kernels.hip -- gfx950 kernels of the PIC Boltzmann step (arXiv:1208.0961).
//
// State layout: two structure-of-arrays buffers with a fixed capacity of
// `cap` slots per cell; cell c owns slots [c cap, c cap + count[c]).  One
// buffer holds the current state, the other receives the next binning.
//
// A step t is stream + reflect + bin (Eq. (2), walls, cells), then the
// collisions of every cell (Eq. (3), claims, CM kinematics).  The kernels:
//   k_stream_bin   one wave per source cell: stream + reflect each particle,
//                  find its new cell, append it there (wave-aggregated slot
//                  atomics, one round trip per wave).       HBM: 52 B + 52 B
//   k_step<F>      one wave per cell: ids to LDS, canonical (id) order by
//                  rank counting, all n(n-1)/2 pair tests over the lanes with
//                  a Philox block each, ballot compaction of the pairs that
//                  can pass, exact Eq. (3) test on those, greedy claim in
//                  pair order, CM kinematics (written back in place, or
//                  with F kept in LDS).  With F (fused) the same wave then
//                  streams and bins its particles for step t+1, so the
//                  binning traffic overlaps the ALU-bound pair tests.
//   k_step_small   64 / G cells per wave, one particle per lane (sparse
//                  cells); k_step_large / k_step_over step the cells that
//                  do not fit G lanes.
//   k_step2        a workgroup of two waves per cell, splitting its pair
//                  tests (boxes of fewer cells than SIMDs).
//   observe        per-cell sums of E, p_x, p_x^2/E and counts, then
//                  fixed-order slab sums.
//   gather         state export by id.
// A run of n steps is one stream_bin, n-1 fused steps and one collide-only
// step, which leaves the state binned and collided (positions of step t+n-1).
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <type_traits>

#include "internal.hpp"

namespace cuba {

namespace {

constexpr int kBlock = 256;
constexpr uint32_t kCellsPerBlock = kBlock / 64;

// Waves per SIMD the one-wave-per-cell kernels are held to: six with the
// LDS of 512-slot cells (80 VGPRs; the rare paths for overflowing cells
// would otherwise raise the count for all), four with that of 1024 (the
// LDS allows no more).
template <uint32_t kCap>
constexpr int cell_waves() {
  return kCap <= kSmallCap ? 6 : 4;
}

// Device views of the particle buffers with global-address-space pointers:
// every kernel converts its Cells once at entry, so that all buffer accesses
// compile to global (not flat) memory instructions, also where the pointers
// are loaded from memory (the batch table) rather than passed as arguments.
template <typename T>
using gptr = __attribute__((address_space(1))) T *;

struct GSoA {
  gptr<double> x, y, z, px, py, pz;
  gptr<uint32_t> id;
};

struct GCells {
  GSoA st;
  gptr<uint32_t> count;
  uint32_t cap;
  SpillDesc *sp;
  uint32_t q;  // the spill counter set of the binning this view holds or receives
};

__device__ __forceinline__ GCells to_global(const Cells &c) {
  GCells g;
  g.st.x = (gptr<double>)c.st.x;
  g.st.y = (gptr<double>)c.st.y;
  g.st.z = (gptr<double>)c.st.z;
  g.st.px = (gptr<double>)c.st.px;
  g.st.py = (gptr<double>)c.st.py;
  g.st.pz = (gptr<double>)c.st.pz;
  g.st.id = (gptr<uint32_t>)c.st.id;
  g.count = (gptr<uint32_t>)c.count;
  g.cap = c.cap;
  g.sp = c.sp;
  g.q = 0u;
  return g;
}

// The view of a buffer holding (or receiving) the binning of step b.
__device__ __forceinline__ GCells binning(GCells c, uint32_t b) {
  c.q = spill_set(b);
  return c;
}

__device__ __forceinline__ uint32_t atomic_add(gptr<uint32_t> p, uint32_t v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Slot = old value of ctr[key] + rank of this lane among the active lanes
// of its wave with the same key.  The lanes are grouped by key with ballots
// first (ALU only); then every group leader issues its atomic in the same
// instruction, so the wave waits for one atomic round trip, not one per key.
__device__ __forceinline__ uint32_t aggregated_fetch_add(gptr<uint32_t> ctr, uint32_t key,
                                                         bool active) {
  const uint32_t lane = lane_id();
  const uint64_t below = (1ull << lane) - 1ull;
  uint32_t leader = lane, rank = 0, size = 0;
  uint64_t todo = __ballot(active);
  while (todo != 0) {
    const int l = __builtin_ctzll(todo);
    const uint32_t lkey = (uint32_t)__builtin_amdgcn_readlane((int)key, l);
    const uint64_t group = __ballot(active && key == lkey);
    if (active && key == lkey) {
      leader = (uint32_t)l;
      rank = (uint32_t)__popcll(group & below);
      size = (uint32_t)__popcll(group);
    }
    todo &= ~group;
  }
  uint32_t base = 0;
  if (active && leader == lane) base = atomic_add(ctr + key, size);
  base = __shfl(base, (int)leader);
  return base + rank;
}

// Workgroups are dispatched round-robin over the 8 XCDs of the MI355X
// (workgroup b runs on XCD b mod 8), each XCD with its own L2.  This
// bijection on [0, nblocks) gives each XCD runs of kRun consecutive logical
// blocks, interleaved over the XCDs: neighbouring cells (which share cache
// lines at their boundaries and exchange particles) stay on one L2, while
// work that varies along the cell range stays balanced.
constexpr uint32_t kXcds = 8;
template <uint32_t kRun>
__device__ __forceinline__ uint32_t xcd_runs(uint32_t b, uint32_t nblocks) {
  constexpr uint32_t kSuper = kXcds * kRun;
  const uint32_t full = nblocks / kSuper * kSuper;
  if (b >= full) return b;
  const uint32_t s = b / kSuper, r = b % kSuper;
  return s * kSuper + (r % kXcds) * kRun + r / kXcds;
}

// A particle that took slot `slot` >= cap of cell c2 goes to a spill slot
// of dst, tagged with its cell; the one particle that takes slot cap lists
// the cell among the overflowing ones.  The spill slots hold every particle
// of the context, so the index check only guards against an internal error.
__device__ __forceinline__ void spill_particle(const GCells &dst, uint32_t c2, uint32_t slot,
                                               double x, double y, double z, double px,
                                               double py, double pz, uint32_t id,
                                               DevStatus *status) {
  SpillDesc *const sp = dst.sp;
  uint32_t *const h = sp->hdr + 2u * dst.q;
  const uint32_t i = atomicAdd(&h[0], 1u);
  if (i < sp->capacity) {
    const size_t o = sp->base + i;
    dst.st.x[o] = x;
    dst.st.y[o] = y;
    dst.st.z[o] = z;
    dst.st.px[o] = px;
    dst.st.py[o] = py;
    dst.st.pz[o] = pz;
    dst.st.id[o] = id;
    sp->cell[i] = c2;
  } else {
    atomicOr(&status->err, kErrSpill);
  }
  if (slot == dst.cap) sp->ocell[atomicAdd(&h[1], 1u)] = c2;
}

// Stores particle (r, p, id) at slot `slot` of cell c2 of dst: in the
// cell's block, or past its capacity in the spill region.
__device__ __forceinline__ void store_at_slot(const GCells &dst, uint32_t c2, uint32_t slot,
                                              bool active, double x, double y, double z,
                                              double px, double py, double pz, uint32_t id,
                                              DevStatus *status) {
  if (active) {
    if (slot < dst.cap) {
      const size_t o = (size_t)c2 * dst.cap + slot;
      dst.st.x[o] = x;
      dst.st.y[o] = y;
      dst.st.z[o] = z;
      dst.st.px[o] = px;
      dst.st.py[o] = py;
      dst.st.pz[o] = pz;
      dst.st.id[o] = id;
    } else {
      spill_particle(dst, c2, slot, x, y, z, px, py, pz, id, status);
    }
  }
}

// Appends particle (r, p, id) to cell c2 of dst (a slot by the
// wave-aggregated counter atomic).
__device__ __forceinline__ void append(const GCells &dst, uint32_t c2, bool active,
                                       double x, double y, double z, double px,
                                       double py, double pz, uint32_t id,
                                       DevStatus *status) {
  const uint32_t slot = aggregated_fetch_add(dst.count, c2, active);
  store_at_slot(dst, c2, slot, active, x, y, z, px, py, pz, id, status);
}

// The buffer laid out like c, `shift` bytes away.
template <typename T>
__device__ __forceinline__ gptr<T> shift_ptr(gptr<T> p, int64_t shift) {
  return (gptr<T>)((gptr<char>)p + shift);
}

// The destination of a collision launch of step t: src shifted by the
// distance between the two buffers, receiving the binning of step t + 1.
__device__ __forceinline__ GCells shifted(const GCells &c, int64_t shift);
__device__ __forceinline__ GCells dst_of(const GCells &src, int64_t shift, uint32_t t);

__device__ __forceinline__ GCells shifted(const GCells &c, int64_t shift) {
  GCells d;
  d.st.x = shift_ptr(c.st.x, shift);
  d.st.y = shift_ptr(c.st.y, shift);
  d.st.z = shift_ptr(c.st.z, shift);
  d.st.px = shift_ptr(c.st.px, shift);
  d.st.py = shift_ptr(c.st.py, shift);
  d.st.pz = shift_ptr(c.st.pz, shift);
  d.st.id = shift_ptr(c.st.id, shift);
  d.count = shift_ptr(c.count, shift);
  d.cap = c.cap;
  d.sp = (SpillDesc *)((char *)c.sp + shift);
  d.q = c.q;
  return d;
}

__device__ __forceinline__ GCells dst_of(const GCells &src, int64_t shift, uint32_t t) {
  return binning(shifted(src, shift), t + 1u);
}

// One particle in registers.
struct Particle {
  double x, y, z, px, py, pz;
  uint32_t id;
};

__device__ __forceinline__ Particle load_particle(const GSoA &st, size_t o) {
  return Particle{st.x[o], st.y[o], st.z[o], st.px[o], st.py[o], st.pz[o], st.id[o]};
}

__device__ __forceinline__ void store_particle(const GCells &dst, uint32_t c2, uint32_t slot,
                                               const Particle &q, DevStatus *status) {
  if (slot < dst.cap) {
    const size_t o = (size_t)c2 * dst.cap + slot;
    dst.st.x[o] = q.x;
    dst.st.y[o] = q.y;
    dst.st.z[o] = q.z;
    dst.st.px[o] = q.px;
    dst.st.py[o] = q.py;
    dst.st.pz[o] = q.pz;
    dst.st.id[o] = q.id;
  } else {
    spill_particle(dst, c2, slot, q.x, q.y, q.z, q.px, q.py, q.pz, q.id, status);
  }
}

// Appends two particles per lane (a and b, up to 128 per wave) to cells ca
// and cb of dst: the 128 keys are grouped by ballots (ALU only), the group's
// leader (its lowest lane, among the a particles first) adds the group size
// to the cell's count, and all leaders' atomics are in flight together, so
// the wave waits for one round trip for both halves.  A lane may lead one
// group through its a particle and one through its b particle.
__device__ __forceinline__ void append_two(const GCells &dst, uint32_t ca, bool act_a,
                                           const Particle &qa, uint32_t cb, bool act_b,
                                           const Particle &qb, DevStatus *status) {
  const uint32_t lane = lane_id();
  const uint64_t below = (1ull << lane) - 1ull;
  uint32_t lead_a = lane, lead_b = lane, sel_a = 0, sel_b = 0, rank_a = 0, rank_b = 0;
  uint32_t size_via_a = 0, size_via_b = 0;
  uint64_t todo_a = __ballot(act_a), todo_b = __ballot(act_b);
  while ((todo_a | todo_b) != 0) {
    const bool from_a = todo_a != 0;
    const int l = __builtin_ctzll(from_a ? todo_a : todo_b);
    const uint32_t key = (uint32_t)__builtin_amdgcn_readlane((int)(from_a ? ca : cb), l);
    const bool in_a = act_a && ca == key, in_b = act_b && cb == key;
    const uint64_t ma = __ballot(in_a), mb = __ballot(in_b);
    const uint32_t na = (uint32_t)__popcll(ma);
    if (in_a) {
      lead_a = (uint32_t)l;
      sel_a = from_a ? 0u : 1u;
      rank_a = (uint32_t)__popcll(ma & below);
    }
    if (in_b) {
      lead_b = (uint32_t)l;
      sel_b = from_a ? 0u : 1u;
      rank_b = na + (uint32_t)__popcll(mb & below);
    }
    if (lane == (uint32_t)l) {
      if (from_a) size_via_a = na + (uint32_t)__popcll(mb);
      else size_via_b = (uint32_t)__popcll(mb);
    }
    todo_a &= ~ma;
    todo_b &= ~mb;
  }
  uint32_t base0 = 0, base1 = 0;
  if (size_via_a != 0) base0 = atomic_add(dst.count + ca, size_via_a);
  if (size_via_b != 0) base1 = atomic_add(dst.count + cb, size_via_b);
  const uint32_t a0 = __shfl(base0, (int)lead_a), a1 = __shfl(base1, (int)lead_a);
  const uint32_t b0 = __shfl(base0, (int)lead_b), b1 = __shfl(base1, (int)lead_b);
  if (act_a) store_particle(dst, ca, (sel_a ? a1 : a0) + rank_a, qa, status);
  if (act_b) store_particle(dst, cb, (sel_b ? b1 : b0) + rank_b, qb, status);
}

// Particles of a cell held in its block (the rest, if any, are spilled).
__device__ __forceinline__ uint32_t occupancy(const GCells &c, uint32_t cell) {
  const uint32_t n = c.count[cell];
  return n < c.cap ? n : c.cap;
}

__global__ __launch_bounds__(kBlock) void k_fill_u32(uint32_t *p, uint32_t v,
                                                     int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < count) p[i] = v;
}

__global__ __launch_bounds__(64) void k_store_f64(double *p, double v) {
  if (threadIdx.x == 0) *p = v;
}

// Up to kWriteWords words carried as a kernel argument and stored to device
// memory in stream order (the host copy needs to live only until the launch
// returns, and no host-to-device copy waits for the stream).
constexpr uint32_t kWriteWords = 64;
struct WriteWords {
  uint32_t w[kWriteWords];
};
__global__ __launch_bounds__(64) void k_write_words(uint32_t *dst, WriteWords v,
                                                    uint32_t nwords) {
  for (uint32_t i = threadIdx.x; i < nwords; i += 64) dst[i] = v.w[i];
}

// Initial state (id order) -> validated and binned without streaming.
__global__ __launch_bounds__(kBlock) void k_init_bin(
    const double *__restrict__ x, const double *__restrict__ y,
    const double *__restrict__ z, const double *__restrict__ px,
    const double *__restrict__ py, const double *__restrict__ pz, Cells dst_arg,
    int64_t n, Geometry g, DevStatus *status, uint32_t binning_step) {
  const GCells dst = binning(to_global(dst_arg), binning_step);
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const bool active = i < n;
  double a = 0, b = 0, c = 0, qa = 0, qb = 0, qc = 0;
  uint32_t cell = 0;
  if (active) {
    a = x[i];
    b = y[i];
    c = z[i];
    qa = px[i];
    qb = py[i];
    qc = pz[i];
    const bool ok = __builtin_isfinite(a) && __builtin_isfinite(b) &&
                    __builtin_isfinite(c) && __builtin_isfinite(qa) &&
                    __builtin_isfinite(qb) && __builtin_isfinite(qc) && a >= 0.0 &&
                    a <= g.L[0] && b >= 0.0 && b <= g.L[1] && c >= 0.0 &&
                    c <= g.L[2] && norm3(qa, qb, qc) > 0.0;
    if (!ok) atomicOr(&status->err, kErrRange);
    cell = cell_id(g, a, b, c);
  }
  append(dst, cell, active, a, b, c, qa, qb, qc, (uint32_t)i, status);
}

// Cells holding more than 8, 16, 32 and 64 particles, added into over[4]:
// a grid stride over the cells, counts kept per wave, summed per block in
// LDS, then four atomics per block (one atomic per wave and counter
// serialised on the four addresses at 2 M cells).
__global__ __launch_bounds__(kBlock) void k_occupancy_over(Cells cur_arg, uint32_t n_cells,
                                                           uint32_t *over) {
  const GCells cur = to_global(cur_arg);
  __shared__ uint32_t part[kBlock / 64][4];
  uint32_t acc[4] = {0u, 0u, 0u, 0u};
  for (uint32_t c0 = blockIdx.x * kBlock; c0 < n_cells; c0 += gridDim.x * kBlock) {
    const uint32_t c = c0 + threadIdx.x;
    const uint32_t n = c < n_cells ? cur.count[c] : 0u;
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) acc[k] += (uint32_t)__popcll(__ballot(n > (8u << k)));
  }
  const uint32_t w = threadIdx.x / 64;
  if (lane_id() == 0)
    for (uint32_t k = 0; k < 4; ++k) part[w][k] = acc[k];
  __syncthreads();
  if (threadIdx.x < 4) {
    uint32_t sum = 0;
    for (uint32_t i = 0; i < kBlock / 64; ++i) sum += part[i][threadIdx.x];
    if (sum != 0) atomicAdd(&over[threadIdx.x], sum);
  }
}

// Stream + reflect + bin the spilled members of overflowing cell cv of src
// (found by a scan of the spill slots) into dst.  The whole wave.
__device__ __forceinline__ void stream_spilled(const GCells &src, const GCells &dst, uint32_t cv,
                                               const Geometry &g, DevStatus *status,
                                               uint32_t *trace_cell) {
  const SpillDesc *const sp = src.sp;
  const uint32_t ns = min(sp->hdr[2u * src.q], sp->capacity);
  const size_t sbase = sp->base;
  const uint32_t lane = lane_id();
  for (uint32_t i0 = 0; i0 < ns; i0 += 64u) {
    const uint32_t i = i0 + lane;
    const bool hit = i < ns && sp->cell[i] == cv;
    if (__ballot(hit) == 0) continue;
    Particle q{};
    uint32_t c2 = 0;
    if (hit) {
      q = load_particle(src.st, sbase + i);
      advance<true>(g, q.x, q.y, q.z, q.px, q.py, q.pz);
      c2 = cell_id(g, q.x, q.y, q.z);
      if (trace_cell) trace_cell[q.id] = c2;
    }
    append(dst, c2, hit, q.x, q.y, q.z, q.px, q.py, q.pz, q.id, status);
  }
}

// Clears the spill counter set of `c` that no launch uses now: the one of
// the binning two steps after (or before) the one c holds.
__device__ __forceinline__ void clear_idle_spill_set(const GCells &c) {
  uint32_t *const h = c.sp->hdr + 2u * (c.q ^ 1u);
  h[0] = 0u;
  h[1] = 0u;
}

// Stream + reflect + bin the particles of the source cells c0 .. c_end - 1
// (at most 64 / G of them), G lanes per cell; G = 64 is one wave per cell.
// Clears the source counts, so the source buffer can receive the next
// binning.
template <uint32_t G>
__device__ __forceinline__ void cells_stream_bin(const GCells &src, const GCells &dst,
                                                 uint32_t c0, uint32_t c_end,
                                                 const Geometry &g, DevStatus *status,
                                                 uint32_t *trace_cell) {
  const uint32_t lane = lane_id();
  const uint32_t c = c0 + lane / G, gl = lane % G;
  const bool in_range = c < c_end;
  const uint32_t cnt = in_range ? src.count[c] : 0u;
  const uint32_t n = cnt < src.cap ? cnt : src.cap;  // the block part
  const size_t base = (size_t)c * src.cap;
  // then the spilled members of overflowing cells
  const uint64_t ovm = __ballot(in_range && gl == 0 && cnt > src.cap);
  if (ovm != 0) {
    for (uint64_t m = ovm; m != 0; m &= m - 1ull) {
      const uint32_t cv = (uint32_t)__builtin_amdgcn_readlane((int)c, __builtin_ctzll(m));
      stream_spilled(src, dst, cv, g, status, trace_cell);
    }
  }
  if (G == 64) {
    // one cell: 128 particles per round, both halves' atomics in flight together
    for (uint32_t j0 = 0; j0 < n; j0 += 128) {
      const uint32_t ja = j0 + lane, jb = j0 + 64 + lane;
      const bool act_a = ja < n, act_b = jb < n;
      Particle qa{}, qb{};
      if (act_a) qa = load_particle(src.st, base + ja);
      if (act_b) qb = load_particle(src.st, base + jb);
      uint32_t ca = 0, cb = 0;
      if (act_a) {
        advance<true>(g, qa.x, qa.y, qa.z, qa.px, qa.py, qa.pz);
        ca = cell_id(g, qa.x, qa.y, qa.z);
        if (trace_cell) trace_cell[qa.id] = ca;
      }
      if (act_b) {
        advance<true>(g, qb.x, qb.y, qb.z, qb.px, qb.py, qb.pz);
        cb = cell_id(g, qb.x, qb.y, qb.z);
        if (trace_cell) trace_cell[qb.id] = cb;
      }
      append_two(dst, ca, act_a, qa, cb, act_b, qb, status);
    }
    if (in_range && gl == 0) src.count[c] = 0u;
    return;
  }
  for (uint32_t j0 = 0; __ballot(j0 < n) != 0; j0 += G) {
    const uint32_t j = j0 + gl;
    const bool active = j < n;
    double x = 0, y = 0, z = 0, px = 0, py = 0, pz = 0;
    uint32_t id = 0, c2 = 0;
    if (active) {
      x = src.st.x[base + j];
      y = src.st.y[base + j];
      z = src.st.z[base + j];
      px = src.st.px[base + j];
      py = src.st.py[base + j];
      pz = src.st.pz[base + j];
      id = src.st.id[base + j];
      advance<true>(g, x, y, z, px, py, pz);
      c2 = cell_id(g, x, y, z);
      if (trace_cell) trace_cell[id] = c2;
    }
    append(dst, c2, active, x, y, z, px, py, pz, id, status);
  }
  if (in_range && gl == 0) src.count[c] = 0u;
}

// Four waves per block; each wave takes 64 / G consecutive source cells;
// src holds the binning of step t - 1, dst receives that of step t.
template <uint32_t G>
__global__ __launch_bounds__(kBlock) void k_stream_bin(Cells src_arg, Cells dst_arg,
                                                       uint32_t n_cells, Geometry g,
                                                       DevStatus *status,
                                                       uint32_t *trace_cell, uint32_t t) {
  const GCells src = binning(to_global(src_arg), t - 1u);
  const GCells dst = binning(to_global(dst_arg), t);
  constexpr uint32_t kPer = 64 / G;
  const uint32_t c0 =
      (xcd_runs<2>(blockIdx.x, gridDim.x) * kCellsPerBlock + threadIdx.x / 64) * kPer;
  if (c0 >= n_cells) return;
  if (c0 == 0 && lane_id() == 0) clear_idle_spill_set(src);
  const uint32_t c_end = c0 + kPer < n_cells ? c0 + kPer : n_cells;
  cells_stream_bin<G>(src, dst, c0, c_end, g, status, trace_cell);
}

// Orders the calling wave's LDS accesses before and after this point for
// its own lanes (LDS executes one wave's operations in order; the fence
// keeps the compiler from moving accesses across and waits for them).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

// Slots in the destination cells of a wave's particles that all move from
// cell c0 to c0 or one of its 26 neighbours, direction
// dir = 9 (dx + 1) + 3 (dy + 1) + (dz + 1) for axis offsets dx, dy, dz in
// {-1, 0, 1} (x-major ids: the neighbour is c0 + dx sx + dy sy + dz).  LDS
// atomics number each direction's lanes; lane d then adds direction d's
// count to that cell's counter, one global atomic for every direction in
// use, so the wave makes one round trip and no loop over its distinct
// destinations.  s_dir: 54 words of LDS owned by the wave.  Every lane of
// the wave calls it; an inactive lane passes dir 13 and ignores the result.
__device__ __forceinline__ uint32_t neighbour_fetch_add(gptr<uint32_t> ctr, uint32_t c0,
                                                        uint32_t sx, uint32_t sy, uint32_t dir,
                                                        bool active, uint32_t *s_dir) {
  const uint32_t lane = lane_id();
  if (lane < 27u) s_dir[lane] = 0u;
  wave_lds_sync();
  uint32_t rank = 0;
  if (active) rank = atomicAdd(&s_dir[dir], 1u);
  wave_lds_sync();
  if (lane < 27u) {
    const uint32_t cnt = s_dir[lane];
    uint32_t base = 0;
    if (cnt != 0u) {
      const int32_t dx = (int32_t)(lane / 9u) - 1, dy = (int32_t)(lane / 3u % 3u) - 1,
                    dz = (int32_t)(lane % 3u) - 1;
      const uint32_t key =
          (uint32_t)((int32_t)c0 + dx * (int32_t)sx + dy * (int32_t)sy + dz);
      base = atomic_add(ctr + key, cnt);
    }
    s_dir[27u + lane] = base;
  }
  wave_lds_sync();
  return s_dir[27u + dir] + rank;
}

// Exclusive scan of the counts into compact offsets (trace only; the counts
// are left intact).  Tile-local pass, then carries from earlier tiles.
__global__ __launch_bounds__(kBlock) void k_scan_tiles(Cells cur_arg,
                                                       uint32_t *offsets,
                                                       uint32_t *tile_sums,
                                                       int64_t n_cells) {
  const GCells cur = to_global(cur_arg);
  __shared__ uint32_t s_wave[kBlock / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * 8;
  const uint32_t lane = lane_id(), wave = threadIdx.x / 64;
  uint32_t v[8];
  uint32_t sum = 0;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int64_t idx = base + j;
    const uint32_t cnt = idx < n_cells ? cur.count[idx] : 0u;
    v[j] = sum;
    sum += cnt;
  }
  uint32_t incl = sum;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t up = __shfl_up(incl, o);
    if ((int)lane >= o) incl += up;
  }
  if (lane == 63) s_wave[wave] = incl;
  __syncthreads();
  uint32_t wave_off = 0;
  for (uint32_t w = 0; w < wave; ++w) wave_off += s_wave[w];
  const uint32_t excl = wave_off + incl - sum;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int64_t idx = base + j;
    if (idx < n_cells) offsets[idx] = excl + v[j];
  }
  if (threadIdx.x == kBlock - 1) tile_sums[blockIdx.x] = wave_off + incl;
}

__global__ __launch_bounds__(kBlock) void k_scan_carry(uint32_t *offsets,
                                                       const uint32_t *tile_sums,
                                                       int64_t n_cells) {
  __shared__ uint32_t s_red[kBlock / 64];
  const uint32_t lane = lane_id(), wave = threadIdx.x / 64;
  uint32_t part = 0;
  for (uint32_t j = threadIdx.x; j < blockIdx.x; j += kBlock) part += tile_sums[j];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) part += __shfl_down(part, o);
  if (lane == 0) s_red[wave] = part;
  __syncthreads();
  uint32_t carry = 0;
  for (int w = 0; w < kBlock / 64; ++w) carry += s_red[w];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * 8;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int64_t idx = base + j;
    if (idx < n_cells) offsets[idx] += carry;
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0)
    offsets[n_cells] = carry + tile_sums[blockIdx.x];
}

// ---------------------------------------------------------------------------
// Collisions: one wave64 (one workgroup) per cell, or two (k_step2).
// ---------------------------------------------------------------------------
// A cell being stepped: member j is slot base + j of the buffer's arrays,
// or, in an overflowing cell (ov), for j >= cap spill slot sbase + sidx[j -
// cap] (at_spill).  ov is uniform over the workgroup, so normal cells take
// the first form without a per-lane choice.  Once an overflowing cell's
// slots are listed in LDS (slots), at() reads them there, which keeps fewer
// values live than the two-part form.
struct CellView {
  uint32_t c, n, t;
  size_t base;
  uint32_t cap;
  bool ov;
  size_t sbase;
  const uint32_t *sidx;
  const uint32_t *slots;
  __device__ __forceinline__ size_t at_spill(uint32_t j) const {
    if (ov && j >= cap) return sbase + sidx[j - cap];
    return base + j;
  }
  __device__ __forceinline__ size_t at(uint32_t j) const {
    if (ov) return slots[j];
    return base + j;
  }
};

// kBlockSync: the workgroup is this one wave, and its barriers order the
// LDS accesses; otherwise a wave that shares its workgroup with others
// synchronises with itself only.
template <bool kBlockSync>
__device__ __forceinline__ void cell_sync() {
  if (kBlockSync)
    __syncthreads();
  else
    wave_lds_sync();
}

// Exact Eq. (3) test of the nf filtered pairs in s_filt (increasing pair
// index), then greedy claim in that order.  Entries are rewritten as
// flag | a << 10 | b.  claimed_bits holds, per lane, the claimed flags of
// canonical indices lane + 64 j.  One wave; see cell_sync for kBlockSync.
template <bool kTrace, bool kBlockSync = true>
__device__ __forceinline__ void resolve_filtered(
    uint32_t nf, const CellView &cv, const PairArgs &pa, const GSoA &st,
    const uint16_t *s_perm, uint32_t *s_filt, uint32_t *s_claim,
    uint32_t &nclaim, uint32_t &claimed_bits, uint32_t &n_acc,
    const TraceArgs &tr, DevStatus *status) {
  const uint32_t lane = lane_id();
  cell_sync<kBlockSync>();
  for (uint32_t i = lane; i < nf; i += 64) {
    const uint32_t k = s_filt[i];
    const Words4 w = philox10(k, cv.c, cv.t, 0u, pa.key0, pa.key1);
    const double u = uniform53(w.w0, w.w1);
    uint32_t a, b;
    pair_of_index(k, cv.n, a, b);
    const size_t ia = cv.at(s_perm[a]), ib = cv.at(s_perm[b]);
    const double P = p22(st.px[ia], st.py[ia], st.pz[ia], st.px[ib], st.py[ib],
                         st.pz[ib], pa.kfac);
    const bool acc = u < P;
    n_acc += acc ? 1u : 0u;
    s_filt[i] = acc ? (0x80000000u | (a << 10) | b) : 0u;
    if (kTrace && acc && tr.cand) {
      const uint32_t slot = atomicAdd(&tr.counts[0], 1u);
      if (slot < tr.cand_cap) {
        tr.cand[3 * (size_t)slot + 0] = cv.c;
        tr.cand[3 * (size_t)slot + 1] = a;
        tr.cand[3 * (size_t)slot + 2] = b;
      } else {
        atomicOr(&status->err, kErrTrace);
      }
    }
  }
  cell_sync<kBlockSync>();
  // the accepted entries in list order: a row of 64 entries at a time, its
  // accepted ones taken from their lanes in lane order
  for (uint32_t i0 = 0; i0 < nf; i0 += 64u) {
    const uint32_t vr = i0 + lane < nf ? s_filt[i0 + lane] : 0u;
    for (uint64_t m = __ballot((vr & 0x80000000u) != 0u); m != 0; m &= m - 1ull) {
      const uint32_t v = (uint32_t)__builtin_amdgcn_readlane((int)vr,
                                                             (int)__builtin_ctzll(m));
      const uint32_t a = (v >> 10) & 1023u, b = v & 1023u;
      const bool own_a = (a & 63u) == lane, own_b = (b & 63u) == lane;
      const bool hit = (own_a && ((claimed_bits >> (a >> 6)) & 1u)) ||
                       (own_b && ((claimed_bits >> (b >> 6)) & 1u));
      if (__ballot(hit) == 0) {
        if (own_a) claimed_bits |= 1u << (a >> 6);
        if (own_b) claimed_bits |= 1u << (b >> 6);
        if (lane == 0) s_claim[nclaim] = v;
        ++nclaim;
      }
    }
  }
  cell_sync<kBlockSync>();
}

// Pair tests k = k_begin .. k_end - 1 of a cell by one wave, lane-strided,
// two rows of 64 pairs per iteration while two rows remain.  A pair whose
// Philox word w1 rules out acceptance (u >= w1 2^-32 > P22) is dropped at
// once; the others are appended to filt (nf entries, increasing k; at most
// kFiltCap).  kResolve: when filt nears full its entries are resolved
// (exact test and claims) and the tests go on; otherwise the tests stop
// there.  Returns the first pair not tested (k_end when all were).
template <bool kResolve, bool kTrace, bool kBlockSync, uint32_t kFiltCap>
__device__ __forceinline__ uint32_t test_pairs(
    uint32_t k_begin, uint32_t k_end, const CellView &cv, const PairArgs &pa,
    const GSoA &st, const uint16_t *s_perm, uint32_t *filt, uint32_t &nf,
    uint32_t *s_claim, uint32_t &nclaim, uint32_t &claimed_bits, uint32_t &n_acc,
    const TraceArgs &tr, DevStatus *status) {
  static_assert(kFiltCap >= 256, "filter buffer");
  const uint32_t lane = lane_id();
  const uint64_t below = (1ull << lane) - 1ull;
  const uint32_t lim = pa.w1_max;
  uint32_t k0 = k_begin;
  for (; k0 + 128u <= k_end; k0 += 128u) {
    const uint32_t ka = k0 + lane, kb = k0 + 64u + lane;
    const uint32_t wa = philox10_w1(ka, cv.c, cv.t, 0u, pa.key0, pa.key1);
    const uint32_t wb = philox10_w1(kb, cv.c, cv.t, 0u, pa.key0, pa.key1);
    const bool pass_a = wa <= lim, pass_b = wb <= lim;
    const uint64_t ma = __ballot(pass_a), mb = __ballot(pass_b);
    if ((ma | mb) != 0) {
      if (pass_a) filt[nf + (uint32_t)__popcll(ma & below)] = ka;
      nf += (uint32_t)__popcll(ma);
      if (pass_b) filt[nf + (uint32_t)__popcll(mb & below)] = kb;
      nf += (uint32_t)__popcll(mb);
      if (nf > kFiltCap - 128u) {
        if (!kResolve) return k0 + 128u;
        resolve_filtered<kTrace, kBlockSync>(nf, cv, pa, st, s_perm, filt, s_claim, nclaim,
                                             claimed_bits, n_acc, tr, status);
        nf = 0;
      }
    }
  }
  for (; k0 < k_end; k0 += 64u) {
    const uint32_t k = k0 + lane;
    bool pass = false;
    if (k < k_end) pass = philox10_w1(k, cv.c, cv.t, 0u, pa.key0, pa.key1) <= lim;
    const uint64_t m = __ballot(pass);
    if (m != 0) {
      if (pass) filt[nf + (uint32_t)__popcll(m & below)] = k;
      nf += (uint32_t)__popcll(m);
      if (nf > kFiltCap - 64u) {
        if (!kResolve) return k0 + 64u < k_end ? k0 + 64u : k_end;
        resolve_filtered<kTrace, kBlockSync>(nf, cv, pa, st, s_perm, filt, s_claim, nclaim,
                                             claimed_bits, n_acc, tr, status);
        nf = 0;
      }
    }
  }
  return k_end;
}

// Cells of more than kBucketRankMin particles rank their ids through
// kRankBuckets buckets by value; smaller cells (one particle a lane) count
// all ids, a shorter chain of independent LDS reads than the buckets'
// reductions, scan and atomics.
constexpr uint32_t kRankBuckets = 256;
constexpr uint32_t kBucketRankMin = 63;

// Minimum / maximum over the wave's 64 lanes (every lane active), the same
// in every lane.  DPP
// moves within the VALU instead of LDS permutes: within quads, half rows
// and rows, then row 15's result into rows 1 and 3 and row 31's into rows
// 2 and 3, so that lane 63 holds the whole wave's; lanes a move does not
// write keep their own value.
template <typename Op>
__device__ __forceinline__ uint32_t wave_reduce(uint32_t v, Op op) {
  v = op(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0xB1, 0xF, 0xF, false));
  v = op(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x4E, 0xF, 0xF, false));
  v = op(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x141, 0xF, 0xF, false));
  v = op(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x140, 0xF, 0xF, false));
  v = op(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x142, 0xA, 0xF, false));
  v = op(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x143, 0xC, 0xF, false));
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// Inclusive prefix sum over the wave's lanes (every lane active): DPP
// shifts by 1, 2, 4 and 8 within rows (lanes without a source add 0), then
// row 15's sum into rows 1 and 3 and row 31's into rows 2 and 3.
__device__ __forceinline__ uint32_t wave_inclusive_sum(uint32_t x) {
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, true);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, true);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, true);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, true);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xA, 0xF, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xC, 0xF, false);
  return x;
}

__device__ __forceinline__ uint32_t wave_min(uint32_t v) {
  return wave_reduce(v, [](uint32_t a, uint32_t b) { return a < b ? a : b; });
}

__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
  return wave_reduce(v, [](uint32_t a, uint32_t b) { return a > b ? a : b; });
}

// LDS of a cell: buf holds the cell's ids while the canonical
// order is built; after that its first half holds the filtered pairs and its
// second half the claimed pairs.
template <bool kFused, uint32_t kCap>
struct CellLds {
  __align__(16) uint32_t buf[kCap];
  uint16_t perm[kCap];
  __align__(16) uint32_t bkt[kRankBuckets + 4];  // bucket ends, then starts
  __align__(16) uint32_t sorted[kCap];           // ids in bucket order
  uint32_t ov_pool_lo, ov_pool_hi, ov_ok, pad;   // an overflowing cell's scratch
};

// LDS of the second wave of a cell stepped by two: its filtered pairs, and
// what it hands to the first wave (count, first pair it did not test), and
// the first wave's claim count for the kinematics.
template <uint32_t kCap>
struct SecondWaveLds {
  uint32_t filt[kCap / 2];
  uint32_t n_filt, k_resume, nclaim, pad;
};

// The launch of step t clears the scratch that no launch uses now: src's
// idle spill counter set and the pool counter of step t + 1.
__device__ __forceinline__ void clear_idle_scratch(const GCells &src, uint32_t t) {
  clear_idle_spill_set(src);
  src.sp->pool->hdr[(t + 1u) & 1u] = 0ull;
}

// Observation sums of a cell (Sec. 5 profiles): sum E, sum p_x and
// sum p_x^2 / E of the momenta after the step's collisions, accumulated per
// lane, then reduced over the wave and written with the cell's count by
// lane 0 (obs: kCellSums doubles a cell).
__device__ __forceinline__ void obs_add(double px, double py, double pz, double &se,
                                        double &sp, double &sxx) {
  const double e = norm3(px, py, pz);
  se += e;
  sp += px;
  sxx += (px * px) / e;
}

__device__ __forceinline__ void obs_write_wave(double *obs, uint32_t c, uint32_t cnt,
                                               double se, double sp, double sxx) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    se += __shfl_down(se, o);
    sp += __shfl_down(sp, o);
    sxx += __shfl_down(sxx, o);
  }
  if (lane_id() == 0) {
    double *const out = obs + kCellSums * (size_t)c;
    out[0] = se;
    out[1] = sp;
    out[2] = sxx;
    out[3] = (double)cnt;
  }
}

// Wave 0 of an overflowing cell's workgroup: takes scratch from the pool
// (counter t & 1) for the slots of the cell's spilled members -- and, for a
// cell larger than the LDS holds, its canonical order, claimed flags and
// claims -- and lists those slots (a scan of the spill slots, in increasing
// order).  Leaves the scratch offset and a success flag in LDS.
template <bool kFused, uint32_t kCap>
__device__ void find_spilled(const GCells &src, const CellView &cv, CellLds<kFused, kCap> &lds,
                             DevStatus *status) {
  const uint32_t lane = lane_id();
  const uint64_t below = (1ull << lane) - 1ull;
  const SpillDesc *const sd = src.sp;
  OverflowPool *const pool = sd->pool;
  const uint32_t n = cv.n, nsp = n - cv.cap;
  const uint32_t ns = min(sd->hdr[2u * src.q], sd->capacity);
  uint64_t need = nsp;
  if (n > kCap) need += (uint64_t)n + n / 2u + 1u + (n + 31u) / 32u;
  uint32_t lo = 0, hi = 0;
  if (lane == 0) {
    const unsigned long long b = atomicAdd(&pool->hdr[cv.t & 1u], (unsigned long long)need);
    lo = (uint32_t)b;
    hi = (uint32_t)(b >> 32);
  }
  lo = (uint32_t)__shfl((int)lo, 0);
  hi = (uint32_t)__shfl((int)hi, 0);
  const uint64_t b = ((uint64_t)hi << 32) | lo;
  bool ok = b + need <= pool->capacity;
  if (ok) {
    uint32_t *const mem = pool->buf + b;
    uint32_t found = 0;
    for (uint32_t i0 = 0; i0 < ns; i0 += 64u) {
      const uint32_t i = i0 + lane;
      const bool hit = i < ns && sd->cell[i] == cv.c;
      const uint64_t mk = __ballot(hit);
      if (hit) {
        const uint32_t slot = found + (uint32_t)__popcll(mk & below);
        if (slot < nsp) mem[slot] = i;
      }
      found += (uint32_t)__popcll(mk);
    }
    ok = found == nsp;
  }
  if (lane == 0) {
    if (!ok) atomicOr(&status->err, kErrSpill);
    lds.ov_pool_lo = lo;
    lds.ov_pool_hi = hi;
    lds.ov_ok = ok ? 1u : 0u;
  }
}

// The collisions of an overflowing cell larger than the LDS holds (then,
// kFused, the binning of its members), by one wave with its canonical
// order, claimed flags and claims in global scratch: ranks by counting
// smaller ids against chunks staged in LDS, pair tests 64 at a time in
// increasing k (Philox w1 filter, then Eq. (3)), each row's accepted pairs
// claimed in k order, then the kinematics.  A cell past the 32-bit pair
// index skips its collisions (flagged); its members are still binned.
template <bool kFused, bool kTrace, uint32_t kCap>
__device__ void large_cell_step(const GCells &src, const GCells &dst, const CellView &cv,
                                const PairArgs &pa, const Geometry &g, DevStatus *status,
                                const TraceArgs &tr, CellLds<kFused, kCap> &lds,
                                double *obs) {
  const uint32_t lane = lane_id();
  const uint32_t n = cv.n;
  uint32_t *const perm = const_cast<uint32_t *>(cv.sidx) + (n - cv.cap);
  uint32_t *const claims = perm + n;
  uint32_t *const bits = claims + n / 2u + 1u;
  const GSoA &st = src.st;
  uint32_t npairs = 0;  // < 2^32 below the pair-index bound
  uint32_t nclaim = 0, n_acc = 0;
  if (n > kMaxPairIndexCell) {
    if (lane == 0) atomicOr(&status->err, kErrPairIndex);
  } else {
    for (uint32_t j0 = 0; j0 < n; j0 += 64u) {
      const uint32_t j = j0 + lane;
      const uint32_t me = j < n ? st.id[cv.at_spill(j)] : 0xFFFFFFFFu;
      uint32_t r = 0;
      for (uint32_t i0 = 0; i0 < n; i0 += kCap) {
        const uint32_t cnt = min(kCap, n - i0);
        wave_lds_sync();
        for (uint32_t i = lane; i < cnt; i += 64u) lds.buf[i] = st.id[cv.at_spill(i0 + i)];
        wave_lds_sync();
        if (j < n)
          for (uint32_t i = 0; i < cnt; ++i) r += lds.buf[i] < me ? 1u : 0u;
      }
      if (j < n) {
        perm[r] = j;
        if (kTrace && tr.perm) tr.perm[tr.offsets[cv.c] + r] = me;
      }
    }
    for (uint32_t w = lane; w < (n + 31u) / 32u; w += 64u) bits[w] = 0u;
    wave_lds_sync();
    npairs = (uint32_t)((uint64_t)n * (n - 1u) / 2u);
    // k0 + 64 stays below 2^32: npairs <= 4 294 930 221
    for (uint32_t k0 = 0; pa.any && k0 < npairs; k0 += 64u) {
      const uint32_t k = k0 + lane;
      bool acc = false;
      if (k < npairs && philox10_w1(k, cv.c, cv.t, 0u, pa.key0, pa.key1) <= pa.w1_max) {
        const Words4 w = philox10(k, cv.c, cv.t, 0u, pa.key0, pa.key1);
        uint32_t a, b;
        pair_of_index64(k, n, a, b);
        const size_t ia = cv.at_spill(perm[a]), ib = cv.at_spill(perm[b]);
        acc = uniform53(w.w0, w.w1) <
              p22(st.px[ia], st.py[ia], st.pz[ia], st.px[ib], st.py[ib], st.pz[ib], pa.kfac);
        if (kTrace && acc && tr.cand) {
          const uint32_t slot = atomicAdd(&tr.counts[0], 1u);
          if (slot < tr.cand_cap) {
            tr.cand[3 * (size_t)slot + 0] = cv.c;
            tr.cand[3 * (size_t)slot + 1] = a;
            tr.cand[3 * (size_t)slot + 2] = b;
          } else {
            atomicOr(&status->err, kErrTrace);
          }
        }
      }
      n_acc += acc ? 1u : 0u;
      for (uint64_t m = __ballot(acc); m != 0; m &= m - 1ull) {
        const uint32_t kk = k0 + (uint32_t)__builtin_ctzll(m);
        uint32_t a, b;
        pair_of_index64(kk, n, a, b);
        const uint32_t wa = bits[a >> 5], wb = bits[b >> 5];
        if (((wa >> (a & 31u)) & 1u) == 0u && ((wb >> (b & 31u)) & 1u) == 0u) {
          if (lane == 0) {
            if ((a >> 5) == (b >> 5)) {
              bits[a >> 5] = wa | (1u << (a & 31u)) | (1u << (b & 31u));
            } else {
              bits[a >> 5] = wa | (1u << (a & 31u));
              bits[b >> 5] = wb | (1u << (b & 31u));
            }
            claims[nclaim] = kk;
          }
          ++nclaim;
          wave_lds_sync();
        }
      }
    }
  }
  wave_lds_sync();
  for (uint32_t i0 = 0; i0 < nclaim; i0 += 64u) {
    const uint32_t i = i0 + lane;
    if (i < nclaim) {
      const uint32_t k = claims[i];
      uint32_t a, b;
      pair_of_index64(k, n, a, b);
      const Words4 w = philox10(k, cv.c, cv.t, 1u, pa.key0, pa.key1);
      const size_t ia = cv.at_spill(perm[a]), ib = cv.at_spill(perm[b]);
      double ax = st.px[ia], ay = st.py[ia], az = st.pz[ia];
      double bx = st.px[ib], by = st.py[ib], bz = st.pz[ib];
      scatter_pair(ax, ay, az, bx, by, bz, uniform53(w.w0, w.w1), uniform53(w.w2, w.w3));
      st.px[ia] = ax;
      st.py[ia] = ay;
      st.pz[ia] = az;
      st.px[ib] = bx;
      st.py[ib] = by;
      st.pz[ib] = bz;
      if (kTrace && tr.claim) {
        const uint32_t slot = atomicAdd(&tr.counts[1], 1u);
        if (slot < tr.claim_cap) {
          tr.claim[3 * (size_t)slot + 0] = cv.c;
          tr.claim[3 * (size_t)slot + 1] = a;
          tr.claim[3 * (size_t)slot + 2] = b;
        } else {
          atomicOr(&status->err, kErrTrace);
        }
      }
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) n_acc += __shfl_down(n_acc, o);
  if (lane == 0) {
    const uint32_t slot = cv.c % kCounterSlots;
    atomicAdd(&status->pairs[slot], (unsigned long long)npairs);
    atomicAdd(&status->cand[slot], (unsigned long long)n_acc);
    atomicAdd(&status->claims[slot], (unsigned long long)nclaim);
  }
  wave_lds_sync();  // new momenta visible to the binning lanes
  double se = 0.0, sp = 0.0, sxx = 0.0;
  if (kFused) {
    const Geometry g_l = g;
    for (uint32_t j0 = 0; j0 < n; j0 += 64u) {
      const uint32_t j = j0 + lane;
      const bool active = j < n;
      Particle q{};
      uint32_t c2 = 0;
      if (active) {
        q = load_particle(st, cv.at_spill(j));
        if (obs) obs_add(q.px, q.py, q.pz, se, sp, sxx);
        advance<true>(g_l, q.x, q.y, q.z, q.px, q.py, q.pz);
        c2 = cell_id(g_l, q.x, q.y, q.z);
      }
      append(dst, c2, active, q.x, q.y, q.z, q.px, q.py, q.pz, q.id, status);
    }
    if (lane == 0) src.count[cv.c] = 0u;
  } else if (obs) {
    for (uint32_t j = lane; j < n; j += 64u) {
      const size_t o = cv.at_spill(j);
      obs_add(st.px[o], st.py[o], st.pz[o], se, sp, sxx);
    }
  }
  if (obs) obs_write_wave(obs, cv.c, n, se, sp, sxx);
}

// Collisions of cell c of src at step t by a workgroup of kW waves (1 or
// 2).  kFused: afterwards stream and bin the cell's particles into dst for
// step t+1 and clear src's count.  Starts with a barrier, so a wave may call
// it for several cells.  With two waves (x2: the second wave's LDS) the
// pair range is split: the first wave tests the pairs below kh, resolving
// and claiming as it goes, while the second filters the pairs from kh on
// into its own buffer; the first wave then resolves those in order (they
// all follow its own) and tests any pairs the second left once its buffer
// filled.  Claims are thus made in increasing pair order as with one wave,
// and every other phase is split over the workgroup's lanes.  Both waves
// pass the same barriers; code that one wave runs alone synchronises with
// itself only.
template <bool kFused, bool kTrace, uint32_t kCap, uint32_t kW = 1>
__device__ __forceinline__ void cell_step(const GCells &src, const GCells &dst, uint32_t c,
                                          uint32_t t, const PairArgs &pa,
                                          const Geometry &g, DevStatus *status,
                                          const TraceArgs &tr, CellLds<kFused, kCap> &lds,
                                          SecondWaveLds<kCap> *x2 = nullptr,
                                          double *obs = nullptr) {
  static_assert(kW == 1 || (kW == 2 && !kTrace), "one or two waves, traces with one");
  constexpr uint32_t kT = 64 * kW;
  // filtered pairs and claimed pairs share the id buffer, kCap / 2 each
  constexpr uint32_t kFilt = kCap / 2;
  static_assert(kCap <= kCellCap && kFilt >= 256, "cell capacity");
  uint32_t *const s_id = lds.buf;
  uint32_t *const s_filt = lds.buf;
  uint32_t *const s_claim = lds.buf + kFilt;
  uint16_t *const s_perm = lds.perm;
  __syncthreads();
  // A fused one-wave step of a cell whose members are all in its block
  // keeps the new momenta of up to kMomCap claims in LDS (where the rank
  // sorted its ids; claim i's two members at 2i, 2i + 1, and by member a
  // byte map to them, in the rank's buckets) for its binning, instead of
  // writing them back to the source block, whose lines would then be
  // written to memory once more though no one reads them again.
  constexpr bool kMomInLds = kFused && kW == 1;
  constexpr uint32_t kMomCap = kCap / 12u;  // 6 doubles a claim in sorted[]
  static_assert(6u * kMomCap * sizeof(double) <= kCap * sizeof(uint32_t), "claim momenta");
  static_assert(2u * kMomCap + 2u <= 255u && kCap <= 4u * (kRankBuckets + 4u), "claim map");
  double *const s_mx = reinterpret_cast<double *>(lds.sorted);
  double *const s_my = s_mx + 2u * kMomCap;
  double *const s_mz = s_my + 2u * kMomCap;
  uint8_t *const s_cmap = reinterpret_cast<uint8_t *>(lds.bkt);
  bool mom_lds = false;

  const uint32_t lane = lane_id();
  const uint32_t tid = kW == 1 ? lane : (uint32_t)threadIdx.x;
  const uint32_t wv = tid / 64;  // this wave within the cell's workgroup
  CellView cv;
  cv.c = c;
  cv.t = t;
  cv.base = (size_t)cv.c * src.cap;
  cv.cap = src.cap;
  cv.n = src.count[cv.c];
  cv.ov = cv.n > src.cap;
  cv.sbase = 0;
  cv.sidx = nullptr;
  cv.slots = lds.sorted;
  if (cv.c == 0 && tid == 0) clear_idle_scratch(src, t);
  // Wave priority: the phases that are chains of dependent loads, LDS
  // atomics and barriers (ids and rank; claims, kinematics and binning)
  // issue ahead of the other waves' pair-test loops, which keep the VALU
  // busy meanwhile; the pair tests run at the base priority.
  if (kW == 1) __builtin_amdgcn_s_setprio(1);
  if (cv.ov) {
    // an overflowing cell: find its spilled members (wave 0), then step it
    // here, in LDS if it fits, else with the global-memory method
    if (wv == 0) find_spilled<kFused, kCap>(src, cv, lds, status);
    __syncthreads();
    if (lds.ov_ok == 0u) return;  // internal error, flagged
    const SpillDesc *const sd = src.sp;
    cv.sbase = sd->base;
    cv.sidx = sd->pool->buf + (((uint64_t)lds.ov_pool_hi << 32) | lds.ov_pool_lo);
    if (cv.n > kCap) {
      if (wv == 0)
        large_cell_step<kFused, kTrace, kCap>(src, dst, cv, pa, g, status, tr, lds,
                                              kW == 1 ? obs : nullptr);
      return;
    }
  }
  const uint32_t n = cv.n;
  const GSoA &st = src.st;
  // observation sums only for one wave per cell (the batch's shape)
  double *const ob = kW == 1 ? obs : nullptr;

  uint32_t nclaim = 0;
  if (n >= 2) {
    // ids to LDS, padded to a multiple of 4 with an id no particle has
    const uint32_t n4 = (n + 3u) & ~3u;
    for (uint32_t j = tid; j < n4; j += kT)
      s_id[j] = j < n ? st.id[cv.at_spill(j)] : 0xFFFFFFFFu;
    __syncthreads();

    // canonical order: the rank of each id among the cell's ids
    if (n > kBucketRankMin) {
      // Counting by buckets of the id value (monotone in the id, so the
      // rank is exact whatever the ids): the bucket's start plus the number
      // of smaller ids in the same bucket.  Bucket b holds the ids with
      // (id - lo) >> shift == b, shift chosen so that b < kRankBuckets.
      uint32_t lo = 0xFFFFFFFFu, hi = 0u;
      for (uint32_t j = lane; j < n; j += 64) {
        const uint32_t v = s_id[j];
        lo = min(lo, v);
        hi = max(hi, v);
      }
      lo = wave_min(lo);
      hi = wave_max(hi);
      const uint32_t bits = 32u - (uint32_t)__builtin_clz(hi - lo);  // hi > lo: ids differ
      const uint32_t shift = bits > 8u ? bits - 8u : 0u;
      uint32_t *const s_bkt = lds.bkt;
      uint32_t *const s_sorted = lds.sorted;
      for (uint32_t b = tid; b < kRankBuckets; b += kT) s_bkt[b] = 0u;
      if (tid == 0) s_bkt[kRankBuckets] = n;
      __syncthreads();
      for (uint32_t j = tid; j < n; j += kT) atomicAdd(&s_bkt[(s_id[j] - lo) >> shift], 1u);
      __syncthreads();
      if (wv == 0) {  // inclusive scan of the counts: s_bkt[b] = end of bucket b
        uint4 q = reinterpret_cast<uint4 *>(s_bkt)[lane];
        q.y += q.x;
        q.z += q.y;
        q.w += q.z;
        const uint32_t incl = wave_inclusive_sum(q.w);
        const uint32_t excl = incl - q.w;
        q.x += excl;
        q.y += excl;
        q.z += excl;
        q.w += excl;
        reinterpret_cast<uint4 *>(s_bkt)[lane] = q;
      }
      __syncthreads();
      // each bucket filled from its end: afterwards s_bkt[b] is its start
      for (uint32_t j = tid; j < n; j += kT) {
        const uint32_t v = s_id[j];
        const uint32_t pos = atomicSub(&s_bkt[(v - lo) >> shift], 1u) - 1u;
        s_sorted[pos] = v;
      }
      __syncthreads();
      for (uint32_t j = tid; j < n; j += kT) {
        const uint32_t me = s_id[j], b = (me - lo) >> shift;
        const uint32_t p1 = s_bkt[b + 1];
        uint32_t r = s_bkt[b];
        for (uint32_t p = r; p < p1; ++p) r += s_sorted[p] < me ? 1u : 0u;
        s_perm[r] = (uint16_t)j;
        if (kTrace && tr.perm) tr.perm[tr.offsets[cv.c] + r] = me;
      }
    } else {
      // at most kBucketRankMin < 64 particles: one per lane, counting all ids
      const uint4 *s_id4 = reinterpret_cast<const uint4 *>(s_id);
      static_assert(kBucketRankMin < 64, "one particle per lane");
      if (tid < n) {
        const uint32_t me = s_id[lane];
        uint32_t r = 0;
        for (uint32_t m = 0; m < n4 / 4; ++m) {
          const uint4 q = s_id4[m];
          r += (q.x < me) + (q.y < me) + (q.z < me) + (q.w < me);
        }
        s_perm[r] = (uint16_t)lane;
        if (kTrace && tr.perm) tr.perm[tr.offsets[cv.c] + r] = me;
      }
    }
    __syncthreads();
    if (cv.ov) {  // the members' slots, in LDS (the rank no longer needs it)
      for (uint32_t j = tid; j < n; j += kT) lds.sorted[j] = (uint32_t)cv.at_spill(j);
      __syncthreads();
    } else if (kMomInLds) {
      // the claim map (one byte a member, zero: not scattered), in the
      // rank's buckets; the barrier after the pair tests orders it
      for (uint32_t j = lane * 4u; j < n; j += 256u)
        *reinterpret_cast<uint32_t *>(s_cmap + j) = 0u;
    }

    // every pair k = 0 .. n(n-1)/2 - 1 (test_pairs), then the exact test
    // and the claims of the filtered ones in increasing k
    const uint32_t npairs = n * (n - 1u) / 2u;
    uint32_t nf = 0, claimed_bits = 0, n_acc = 0;
    if (kW == 1) __builtin_amdgcn_s_setprio(0);
    if (kW == 1) {
      if (pa.any)
        test_pairs<true, kTrace, true, kFilt>(0u, npairs, cv, pa, st, s_perm, s_filt, nf,
                                              s_claim, nclaim, claimed_bits, n_acc, tr,
                                              status);
      if (nf != 0)
        resolve_filtered<kTrace>(nf, cv, pa, st, s_perm, s_filt, s_claim, nclaim,
                                 claimed_bits, n_acc, tr, status);
      __syncthreads();
    } else {
      const uint32_t kh = npairs / 2u / 128u * 128u;
      if (wv == 0) {
        if (pa.any)
          test_pairs<true, false, false, kFilt>(0u, kh, cv, pa, st, s_perm, s_filt, nf,
                                                s_claim, nclaim, claimed_bits, n_acc, tr,
                                                status);
        if (nf != 0)
          resolve_filtered<false, false>(nf, cv, pa, st, s_perm, s_filt, s_claim, nclaim,
                                         claimed_bits, n_acc, tr, status);
        nf = 0;
      } else {
        uint32_t n1 = 0, k_resume = npairs;
        if (pa.any)
          k_resume = test_pairs<false, false, false, kCap / 2>(
              kh, npairs, cv, pa, st, s_perm, x2->filt, n1, s_claim, nclaim, claimed_bits,
              n_acc, tr, status);
        if (lane == 0) {
          x2->n_filt = n1;
          x2->k_resume = k_resume;
        }
      }
      __syncthreads();
      if (wv == 0) {
        const uint32_t n1 = x2->n_filt, k_resume = x2->k_resume;
        if (n1 != 0)
          resolve_filtered<false, false>(n1, cv, pa, st, s_perm, x2->filt, s_claim, nclaim,
                                         claimed_bits, n_acc, tr, status);
        if (k_resume < npairs) {
          test_pairs<true, false, false, kFilt>(k_resume, npairs, cv, pa, st, s_perm, s_filt,
                                                nf, s_claim, nclaim, claimed_bits, n_acc, tr,
                                                status);
          if (nf != 0)
            resolve_filtered<false, false>(nf, cv, pa, st, s_perm, s_filt, s_claim, nclaim,
                                           claimed_bits, n_acc, tr, status);
        }
        if (lane == 0) x2->nclaim = nclaim;
      }
      __syncthreads();
      nclaim = x2->nclaim;
    }

    if (kW == 1) __builtin_amdgcn_s_setprio(1);
    // work counters (spread over slots by cell against contention)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) n_acc += __shfl_down(n_acc, o);
    if (tid == 0) {
      const uint32_t slot = cv.c % kCounterSlots;
      atomicAdd(&status->pairs[slot], (unsigned long long)npairs);
      atomicAdd(&status->cand[slot], (unsigned long long)n_acc);
      atomicAdd(&status->claims[slot], (unsigned long long)nclaim);
    }

    // kinematics of the claimed pairs (disjoint: one writer per particle),
    // written back in place, or for the binning below into LDS; a fused
    // step then bins every particle
    mom_lds = kMomInLds && !cv.ov && nclaim <= kMomCap;
    for (uint32_t i0 = wv * 64u; i0 < nclaim; i0 += kT) {
      const uint32_t i = i0 + lane;
      const bool active = i < nclaim;
      double ax = 0, ay = 0, az = 0, bx = 0, by = 0, bz = 0;
      uint32_t ja = 0, jb = 0;
      if (active) {
        const uint32_t v = s_claim[i];
        const uint32_t a = (v >> 10) & 1023u, b = v & 1023u;
        const uint32_t k = row_start(a, n) + (b - a - 1u);
        const Words4 w = philox10(k, cv.c, t, 1u, pa.key0, pa.key1);
        const double uc = uniform53(w.w0, w.w1);
        const double uphi = uniform53(w.w2, w.w3);
        ja = s_perm[a];
        jb = s_perm[b];
        const size_t ia = cv.at(ja), ib = cv.at(jb);
        ax = st.px[ia];
        ay = st.py[ia];
        az = st.pz[ia];
        bx = st.px[ib];
        by = st.py[ib];
        bz = st.pz[ib];
        scatter_pair(ax, ay, az, bx, by, bz, uc, uphi);
        if (mom_lds) {
          s_mx[2u * i] = ax;
          s_my[2u * i] = ay;
          s_mz[2u * i] = az;
          s_mx[2u * i + 1u] = bx;
          s_my[2u * i + 1u] = by;
          s_mz[2u * i + 1u] = bz;
          s_cmap[ja] = (uint8_t)(2u * i + 1u);
          s_cmap[jb] = (uint8_t)(2u * i + 2u);
        } else {
          st.px[ia] = ax;
          st.py[ia] = ay;
          st.pz[ia] = az;
          st.px[ib] = bx;
          st.py[ib] = by;
          st.pz[ib] = bz;
        }
        if (kTrace && tr.claim) {
          const uint32_t slot = atomicAdd(&tr.counts[1], 1u);
          if (slot < tr.claim_cap) {
            tr.claim[3 * (size_t)slot + 0] = cv.c;
            tr.claim[3 * (size_t)slot + 1] = a;
            tr.claim[3 * (size_t)slot + 2] = b;
          } else {
            atomicOr(&status->err, kErrTrace);
          }
        }
      }
    }
    if (kFused || ob) __syncthreads();
  } else if (kTrace && n == 1 && tid == 0 && tr.perm) {
    tr.perm[tr.offsets[cv.c]] = st.id[cv.at_spill(0)];
  }

  if (kFused) {
    // stream and bin every particle (scattered momenta are in LDS or were
    // written back in place; the barrier above makes them visible to all
    // lanes).  The geometry is copied to registers once: read through a
    // reference it would be reloaded after every store.
    const Geometry g_l = g;
    double se = 0.0, sp = 0.0, sxx = 0.0;
    // the source cell's axis indices, for the direction of each move
    const uint32_t sy = (uint32_t)g_l.n[2], sx = (uint32_t)g_l.n[1] * sy;
    const int32_t cx = (int32_t)(cv.c / sx), cy = (int32_t)(cv.c % sx / sy),
                  cz = (int32_t)(cv.c % sy);
    uint32_t *const s_dir = lds.buf + (kW == 1 ? 0u : 64u * wv);  // the ids' dead buffer
    for (uint32_t j0 = wv * 64u; j0 < n; j0 += kT) {
      const uint32_t j = j0 + lane;
      const bool active = j < n;
      double x = 0, y = 0, z = 0, px = 0, py = 0, pz = 0;
      uint32_t id = 0, c2 = 0, dir = 13u;
      bool near = true;
      if (active) {
        const size_t o = cv.at(j);
        x = st.x[o];
        y = st.y[o];
        z = st.z[o];
        px = st.px[o];
        py = st.py[o];
        pz = st.pz[o];
        id = st.id[o];
        if (mom_lds) {
          const uint32_t m = s_cmap[j];
          if (m != 0u) {
            px = s_mx[m - 1u];
            py = s_my[m - 1u];
            pz = s_mz[m - 1u];
          }
        }
        if (ob) obs_add(px, py, pz, se, sp, sxx);
        advance<true>(g_l, x, y, z, px, py, pz);
        const int32_t ix = axis_index(x, g_l.dx[0], g_l.n[0]);
        const int32_t iy = axis_index(y, g_l.dx[1], g_l.n[1]);
        const int32_t iz = axis_index(z, g_l.dx[2], g_l.n[2]);
        c2 = (uint32_t)((ix * g_l.n[1] + iy) * g_l.n[2] + iz);
        const int32_t dx = ix - cx, dy = iy - cy, dz = iz - cz;
        // a move of less than a cell edge crosses at most one face per axis
        near = dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1 && dz >= -1 && dz <= 1;
        dir = near ? (uint32_t)(9 * (dx + 1) + 3 * (dy + 1) + (dz + 1)) : 13u;
      }
      if (__ballot(!near) == 0ull) {
        const uint32_t slot = neighbour_fetch_add(dst.count, cv.c, sx, sy, dir, active, s_dir);
        store_at_slot(dst, c2, slot, active, x, y, z, px, py, pz, id, status);
      } else {
        append(dst, c2, active, x, y, z, px, py, pz, id, status);
      }
    }
    if (tid == 0) src.count[cv.c] = 0u;
    if (ob) obs_write_wave(ob, cv.c, n, se, sp, sxx);
  } else if (ob) {
    double se = 0.0, sp = 0.0, sxx = 0.0;
    for (uint32_t j = lane; j < n; j += 64u) {
      const size_t o = cv.at(j);
      obs_add(st.px[o], st.py[o], st.pz[o], se, sp, sxx);
    }
    obs_write_wave(ob, cv.c, n, se, sp, sxx);
  }
}

// ---------------------------------------------------------------------------
// Small cells: one wave takes 64 / G consecutive cells, G lanes per cell and
// one particle per lane.  A lane loads its particle once and keeps it in
// registers through collisions, streaming and binning, so a sparse cell
// costs one load round trip and one slot atomic instead of a wave of its own
// with several dependent round trips.
// ---------------------------------------------------------------------------
struct SmallLds {
  __align__(16) uint32_t id[64];  // by lane (the cell's storage order)
  double x[64], y[64], z[64];     // by lane
  double px[64], py[64], pz[64];  // by group and canonical rank
};

template <uint32_t G>
using ClaimMask = typename std::conditional<(G == 64), uint64_t, uint32_t>::type;

// Collisions of the cells c0 .. c_end - 1 (at most 64 / G) of src at step t.
// The canonical rank of each particle is counted over its cell's ids in
// LDS, where the momenta are then stored in canonical order (and the
// positions by lane, so that no particle state stays live in registers
// through the pair loop).  Pairs k = gl, gl + G, ... of each cell are tested
// as in cell_step (Philox w1 filter, then the exact Eq. (3) test in the same
// lane); a cell's accepted pairs of one round appear in its bits of the
// wave's ballot in increasing k, so the greedy claim walks those bits in
// order, with the cell's claimed set kept identically by all its lanes.
// Both lanes of a claimed pair evaluate its kinematics (same inputs, same
// code, hence the same result) and keep their own half.  kFused: every lane
// then streams and bins its particle into dst for step t+1.  Cells holding
// more than G particles are left alone; the result has bit grp G set for
// each such cell c0 + grp.
template <bool kFused, bool kTrace, uint32_t G>
__device__ __forceinline__ uint64_t small_cells_step(const GCells &src, const GCells &dst,
                                                     uint32_t c0, uint32_t c_end,
                                                     uint32_t t, const PairArgs &pa,
                                                     const Geometry &g, DevStatus *status,
                                                     const TraceArgs &tr, SmallLds &lds,
                                                     double *obs = nullptr) {
  static_assert(G == 8 || G == 16 || G == 32 || G == 64, "lanes per cell");
  constexpr uint32_t kNone = 0xFFFFFFFFu;
  const uint32_t lane = lane_id();
  const uint32_t grp = lane / G, gl = lane % G;
  const uint32_t c = c0 + grp;
  const bool in_range = c < c_end;
  if (c0 == 0 && lane == 0) clear_idle_scratch(src, t);
  // overflowing cells are left to the kernel for larger cells
  const uint32_t cnt = in_range ? src.count[c] : 0u;
  const bool overflowing = cnt > src.cap;
  const uint32_t n = overflowing ? 0u : cnt;
  const bool small = in_range && !overflowing && n <= G;
  const bool mine = small && gl < n;
  const size_t o = (size_t)c * src.cap + gl;
  __syncthreads();  // a previous call's readers of lds are done
  {
    uint32_t id = kNone;  // ids are below 2^32 - 1, so kNone ranks after all
    if (mine) {
      lds.x[lane] = src.st.x[o];
      lds.y[lane] = src.st.y[o];
      lds.z[lane] = src.st.z[o];
      id = src.st.id[o];
    }
    lds.id[lane] = id;
  }
  double qx = 0, qy = 0, qz = 0;
  if (mine) {
    qx = src.st.px[o];
    qy = src.st.py[o];
    qz = src.st.pz[o];
  }
  __syncthreads();
  uint32_t r = 0;
  if (mine) {
    const uint32_t id = lds.id[lane];
    const uint4 *q4 = reinterpret_cast<const uint4 *>(lds.id + grp * G);
#pragma unroll
    for (uint32_t m = 0; m < G / 4; ++m) {
      const uint4 q = q4[m];
      r += (q.x < id) + (q.y < id) + (q.z < id) + (q.w < id);
    }
    lds.px[grp * G + r] = qx;
    lds.py[grp * G + r] = qy;
    lds.pz[grp * G + r] = qz;
    if (kTrace && tr.perm) tr.perm[tr.offsets[c] + r] = id;
  }
  __syncthreads();

  const double *const spx = lds.px + grp * G;
  const double *const spy = lds.py + grp * G;
  const double *const spz = lds.pz + grp * G;
  const uint32_t npairs = small ? n * (n - 1u) / 2u : 0u;
  ClaimMask<G> claimed = 0;  // the cell's claimed canonical indices
  uint32_t partner = kNone, kpair = 0, n_acc = 0;
  if (pa.any) {
    for (uint32_t k0 = 0; __ballot(k0 < npairs) != 0; k0 += G) {
      const uint32_t k = k0 + gl;
      bool acc = false;
      if (k < npairs && philox10_w1(k, c, t, 0u, pa.key0, pa.key1) <= pa.w1_max) {
        const Words4 w = philox10(k, c, t, 0u, pa.key0, pa.key1);
        uint32_t a, b;
        pair_of_index(k, n, a, b);
        acc = uniform53(w.w0, w.w1) <
              p22(spx[a], spy[a], spz[a], spx[b], spy[b], spz[b], pa.kfac);
        if (kTrace && acc && tr.cand) {
          const uint32_t slot = atomicAdd(&tr.counts[0], 1u);
          if (slot < tr.cand_cap) {
            tr.cand[3 * (size_t)slot + 0] = c;
            tr.cand[3 * (size_t)slot + 1] = a;
            tr.cand[3 * (size_t)slot + 2] = b;
          } else {
            atomicOr(&status->err, kErrTrace);
          }
        }
      }
      n_acc += acc ? 1u : 0u;
      uint64_t seg = __ballot(acc);
      if (G < 64) seg = (seg >> (grp * G)) & ((1ull << (G % 64)) - 1ull);
      while (seg != 0) {
        const uint32_t kk = k0 + (uint32_t)__builtin_ctzll(seg);
        seg &= seg - 1ull;
        uint32_t a, b;
        pair_of_index(kk, n, a, b);
        const ClaimMask<G> ab = ((ClaimMask<G>)1 << a) | ((ClaimMask<G>)1 << b);
        if ((claimed & ab) == 0) {
          claimed |= ab;
          if (mine && (r == a || r == b)) {
            partner = r == a ? b : a;
            kpair = kk;
          }
          if (kTrace && tr.claim && gl == 0) {
            const uint32_t slot = atomicAdd(&tr.counts[1], 1u);
            if (slot < tr.claim_cap) {
              tr.claim[3 * (size_t)slot + 0] = c;
              tr.claim[3 * (size_t)slot + 1] = a;
              tr.claim[3 * (size_t)slot + 2] = b;
            } else {
              atomicOr(&status->err, kErrTrace);
            }
          }
        }
      }
    }
  }

  // work counters of the wave's cells, in one slot
  const bool scat = partner != kNone;
  {
    uint32_t cnt_pairs = small && gl == 0 ? npairs : 0u;
    uint32_t cnt_claims = scat && r < partner ? 1u : 0u;
#pragma unroll
    for (int s = 32; s > 0; s >>= 1) {
      cnt_pairs += __shfl_down(cnt_pairs, s);
      n_acc += __shfl_down(n_acc, s);
      cnt_claims += __shfl_down(cnt_claims, s);
    }
    if (lane == 0 && cnt_pairs != 0) {
      const uint32_t slot = c0 % kCounterSlots;
      atomicAdd(&status->pairs[slot], (unsigned long long)cnt_pairs);
      atomicAdd(&status->cand[slot], (unsigned long long)n_acc);
      atomicAdd(&status->claims[slot], (unsigned long long)cnt_claims);
    }
  }

  double px = 0, py = 0, pz = 0;
  if (mine) {
    px = spx[r];
    py = spy[r];
    pz = spz[r];
  }
  if (scat) {
    const bool lo = r < partner;
    const uint32_t a = lo ? r : partner, b = lo ? partner : r;
    const Words4 w = philox10(kpair, c, t, 1u, pa.key0, pa.key1);
    double ax = spx[a], ay = spy[a], az = spz[a];
    double bx = spx[b], by = spy[b], bz = spz[b];
    scatter_pair(ax, ay, az, bx, by, bz, uniform53(w.w0, w.w1), uniform53(w.w2, w.w3));
    px = lo ? ax : bx;
    py = lo ? ay : by;
    pz = lo ? az : bz;
    if (!kFused) {
      src.st.px[o] = px;
      src.st.py[o] = py;
      src.st.pz[o] = pz;
    }
  }

  if (obs) {  // the cell's sums over its G lanes, written by its first lane
    double se = 0.0, sp = 0.0, sxx = 0.0;
    if (mine) obs_add(px, py, pz, se, sp, sxx);
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) {
      se += __shfl_xor(se, o);
      sp += __shfl_xor(sp, o);
      sxx += __shfl_xor(sxx, o);
    }
    if (small && gl == 0) {
      double *const out = obs + kCellSums * (size_t)c;
      out[0] = se;
      out[1] = sp;
      out[2] = sxx;
      out[3] = (double)n;
    }
  }
  if (kFused) {
    double x = 0, y = 0, z = 0;
    uint32_t id = 0, c2 = 0;
    if (mine) {
      x = lds.x[lane];
      y = lds.y[lane];
      z = lds.z[lane];
      id = lds.id[lane];
      advance<true>(g, x, y, z, px, py, pz);
      c2 = cell_id(g, x, y, z);
    }
    append(dst, c2, mine, x, y, z, px, py, pz, id, status);
    if (small && gl == 0) src.count[c] = 0u;
  }
  return __ballot(in_range && !small && !overflowing && gl == 0);
}

// The cells among c0 .. c_end - 1 (at most 64) holding more than `lanes`
// particles, stepped one after another by the whole wave: the cells that a
// small-cell launch with that many lanes per cell left alone (lanes = 0:
// every non-empty cell).  A separate launch, so that each kernel keeps the
// registers of its own path (the small-cell kernel runs at twice the
// occupancy of the wave-per-cell code).
template <bool kFused, bool kTrace, uint32_t kCap>
__device__ __forceinline__ void large_cells_step(const GCells &src, const GCells &dst,
                                                 uint32_t c0, uint32_t c_end, uint32_t lanes,
                                                 uint32_t t, const PairArgs &pa,
                                                 const Geometry &g, DevStatus *status,
                                                 const TraceArgs &tr,
                                                 CellLds<kFused, kCap> &lds,
                                                 double *obs = nullptr) {
  const uint32_t c = c0 + lane_id();
  const uint32_t n = c < c_end ? src.count[c] : 0u;
  // the cells the small-cell kernel leaves: more particles than lanes, or
  // overflowing (more than the block holds)
  uint64_t big = __ballot(n > lanes || n > src.cap);
  while (big != 0) {
    const uint32_t l = (uint32_t)__builtin_ctzll(big);
    big &= big - 1ull;
    cell_step<kFused, kTrace, kCap>(src, dst, c0 + l, t, pa, g, status, tr, lds, nullptr, obs);
  }
}

template <bool kFused, bool kTrace, uint32_t G>
__global__ __launch_bounds__(64) void k_step_small(Cells src_arg, Cells dst_arg, uint32_t n_cells,
                                                   uint32_t t, PairArgs pa, Geometry g,
                                                   DevStatus *status, TraceArgs tr) {
  const GCells src = binning(to_global(src_arg), t);
  const GCells dst = binning(to_global(dst_arg), t + 1u);
  __shared__ SmallLds lds;
  constexpr uint32_t kPer = 64 / G;
  const uint32_t c0 = xcd_runs<8>(blockIdx.x, gridDim.x) * kPer;
  const uint32_t c_end = c0 + kPer < n_cells ? c0 + kPer : n_cells;
  (void)small_cells_step<kFused, kTrace, G>(src, dst, c0, c_end, t, pa, g, status, tr, lds);
}

// ---------------------------------------------------------------------------
// Packed cells: a wave takes a tile of 64 consecutive cells and packs whole
// cells, in cell order, into units of at most 64 particles, one particle per
// lane (a unit ends before the cell that would not fit).  So a sparse box
// steps with few idle lanes whatever its mix of occupancies, where a fixed
// number of lanes per cell idles most of them in its emptier cells.  Each
// unit:
//   1. loads its particles (a lane each), ids and positions into LDS;
//   2. ranks each id among its cell's ids and stores the momentum at the
//      canonical position (cell start + rank);
//   3. tests each cell's pairs k = i, i + n, i + 2n, ... in its n lanes with
//      the Philox w1 filter, appending the passing ones to an LDS list (in
//      increasing k per cell);
//   4. in rows of 64 list entries: the exact Eq. (3) test, one entry a
//      lane, then the greedy claims of the row's accepted pairs in list
//      order, with the claimed flags of all canonical positions in one
//      wave-uniform mask (a row is resolved early when the list nears full,
//      which keeps each cell's claims in increasing k);
//   5. computes the kinematics of each claimed pair in both of its lanes
//      (same inputs and code, so the same result) and keeps its half;
//   6. fused: streams and bins every particle; else writes the scattered
//      momenta back.
// Cells holding more than 64 particles, or more than their block holds,
// are left to the kernel for larger cells.
// ---------------------------------------------------------------------------
constexpr uint32_t kPackedMax = 64;    // particles of a unit, and of a cell it takes
constexpr uint32_t kPackedFilt = 256;  // filtered pairs held before a row is resolved

struct PackedLds {
  __align__(16) uint32_t id[64];   // by lane: the unit's particles, cell by cell
  double x[64], y[64], z[64];      // by lane
  double px[64], py[64], pz[64];   // by canonical position
  uint32_t filt[kPackedFilt];      // filtered pairs: tile cell << 16 | k
  uint32_t incl[64];               // by tile cell: inclusive prefix of the packed counts
  uint32_t start[64], cnt[64];     // by tile cell: first lane, particles
  uint32_t partner[64];            // by canonical position: the claimed partner's
};

// Exact test and claims of filt[i0 .. i0 + 63] (< nf), in list order.
template <bool kTrace>
__device__ __forceinline__ void packed_resolve_row(
    uint32_t i0, uint32_t nf, uint32_t c0, uint32_t t, const PairArgs &pa, PackedLds &lds,
    uint64_t &claimed, uint32_t &nclaim, uint32_t &n_acc, const TraceArgs &tr,
    DevStatus *status) {
  const uint32_t lane = lane_id();
  const uint32_t i = i0 + lane;
  bool acc = false;
  uint32_t v = 0;
  if (i < nf) {
    const uint32_t e = lds.filt[i];
    const uint32_t cl = e >> 16, k = e & 0xFFFFu;
    const uint32_t n = lds.cnt[cl], st = lds.start[cl];
    const Words4 w = philox10(k, c0 + cl, t, 0u, pa.key0, pa.key1);
    uint32_t a, b;
    pair_of_index(k, n, a, b);
    acc = uniform53(w.w0, w.w1) < p22(lds.px[st + a], lds.py[st + a], lds.pz[st + a],
                                      lds.px[st + b], lds.py[st + b], lds.pz[st + b],
                                      pa.kfac);
    v = (st + a) << 8 | (st + b);
    if (kTrace && acc && tr.cand) {
      const uint32_t slot = atomicAdd(&tr.counts[0], 1u);
      if (slot < tr.cand_cap) {
        tr.cand[3 * (size_t)slot + 0] = c0 + cl;
        tr.cand[3 * (size_t)slot + 1] = a;
        tr.cand[3 * (size_t)slot + 2] = b;
      } else {
        atomicOr(&status->err, kErrTrace);
      }
    }
  }
  n_acc += acc ? 1u : 0u;
  for (uint64_t m = __ballot(acc); m != 0; m &= m - 1ull) {
    const uint32_t l = (uint32_t)__builtin_ctzll(m);
    const uint32_t vl = (uint32_t)__builtin_amdgcn_readlane((int)v, (int)l);
    const uint32_t pa_ = vl >> 8, pb_ = vl & 0xFFu;
    const uint64_t ab = (1ull << pa_) | (1ull << pb_);
    if ((claimed & ab) == 0) {
      claimed |= ab;
      if (lane == 0) {
        lds.partner[pa_] = pb_;
        lds.partner[pb_] = pa_;
      }
      ++nclaim;
      if (kTrace && tr.claim && lane == l) {
        const uint32_t e = lds.filt[i];
        const uint32_t cl = e >> 16, st = lds.start[cl];
        const uint32_t slot = atomicAdd(&tr.counts[1], 1u);
        if (slot < tr.claim_cap) {
          tr.claim[3 * (size_t)slot + 0] = c0 + cl;
          tr.claim[3 * (size_t)slot + 1] = pa_ - st;
          tr.claim[3 * (size_t)slot + 2] = pb_ - st;
        } else {
          atomicOr(&status->err, kErrTrace);
        }
      }
    }
  }
}

template <bool kFused, bool kTrace>
__device__ __forceinline__ void packed_cells_step(const GCells &src, const GCells &dst,
                                                  uint32_t c0, uint32_t n_cells, uint32_t t,
                                                  const PairArgs &pa, const Geometry &g,
                                                  DevStatus *status, const TraceArgs &tr,
                                                  PackedLds &lds) {
  // wave priority as in cell_step: the filter loop at the base priority,
  // the latency-bound rest of a unit above it
  __builtin_amdgcn_s_setprio(1);
  constexpr uint32_t kNone = 0xFFFFFFFFu;
  const uint32_t lane = lane_id();
  const uint64_t below = (1ull << lane) - 1ull;
  if (c0 == 0 && lane == 0) clear_idle_scratch(src, t);
  // the tile's cells, one a lane; overflowing and larger cells are left out
  const uint32_t cc = c0 + lane;
  const uint32_t ccnt = cc < n_cells ? src.count[cc] : 0u;
  const bool packed = cc < n_cells && ccnt <= kPackedMax && ccnt <= src.cap;
  const uint32_t nl = packed ? ccnt : 0u;
  const uint32_t incl = wave_inclusive_sum(nl);  // inclusive prefix of the packed counts
  const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
  uint32_t cnt_pairs = 0, n_acc = 0, n_claims = 0;
  for (uint32_t base = 0; base < total;) {
    // the unit: the cells whose particles end within base + 64 (a prefix of
    // the tile's lanes beyond the previous unit; each cell fits alone)
    const uint64_t fit = __ballot(incl <= base + kPackedMax);
    const uint32_t e = 63u - (uint32_t)__builtin_clzll(fit);
    const uint32_t end = (uint32_t)__builtin_amdgcn_readlane((int)incl, (int)e);
    const uint32_t p = end - base;  // particles of the unit
    const bool in_unit = nl > 0 && incl - nl >= base && lane <= e;
    wave_lds_sync();  // the previous unit's readers of lds are done
    lds.incl[lane] = incl;
    if (in_unit) {
      lds.start[lane] = incl - nl - base;
      lds.cnt[lane] = nl;
      cnt_pairs += nl * (nl - 1u) / 2u;
    }
    wave_lds_sync();
    // each lane's cell: the first tile cell whose particles end beyond it
    // (binary search of the inclusive prefix)
    const bool mine = lane < p;
    uint32_t cl = 0;
    {
      const uint32_t key = base + lane;
      uint32_t lo = 0, hi = 63;  // first index with incl > key, in [lo, hi]
      for (int it = 0; it < 6; ++it) {
        const uint32_t mid = (lo + hi) / 2u;
        if (lds.incl[mid] > key) hi = mid; else lo = mid + 1u;
      }
      cl = mine ? lo : 0u;
    }
    const uint32_t st = mine ? lds.start[cl] : 0u;
    const uint32_t n = mine ? lds.cnt[cl] : 0u;
    const uint32_t gl = lane - st;
    const uint32_t c = c0 + cl;
    {
      uint32_t id = kNone;
      if (mine) {
        const size_t o = (size_t)c * src.cap + gl;
        lds.x[lane] = src.st.x[o];
        lds.y[lane] = src.st.y[o];
        lds.z[lane] = src.st.z[o];
        lds.px[lane] = src.st.px[o];  // by lane until ranked
        lds.py[lane] = src.st.py[o];
        lds.pz[lane] = src.st.pz[o];
        id = src.st.id[o];
      }
      lds.id[lane] = id;
    }
    wave_lds_sync();
    // canonical rank among the cell's ids; the momenta move to their
    // canonical positions
    uint32_t pos;
    {
      const uint32_t id = lds.id[lane];
      const uint32_t maxn = wave_max(n);
      uint32_t r = 0;
      for (uint32_t m = 0; m < maxn; ++m)
        if (m < n) r += lds.id[st + m] < id ? 1u : 0u;
      pos = st + r;
      const double qx = lds.px[lane], qy = lds.py[lane], qz = lds.pz[lane];
      wave_lds_sync();
      if (mine) {
        lds.px[pos] = qx;
        lds.py[pos] = qy;
        lds.pz[pos] = qz;
        if (kTrace && tr.perm) tr.perm[tr.offsets[c] + r] = id;
      }
    }
    wave_lds_sync();

    // pair tests, the w1 filter first, in passes that fill the list; then
    // the exact test and claims of the list by rows
    uint64_t claimed = 0;
    uint32_t nclaim = 0;
    if (pa.any) {
      const uint32_t npairs = n * (n - 1u) / 2u;
      uint32_t k = gl;
      while (__ballot(k < npairs) != 0) {
        uint32_t nf = 0;
        __builtin_amdgcn_s_setprio(0);
        do {
          const bool pass = k < npairs &&
                            philox10_w1(k, c, t, 0u, pa.key0, pa.key1) <= pa.w1_max;
          const uint64_t mk = __ballot(pass);
          if (pass) lds.filt[nf + (uint32_t)__popcll(mk & below)] = cl << 16 | k;
          nf += (uint32_t)__popcll(mk);
          k += n;
        } while (nf <= kPackedFilt - 64u && __ballot(k < npairs) != 0);
        __builtin_amdgcn_s_setprio(1);
        wave_lds_sync();
        for (uint32_t i0 = 0; i0 < nf; i0 += 64u)
          packed_resolve_row<kTrace>(i0, nf, c0, t, pa, lds, claimed, nclaim, n_acc, tr,
                                     status);
        wave_lds_sync();
      }
    }
    n_claims += nclaim;

    // kinematics of the claimed pairs, in both lanes of each
    double px = lds.px[pos], py = lds.py[pos], pz = lds.pz[pos];
    const bool scat = mine && ((claimed >> pos) & 1ull) != 0;
    if (scat) {
      const uint32_t other = lds.partner[pos];
      const bool lo = pos < other;
      const uint32_t A = lo ? pos : other, B = lo ? other : pos;
      const uint32_t ra = A - st, rb = B - st;
      const uint32_t k = row_start(ra, n) + (rb - ra - 1u);
      const Words4 w = philox10(k, c, t, 1u, pa.key0, pa.key1);
      double ax = lds.px[A], ay = lds.py[A], az = lds.pz[A];
      double bx = lds.px[B], by = lds.py[B], bz = lds.pz[B];
      scatter_pair(ax, ay, az, bx, by, bz, uniform53(w.w0, w.w1), uniform53(w.w2, w.w3));
      px = lo ? ax : bx;
      py = lo ? ay : by;
      pz = lo ? az : bz;
      if (!kFused) {
        const size_t o = (size_t)c * src.cap + gl;
        src.st.px[o] = px;
        src.st.py[o] = py;
        src.st.pz[o] = pz;
      }
    }
    if (kFused) {
      double x = 0, y = 0, z = 0;
      uint32_t c2 = 0, id = 0;
      if (mine) {
        const Geometry g_l = g;
        x = lds.x[lane];
        y = lds.y[lane];
        z = lds.z[lane];
        id = lds.id[lane];
        advance<true>(g_l, x, y, z, px, py, pz);
        c2 = cell_id(g_l, x, y, z);
      }
      append(dst, c2, mine, x, y, z, px, py, pz, id, status);
    }
    base = end;
  }
  // work counters of the tile, in one slot; the packed cells' counts
  // cleared for the buffer's next use
#pragma unroll
  for (int s = 32; s > 0; s >>= 1) {
    cnt_pairs += __shfl_down(cnt_pairs, s);
    n_acc += __shfl_down(n_acc, s);
  }
  if (lane == 0 && cnt_pairs != 0) {
    const uint32_t slot = c0 % kCounterSlots;
    atomicAdd(&status->pairs[slot], (unsigned long long)cnt_pairs);
    atomicAdd(&status->cand[slot], (unsigned long long)n_acc);
    atomicAdd(&status->claims[slot], (unsigned long long)n_claims);
  }
  if (kFused && packed) src.count[cc] = 0u;
}

// dst is src shifted by dst_shift bytes and g is read from device memory
// where the binning uses it (as for k_step: fewer values held through the
// loops).  Five waves per SIMD: the compiler's choice (4, 101-104 VGPRs)
// made the 32^3 fm^3 set's fused step 5 % slower, six (80 VGPRs, 12
// spilled) 4 %.
template <bool kFused, bool kTrace>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(5))) void k_step_packed(
    Cells src_arg, int64_t dst_shift, uint32_t n_cells, uint32_t t, PairArgs pa,
    const Geometry *__restrict__ gp, DevStatus *status, TraceArgs tr) {
  const GCells src = binning(to_global(src_arg), t);
  __shared__ PackedLds lds;
  const uint32_t c0 = xcd_runs<8>(blockIdx.x, gridDim.x) * 64u;
  packed_cells_step<kFused, kTrace>(src, dst_of(src, dst_shift, t), c0, n_cells, t, pa, *gp,
                                    status, tr, lds);
}

// One wave per 64 consecutive cells: the cells holding more than `lanes`
// particles.
template <bool kFused, bool kTrace, uint32_t kCap>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void k_step_large(
    Cells src_arg, Cells dst_arg, uint32_t n_cells,
                                                   uint32_t lanes, uint32_t t, PairArgs pa,
                                                   Geometry g, DevStatus *status,
                                                   TraceArgs tr) {
  const GCells src = binning(to_global(src_arg), t);
  const GCells dst = binning(to_global(dst_arg), t + 1u);
  __shared__ CellLds<kFused, kCap> lds;
  const uint32_t c0 = blockIdx.x * 64u;
  const uint32_t c_end = c0 + 64u < n_cells ? c0 + 64u : n_cells;
  large_cells_step<kFused, kTrace, kCap>(src, dst, c0, c_end, lanes, t, pa, g, status, tr,
                                         lds);
}

// One wave per cell, for the cells holding more than `lanes` particles: the
// oversize-cell launch when such cells are common (a wave that scans 64 of
// them would step them one after another).
template <bool kFused, bool kTrace, uint32_t kCap>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(cell_waves<kCap>()))) void k_step_over(
    Cells src_arg, int64_t dst_shift,
                                                  uint32_t lanes, uint32_t t, PairArgs pa,
                                                  const Geometry *__restrict__ gp,
                                                  DevStatus *status, TraceArgs tr) {
  const GCells src = binning(to_global(src_arg), t);
  __shared__ CellLds<kFused, kCap> lds;
  const uint32_t c = xcd_runs<8>(blockIdx.x, gridDim.x);
  const uint32_t cnt = src.count[c];
  if (cnt <= lanes && cnt <= src.cap) return;
  cell_step<kFused, kTrace, kCap>(src, dst_of(src, dst_shift, t), c, t, pa, *gp, status, tr,
                                  lds);
}

// dst is src shifted by dst_shift bytes (the two buffers of a context are
// laid out alike), and g is read from device memory where the binning uses
// it: as kernel arguments both would be loaded at entry and held through the
// pair loop, which spills scalar registers into vector lanes and reloads them
// in the loop.  Derived from src, the dst pointers stay known to address
// global memory.
template <bool kFused, bool kTrace, uint32_t kCap>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(cell_waves<kCap>()))) void k_step(
    Cells src_arg, int64_t dst_shift, uint32_t t,
                                             PairArgs pa, const Geometry *__restrict__ gp,
                                             DevStatus *status, TraceArgs tr) {
  const GCells src = binning(to_global(src_arg), t);
  __shared__ CellLds<kFused, kCap> lds;
  cell_step<kFused, kTrace, kCap>(src, dst_of(src, dst_shift, t),
                                  xcd_runs<8>(blockIdx.x, gridDim.x), t, pa, *gp, status, tr,
                                  lds);
}

// Two waves per cell (a workgroup of 128): half the pair tests each, so a
// box of few cells has twice as many, shorter waves to spread over the
// SIMDs (the tail of a launch whose waves are long and few is idle time).
template <bool kFused, uint32_t kCap>
__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(cell_waves<kCap>()))) void k_step2(
    Cells src_arg, int64_t dst_shift, uint32_t t,
                                               PairArgs pa, const Geometry *__restrict__ gp,
                                               DevStatus *status) {
  const GCells src = binning(to_global(src_arg), t);
  __shared__ CellLds<kFused, kCap> lds;
  __shared__ SecondWaveLds<kCap> x2;
  cell_step<kFused, false, kCap, 2>(src, dst_of(src, dst_shift, t),
                                    xcd_runs<8>(blockIdx.x, gridDim.x), t, pa, *gp, status,
                                    TraceArgs{}, lds, &x2);
}


// ---------------------------------------------------------------------------
// Batched steps: all live events of a batch advance together.  Each kernel
// has a work space in which the events are laid out one after another
// (space_begin[e] = the first unit of event e, ascending from 0):
//   items   cpi consecutive cells, for the binning (every event); a wave
//           takes items with a grid stride, so a grid smaller than the item
//           count is a persistent launch;
//   chunks  64 / lanes cells, one wave each, for the small cells of events
//           with lanes per cell > 0;
//   scans   64 cells, one wave each, stepping the cells of those events that
//           hold more particles than the event's lanes per cell;
//   cells   one cell per wave, for events stepped one wave per cell.
// The step kernels have no loop over units: a loop keeps the descriptor and
// lane constants live across iterations, which costs registers and with
// them the occupancy that hides memory latency.  Within a run of k steps,
// launch j (0: stream + bin, 1..k-1: fused, k: collisions only) reads buffer
// cur ^ (j & 1) of each event and uses step index t + j - 1; the run ends
// with k_batch_advance.
// ---------------------------------------------------------------------------
// The event of `unit` in a work space: the number of entries of begin[]
// that are <= unit, minus one (begin[] is ascending from 0; an event with
// no units has the begin of the next one, so it is never the answer).  Each
// lane counts the entries lane, lane + 64, ... (independent loads, no
// cross-lane step inside the loop, so they are all in flight together),
// then the wave sums the counts.  `unit` must be the same in every lane of
// the wave; so is the result.
__device__ __forceinline__ uint32_t find_event(const uint32_t *__restrict__ begin,
                                               uint32_t n_events, uint32_t unit) {
  uint32_t count = 0;
#pragma unroll 4
  for (uint32_t e = lane_id(); e < n_events; e += 64) count += begin[e] <= unit ? 1u : 0u;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) count += (uint32_t)__shfl_xor((int)count, o);
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)count) - 1u;
}

// The event's fields for launch j of a run, loaded once into registers (the
// kernels store to global memory, so fields read through the table would
// be reloaded after every store).
struct EventView {
  GCells src, dst;
  Geometry g;
  PairArgs pa;
  DevStatus *status;
  uint32_t t, lanes, n_cells;
};

__device__ __forceinline__ EventView event_view(const BatchEvent *__restrict__ E, uint32_t j) {
  EventView v;
  if ((E->cur ^ (j & 1u)) == 0u) {
    v.src = to_global(E->buf[0]);
    v.dst = to_global(E->buf[1]);
  } else {
    v.src = to_global(E->buf[1]);
    v.dst = to_global(E->buf[0]);
  }
  v.g = E->g;
  v.pa = E->pa;
  v.status = E->status;
  v.t = E->t + j - 1u;
  v.src = binning(v.src, v.t);
  v.dst = binning(v.dst, v.t + 1u);
  v.lanes = E->lanes;
  v.n_cells = E->n_cells;
  return v;
}

// Where launch j of a run writes the event's observation sums: its per-cell
// sums array if the step the launch collides (t + j - 1) ends an
// observation interval, else nowhere.
__device__ __forceinline__ double *obs_target(const BatchEvent *__restrict__ E, uint32_t j) {
  const uint32_t every = E->obs_every;
  return every != 0u && (E->t + j) % every == 0u ? E->obs_sums : nullptr;
}

__global__ __launch_bounds__(kBlock) void k_batch_bin(const BatchEvent *__restrict__ ev,
                                                      const uint32_t *__restrict__ item_begin,
                                                      uint32_t n_events, uint32_t n_items) {
  const uint32_t w = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);  // wave-uniform
  for (uint32_t item = blockIdx.x * kCellsPerBlock + w; item < n_items;
       item += gridDim.x * kCellsPerBlock) {
    const BatchEvent *__restrict__ E = ev + find_event(item_begin, n_events, item);
    GCells src, dst;
    if (E->cur == 0u) {
      src = to_global(E->buf[0]);
      dst = to_global(E->buf[1]);
    } else {
      src = to_global(E->buf[1]);
      dst = to_global(E->buf[0]);
    }
    src = binning(src, E->t - 1u);
    dst = binning(dst, E->t);
    if (item == E->item_begin && lane_id() == 0) clear_idle_spill_set(src);
    const Geometry g = E->g;
    DevStatus *const status = E->status;
    const uint32_t cpi = E->cpi, n_cells = E->n_cells, lanes = E->lanes;
    const uint32_t c0 = (item - E->item_begin) * cpi;
    const uint32_t c1 = c0 + cpi < n_cells ? c0 + cpi : n_cells;
    switch (lanes) {
      case 8:
        for (uint32_t c = c0; c < c1; c += 8) cells_stream_bin<8>(src, dst, c, c1, g, status, nullptr);
        break;
      case 16:
        for (uint32_t c = c0; c < c1; c += 4) cells_stream_bin<16>(src, dst, c, c1, g, status, nullptr);
        break;
      case 32:
        for (uint32_t c = c0; c < c1; c += 2) cells_stream_bin<32>(src, dst, c, c1, g, status, nullptr);
        break;
      default:
        for (uint32_t c = c0; c < c1; ++c) cells_stream_bin<64>(src, dst, c, c + 1, g, status, nullptr);
    }
  }
}

// Small cells: one wave per chunk of 64 / lanes cells.
template <bool kFused>
__global__ __launch_bounds__(64) void k_batch_step_small(const BatchEvent *__restrict__ ev,
                                                         const uint32_t *__restrict__ chunk_begin,
                                                         uint32_t n_events, uint32_t j) {
  __shared__ SmallLds lds;
  const uint32_t chunk = xcd_runs<8>(blockIdx.x, gridDim.x);
  const BatchEvent *__restrict__ E = ev + find_event(chunk_begin, n_events, chunk);
  const EventView v = event_view(E, j);
  const uint32_t per = 64u / v.lanes;
  const uint32_t c0 = (chunk - E->chunk_begin) * per;
  const uint32_t c1 = c0 + per < v.n_cells ? c0 + per : v.n_cells;
  const TraceArgs none{};
  double *const obs = obs_target(E, j);
  switch (v.lanes) {
    case 8:
      small_cells_step<kFused, false, 8>(v.src, v.dst, c0, c1, v.t, v.pa, v.g, v.status, none, lds,
                                         obs);
      break;
    case 16:
      small_cells_step<kFused, false, 16>(v.src, v.dst, c0, c1, v.t, v.pa, v.g, v.status, none,
                                          lds, obs);
      break;
    case 32:
      small_cells_step<kFused, false, 32>(v.src, v.dst, c0, c1, v.t, v.pa, v.g, v.status, none,
                                          lds, obs);
      break;
    default:
      small_cells_step<kFused, false, 64>(v.src, v.dst, c0, c1, v.t, v.pa, v.g, v.status, none,
                                          lds, obs);
  }
}

// The cells of 64 consecutive cells of a small-cell event holding more than
// its lanes per cell (rare), by the whole wave.
template <bool kFused, uint32_t kCap>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void k_batch_step_scan(
    const BatchEvent *__restrict__ ev,
                                                        const uint32_t *__restrict__ scan_begin,
                                                        uint32_t n_events, uint32_t j) {
  __shared__ CellLds<kFused, kCap> lds;
  const uint32_t unit = blockIdx.x;
  const BatchEvent *__restrict__ E = ev + find_event(scan_begin, n_events, unit);
  const EventView v = event_view(E, j);
  const uint32_t c0 = (unit - E->scan_begin) * 64u;
  const uint32_t c1 = c0 + 64u < v.n_cells ? c0 + 64u : v.n_cells;
  large_cells_step<kFused, false, kCap>(v.src, v.dst, c0, c1, v.lanes, v.t, v.pa, v.g,
                                        v.status, TraceArgs{}, lds, obs_target(E, j));
}

// One wave per cell of the events stepped one wave per cell.  Held to the
// register budget of 5 waves per SIMD, as the plain kernel (it fits without
// scratch; the event lookup would otherwise push it 1 register over).
template <bool kFused, uint32_t kCap>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(cell_waves<kCap>()))) void k_batch_step_cells(
    const BatchEvent *__restrict__ ev,
                                                         const uint32_t *__restrict__ cell_begin,
                                                         uint32_t n_events, uint32_t j) {
  __shared__ CellLds<kFused, kCap> lds;
  const uint32_t unit = xcd_runs<8>(blockIdx.x, gridDim.x);
  const BatchEvent *__restrict__ E = ev + find_event(cell_begin, n_events, unit);
  // dst is src shifted by the distance between the event's two buffers
  // (laid out alike), g is read by reference from the table where the
  // binning uses it (see k_step)
  const uint32_t s = (E->cur ^ (j & 1u)) & 1u;
  const uint32_t t = E->t + j - 1u;
  const GCells src = binning(to_global(E->buf[s]), t);
  const int64_t shift = (const char *)E->buf[s ^ 1u].st.x - (const char *)E->buf[s].st.x;
  const PairArgs pa = E->pa;
  cell_step<kFused, false, kCap>(src, dst_of(src, shift, t), unit - E->cell_begin, t,
                                 pa, E->g, E->status, TraceArgs{}, lds, nullptr,
                                 obs_target(E, j));
}



// End of a run of k steps: every event moved k buffers and k step indices.
__global__ void k_batch_advance(BatchEvent *ev, uint32_t n_events, uint32_t k) {
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n_events) {
    ev[e].cur ^= (k & 1u);
    ev[e].t += k;
  }
}

// ---------------------------------------------------------------------------
// Observe: per-cell sums of E and p_x (one wave per cell), then per-slab
// sums over the slab's cells in cell order.  Slab ix is the contiguous cell
// range [ix ny nz, (ix+1) ny nz).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_observe_cells(Cells cur_arg, uint32_t n_cells,
                                                          double *cell_sums,
                                                          uint32_t binning_step) {
  const GCells cur = binning(to_global(cur_arg), binning_step);
  const uint32_t lane = lane_id();
  const uint32_t c = blockIdx.x * kCellsPerBlock + threadIdx.x / 64;
  if (c >= n_cells) return;
  const uint32_t cnt = cur.count[c];
  const uint32_t n = occupancy(cur, c);
  const size_t base = (size_t)c * cur.cap;
  double se = 0.0, sp = 0.0, sxx = 0.0;
  for (uint32_t j = lane; j < n; j += 64) {
    const double px = cur.st.px[base + j], py = cur.st.py[base + j],
                 pz = cur.st.pz[base + j];
    const double e = norm3(px, py, pz);
    se += e;
    sp += px;
    sxx += (px * px) / e;
  }
  if (cnt > cur.cap) {  // overflowing: its spilled members, in spill order
    const SpillDesc *const spl = cur.sp;
    const uint32_t ns = min(spl->hdr[2u * cur.q], spl->capacity);
    for (uint32_t i = lane; i < ns; i += 64) {
      if (spl->cell[i] != c) continue;
      const size_t o = spl->base + i;
      const double px = cur.st.px[o], py = cur.st.py[o], pz = cur.st.pz[o];
      const double e = norm3(px, py, pz);
      se += e;
      sp += px;
      sxx += (px * px) / e;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    se += __shfl_down(se, o);
    sp += __shfl_down(sp, o);
    sxx += __shfl_down(sxx, o);
  }
  if (lane == 0) {
    double *const out = cell_sums + kCellSums * (size_t)c;
    out[0] = se;
    out[1] = sp;
    out[2] = sxx;
    out[3] = (double)cnt;
  }
}

// The rest frame (Landau frame of the t-x block of T^{mu nu}) of a slab:
// T^mu_nu u^nu = e u^mu, u = gamma (1, v), in the order the determinism
// contract fixes (a product of two factors under the square root).
__device__ __forceinline__ void rest_frame(double t00, double t0x, double txx, double &e,
                                           double &v) {
  const double a = t00 + txx;
  const double b = 2.0 * __builtin_fabs(t0x);
  double disc = (a - b) * (a + b);
  if (disc < 0.0) disc = 0.0;
  e = ((t00 - txx) + __builtin_sqrt(disc)) / 2.0;
  const double den = e + txx;
  v = den > 0.0 ? t0x / den : 0.0;
}

// Slab ix's sums over its cells in cell order, then the moments (a
// workgroup of kBlock threads).
__device__ __forceinline__ void slab_moments(const double *cell_sums, uint32_t cells_per_slab,
                                             double vol, uint32_t ix, const SlabOut &out) {
  __shared__ double s_sum[kCellSums][kBlock / 64];
  const size_t c0 = (size_t)ix * cells_per_slab;
  double acc[kCellSums] = {0.0, 0.0, 0.0, 0.0};
  for (uint32_t j = threadIdx.x; j < cells_per_slab; j += kBlock)
#pragma unroll
    for (uint32_t k = 0; k < kCellSums; ++k) acc[k] += cell_sums[kCellSums * (c0 + j) + k];
#pragma unroll
  for (uint32_t k = 0; k < kCellSums; ++k)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc[k] += __shfl_down(acc[k], o);
  const uint32_t lane = lane_id(), wave = threadIdx.x / 64;
  if (lane == 0)
#pragma unroll
    for (uint32_t k = 0; k < kCellSums; ++k) s_sum[k][wave] = acc[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot[kCellSums];
#pragma unroll
    for (uint32_t k = 0; k < kCellSums; ++k) {
      tot[k] = 0.0;
      for (int w = 0; w < kBlock / 64; ++w) tot[k] += s_sum[k][w];
    }
    const double t00 = tot[0] / vol, t0x = tot[1] / vol, txx = tot[2] / vol;
    if (out.T00) out.T00[ix] = t00;
    if (out.T0x) out.T0x[ix] = t0x;
    if (out.Txx) out.Txx[ix] = txx;
    if (out.n) out.n[ix] = tot[3] / vol;
    if (out.e || out.v) {
      double e, v;
      rest_frame(t00, t0x, txx, e, v);
      if (out.e) out.e[ix] = e;
      if (out.v) out.v[ix] = v;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_observe_slabs(const double *cell_sums,
                                                          uint32_t cells_per_slab,
                                                          double vol, SlabOut out) {
  slab_moments(cell_sums, cells_per_slab, vol, blockIdx.x, out);
}

// The slabs of the events observed after launch j of a run: block (ix,
// event) sums slab ix of an event due for an observation (its cells' sums,
// written by the launch) into T00 and T0x of the observation's row.
__global__ __launch_bounds__(kBlock) void k_batch_observe(const BatchEvent *__restrict__ ev,
                                                          uint32_t n_events, uint32_t j) {
  const uint32_t e = blockIdx.y;
  if (e >= n_events) return;
  const BatchEvent *__restrict__ E = ev + e;
  const uint32_t every = E->obs_every;
  if (every == 0u || (E->t + j) % every != 0u) return;
  const uint32_t nx = (uint32_t)E->g.n[0];
  if (blockIdx.x >= nx) return;
  const uint32_t row = ((E->t + j) / every) % E->obs_rows;
  double *const out = E->obs_out + (size_t)row * 2u * nx;
  SlabOut o{};
  o.T00 = out;
  o.T0x = out + nx;
  slab_moments(E->obs_sums, (uint32_t)(E->g.n[1] * E->g.n[2]), E->obs_vol, blockIdx.x, o);
}

__global__ __launch_bounds__(kBlock) void k_gather_by_id(Cells cur_arg, uint32_t n_cells,
                                                         double *x, double *y, double *z,
                                                         double *px, double *py,
                                                         double *pz, uint32_t binning_step) {
  const GCells cur = binning(to_global(cur_arg), binning_step);
  const uint32_t lane = lane_id();
  const uint32_t c = blockIdx.x * kCellsPerBlock + threadIdx.x / 64;
  if (c >= n_cells) return;
  const uint32_t n = occupancy(cur, c);
  const size_t base = (size_t)c * cur.cap;
  for (uint32_t j = lane; j < n; j += 64) {
    const uint32_t id = cur.st.id[base + j];
    x[id] = cur.st.x[base + j];
    y[id] = cur.st.y[base + j];
    z[id] = cur.st.z[base + j];
    px[id] = cur.st.px[base + j];
    py[id] = cur.st.py[base + j];
    pz[id] = cur.st.pz[base + j];
  }
  if (cur.count[c] > cur.cap) {  // overflowing: its spilled members
    const SpillDesc *const spl = cur.sp;
    const uint32_t ns = min(spl->hdr[2u * cur.q], spl->capacity);
    for (uint32_t i = lane; i < ns; i += 64) {
      if (spl->cell[i] != c) continue;
      const size_t o = spl->base + i;
      const uint32_t id = cur.st.id[o];
      x[id] = cur.st.x[o];
      y[id] = cur.st.y[o];
      z[id] = cur.st.z[o];
      px[id] = cur.st.px[o];
      py[id] = cur.st.py[o];
      pz[id] = cur.st.pz[o];
    }
  }
}

inline unsigned grid_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }
inline unsigned cell_blocks(int64_t n_cells) {
  return (unsigned)((n_cells + kCellsPerBlock - 1) / kCellsPerBlock);
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
void launch_fill_u32(uint32_t *p, uint32_t v, int64_t count, hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(count)), dim3(kBlock), 0, s, p, v, count);
}

void launch_store_f64(double *p, double v, hipStream_t s) {
  hipLaunchKernelGGL(k_store_f64, dim3(1), dim3(64), 0, s, p, v);
}

bool launch_write_bytes(void *dst, const void *src, size_t bytes, hipStream_t s) {
  if (bytes % 4 != 0 || bytes > sizeof(WriteWords) || ((uintptr_t)dst & 3u) != 0) return false;
  WriteWords v{};
  __builtin_memcpy(v.w, src, bytes);
  hipLaunchKernelGGL(k_write_words, dim3(1), dim3(64), 0, s, (uint32_t *)dst, v,
                     (uint32_t)(bytes / 4));
  return true;
}

namespace {

// A kernel launch that records the stage-timing events ev_start / ev_stop on
// its own dispatch when given (no event packets between launches, and the
// events read the kernel's duration), else a plain launch.
template <typename K, typename... Args>
void launch_timed(K kernel, dim3 grid, dim3 block, hipStream_t s, hipEvent_t ev_start,
                  hipEvent_t ev_stop, Args... args) {
  if (ev_start)
    hipExtLaunchKernelGGL(kernel, grid, block, 0, s, ev_start, ev_stop, 0u, args...);
  else
    hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
}

// A timed stage that launches nothing still records its events.
void record_empty(hipEvent_t ev_start, hipEvent_t ev_stop, hipStream_t s) {
  if (ev_start) (void)hipEventRecord(ev_start, s);
  if (ev_stop) (void)hipEventRecord(ev_stop, s);
}

}  // namespace

void launch_init_bin(const double *x, const double *y, const double *z,
                     const double *px, const double *py, const double *pz,
                     const Cells &dst, int64_t n, const Geometry &g, DevStatus *st,
                     uint32_t binning_step, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_init_bin, dim3(grid_for(n)), dim3(kBlock), 0, s, x, y, z, px, py,
                     pz, dst, n, g, st, binning_step);
}

void launch_stream_bin(const Cells &src, const Cells &dst, int64_t n_cells, uint32_t lanes,
                       const Geometry &g, DevStatus *status, uint32_t *trace_cell,
                       uint32_t t, hipStream_t s, hipEvent_t ev_start, hipEvent_t ev_stop) {
  if (n_cells <= 0) {
    record_empty(ev_start, ev_stop, s);
    return;
  }
  // (packed cells: 16 lanes a cell; a stream-bin that packs 64 particles
  // a round whatever their cells measured the same on the 32^3 fm^3 set,
  // whose sparse cells' cost is their partly used cache lines)
  const uint32_t G = lanes == 0 || lanes == kTwoWavesPerCell ? 64u
                     : lanes == kPackedCells                 ? 16u
                                                             : lanes;
  const int64_t waves = (n_cells + 64 / G - 1) / (64 / G);
  const dim3 grid(cell_blocks(waves)), block(kBlock);
  const uint32_t nc = (uint32_t)n_cells;
  switch (G) {
    case 8:
      launch_timed(k_stream_bin<8>, grid, block, s, ev_start, ev_stop, src, dst, nc, g, status,
                   trace_cell, t);
      break;
    case 16:
      launch_timed(k_stream_bin<16>, grid, block, s, ev_start, ev_stop, src, dst, nc, g, status,
                   trace_cell, t);
      break;
    case 32:
      launch_timed(k_stream_bin<32>, grid, block, s, ev_start, ev_stop, src, dst, nc, g, status,
                   trace_cell, t);
      break;
    default:
      launch_timed(k_stream_bin<64>, grid, block, s, ev_start, ev_stop, src, dst, nc, g, status,
                   trace_cell, t);
  }
}

void launch_offsets(const Cells &cur, uint32_t *offsets, uint32_t *tile_sums,
                    int64_t n_cells, hipStream_t s) {
  const unsigned tiles = (unsigned)((n_cells + kScanTile - 1) / kScanTile);
  hipLaunchKernelGGL(k_scan_tiles, dim3(tiles), dim3(kBlock), 0, s, cur, offsets,
                     tile_sums, n_cells);
  hipLaunchKernelGGL(k_scan_carry, dim3(tiles), dim3(kBlock), 0, s, offsets,
                     (const uint32_t *)tile_sums, n_cells);
}

namespace {

// fork: work queued on s so far precedes the work then queued on side
void fork(hipStream_t s, const SideStream *side) {
  if (!side) return;
  (void)hipEventRecord(side->fork, s);
  (void)hipStreamWaitEvent(side->stream, side->fork, 0);
}

// join: the work queued on side precedes the work then queued on s
void join(hipStream_t s, const SideStream *side) {
  if (!side) return;
  (void)hipEventRecord(side->join, side->stream);
  (void)hipStreamWaitEvent(s, side->join, 0);
}

template <bool kFused, bool kTrace, uint32_t kCap>
void launch_step_cap(const Cells &src, const Cells &dst, uint32_t n_cells, uint32_t lanes,
                     uint32_t t, const PairArgs &pa, const Geometry &g, DevStatus *status,
                     const TraceArgs &tr, hipStream_t s, const SideStream *side,
                     const StepDevice &dev) {
  const dim3 block(64);
  const int64_t shift = (int64_t)((const char *)dst.st.x - (const char *)src.st.x);
  // one kernel: timing events ride on its dispatch (no packets of their own
  // between launches)
  if (lanes == kTwoWavesPerCell && !kTrace) {
    launch_timed(k_step2<kFused, kCap>, dim3(n_cells), dim3(128), s, dev.ev_start, dev.ev_stop,
                 src, shift, t, pa, dev.g, status);
    return;
  }
  if (lanes == 0 || lanes == kTwoWavesPerCell) {
    launch_timed(k_step<kFused, kTrace, kCap>, dim3(n_cells), block, s, dev.ev_start,
                 dev.ev_stop, src, shift, t, pa, dev.g, status, tr);
    return;
  }
  // the small cells and, concurrently, the cells the small-cell kernel
  // leaves alone (disjoint cells; both append to dst through atomics); timed
  // by events recorded around the whole launch
  if (dev.ev_start) (void)hipEventRecord(dev.ev_start, s);
  fork(s, side);
  const uint32_t per = lanes == kPackedCells ? 64u : 64u / lanes;  // cells per wave
  const dim3 grid((n_cells + per - 1) / per);
  // the particles above which a cell goes to the second kernel
  const uint32_t thr = lanes == kPackedCells ? kPackedMax : lanes;
  switch (lanes) {
    case kPackedCells:
      hipLaunchKernelGGL((k_step_packed<kFused, kTrace>), grid, block, 0, s, src,
                         (int64_t)((const char *)dst.st.x - (const char *)src.st.x), n_cells, t,
                         pa, dev.g, status, tr);
      break;
    case 8:
      hipLaunchKernelGGL((k_step_small<kFused, kTrace, 8>), grid, block, 0, s, src, dst,
                         n_cells, t, pa, g, status, tr);
      break;
    case 16:
      hipLaunchKernelGGL((k_step_small<kFused, kTrace, 16>), grid, block, 0, s, src, dst,
                         n_cells, t, pa, g, status, tr);
      break;
    case 32:
      hipLaunchKernelGGL((k_step_small<kFused, kTrace, 32>), grid, block, 0, s, src, dst,
                         n_cells, t, pa, g, status, tr);
      break;
    default:
      hipLaunchKernelGGL((k_step_small<kFused, kTrace, 64>), grid, block, 0, s, src, dst,
                         n_cells, t, pa, g, status, tr);
  }
  hipStream_t so = side ? side->stream : s;
  if (dev.over_span == 1)
    hipLaunchKernelGGL((k_step_over<kFused, kTrace, kCap>), dim3(n_cells), block, 0, so, src,
                       (int64_t)((const char *)dst.st.x - (const char *)src.st.x), thr, t,
                       pa, dev.g, status, tr);
  else
    hipLaunchKernelGGL((k_step_large<kFused, kTrace, kCap>), dim3((n_cells + 63) / 64), block,
                       0, so, src, dst, n_cells, thr, t, pa, g, status, tr);
  join(s, side);
  if (dev.ev_stop) (void)hipEventRecord(dev.ev_stop, s);
}

template <uint32_t kCap>
void launch_step_any(const Cells &src, const Cells &dst, bool fused, uint32_t n_cells,
                     uint32_t lanes, uint32_t t, const PairArgs &pa, const Geometry &g,
                     DevStatus *status, const TraceArgs *trace, hipStream_t s,
                     const SideStream *side, const StepDevice &dev) {
  if (trace)
    launch_step_cap<false, true, kCap>(src, dst, n_cells, lanes, t, pa, g, status, *trace, s,
                                       side, dev);
  else if (fused)
    launch_step_cap<true, false, kCap>(src, dst, n_cells, lanes, t, pa, g, status,
                                       TraceArgs{}, s, side, dev);
  else
    launch_step_cap<false, false, kCap>(src, dst, n_cells, lanes, t, pa, g, status,
                                        TraceArgs{}, s, side, dev);
}

}  // namespace

void launch_step(const Cells &src, const Cells &dst, bool fused, int64_t n_cells,
                 uint32_t lanes, uint32_t t, const PairArgs &pa, const Geometry &g,
                 DevStatus *status, const TraceArgs *trace, hipStream_t s,
                 const SideStream *side, const StepDevice &dev) {
  if (n_cells <= 0) {
    record_empty(dev.ev_start, dev.ev_stop, s);
    return;
  }
  // cells of at most 512 slots use the kernels with half the LDS
  if (src.cap <= kSmallCap)
    launch_step_any<kSmallCap>(src, dst, fused, (uint32_t)n_cells, lanes, t, pa, g, status,
                               trace, s, side, dev);
  else
    launch_step_any<kCellCap>(src, dst, fused, (uint32_t)n_cells, lanes, t, pa, g, status,
                              trace, s, side, dev);
}

namespace {

__global__ __launch_bounds__(kBlock) void k_count_cells(const double *__restrict__ x,
                                                        const double *__restrict__ y,
                                                        const double *__restrict__ z,
                                                        int64_t n, Geometry g,
                                                        uint32_t *count) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double a = x[i], b = y[i], c = z[i];
    if (__builtin_isfinite(a) && __builtin_isfinite(b) && __builtin_isfinite(c))
      atomicAdd(&count[cell_id(g, a, b, c)], 1u);
  }
}

__global__ __launch_bounds__(kBlock) void k_max_u32(const uint32_t *__restrict__ v, int64_t n,
                                                    uint32_t *out) {
  uint32_t m = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    m = max(m, v[i]);
  m = wave_max(m);
  if (lane_id() == 0) atomicMax(out, m);
}

}  // namespace

void launch_count_cells(const double *x, const double *y, const double *z, int64_t n,
                        const Geometry &g, int64_t n_cells, uint32_t *count,
                        uint32_t *max_count, hipStream_t s) {
  launch_fill_u32(count, 0u, n_cells, s);
  launch_fill_u32(max_count, 0u, 1, s);
  if (n > 0) {
    const unsigned grid = grid_for(n) < 4096u ? grid_for(n) : 4096u;
    hipLaunchKernelGGL(k_count_cells, dim3(grid), dim3(kBlock), 0, s, x, y, z, n, g, count);
  }
  const unsigned grid = grid_for(n_cells) < 1024u ? grid_for(n_cells) : 1024u;
  hipLaunchKernelGGL(k_max_u32, dim3(grid), dim3(kBlock), 0, s, (const uint32_t *)count,
                     n_cells, max_count);
}

void launch_occupancy_over(const Cells &cur, int64_t n_cells, DevStatus *status,
                           hipStream_t s) {
  if (n_cells <= 0) return;
  const unsigned grid = grid_for(n_cells) < 1024u ? grid_for(n_cells) : 1024u;
  hipLaunchKernelGGL(k_occupancy_over, dim3(grid), dim3(kBlock), 0, s, cur,
                     (uint32_t)n_cells, status->over);
}

void launch_observe(const Cells &cur, const Geometry &g, double vol, double *cell_sums,
                    const SlabOut &out, uint32_t binning_step, hipStream_t s) {
  const int64_t n_cells = (int64_t)g.n[0] * g.n[1] * g.n[2];
  hipLaunchKernelGGL(k_observe_cells, dim3(cell_blocks(n_cells)), dim3(kBlock), 0, s, cur,
                     (uint32_t)n_cells, cell_sums, binning_step);
  hipLaunchKernelGGL(k_observe_slabs, dim3((unsigned)g.n[0]), dim3(kBlock), 0, s,
                     (const double *)cell_sums, (uint32_t)(g.n[1] * g.n[2]), vol, out);
}

void launch_batch_run(BatchEvent *ev, const BatchSpaces &sp, uint32_t n_events, int32_t k,
                      uint32_t persistent_waves, hipStream_t s, const SideStream *side,
                      void (*between)(void *, int), void *ctx, const uint8_t *obs_at) {
  if (n_events == 0 || sp.n_items == 0 || k <= 0) return;
  const uint32_t bin_waves =
      persistent_waves > 0 && persistent_waves < sp.n_items ? persistent_waves : sp.n_items;
  const uint32_t bin_grid = (bin_waves + kCellsPerBlock - 1) / kCellsPerBlock;
  const BatchEvent *cev = ev;
  const dim3 wave(64);
  if (between) between(ctx, 0);
  hipLaunchKernelGGL(k_batch_bin, dim3(bin_grid), dim3(kBlock), 0, s, cev, sp.item_begin,
                     n_events, sp.n_items);
  // launch j: the small cells on s; concurrently on the side stream the
  // cells of events stepped one wave per cell, then the oversize cells of
  // small-cell events (all disjoint cells; appends go through atomics)
  auto step = [&](auto fused, uint32_t j) {
    constexpr bool kF = decltype(fused)::value;
    const bool both =
        sp.n_chunks > 0 && (sp.n_cells[0] > 0 || sp.n_cells[1] > 0 || sp.n_scans > 0);
    const SideStream *sd = both ? side : nullptr;
    const hipStream_t s2 = sd ? sd->stream : s;
    fork(s, sd);
    if (sp.n_chunks > 0)
      hipLaunchKernelGGL((k_batch_step_small<kF>), dim3(sp.n_chunks), wave, 0, s, cev,
                         sp.chunk_begin, n_events, j);
    if (sp.n_cells[0] > 0)
      hipLaunchKernelGGL((k_batch_step_cells<kF, kSmallCap>), dim3(sp.n_cells[0]), wave, 0, s2,
                         cev, sp.cell_begin[0], n_events, j);
    if (sp.n_cells[1] > 0)
      hipLaunchKernelGGL((k_batch_step_cells<kF, kCellCap>), dim3(sp.n_cells[1]), wave, 0, s2,
                         cev, sp.cell_begin[1], n_events, j);
    if (sp.n_scans > 0) {
      if (sp.scan_large)
        hipLaunchKernelGGL((k_batch_step_scan<kF, kCellCap>), dim3(sp.n_scans), wave, 0, s2,
                           cev, sp.scan_begin, n_events, j);
      else
        hipLaunchKernelGGL((k_batch_step_scan<kF, kSmallCap>), dim3(sp.n_scans), wave, 0, s2,
                           cev, sp.scan_begin, n_events, j);
    }
    join(s, sd);
    // the events due for an observation after this launch
    if (sp.obs_nx > 0 && (!obs_at || obs_at[j]))
      hipLaunchKernelGGL(k_batch_observe, dim3(sp.obs_nx, n_events), dim3(kBlock), 0, s, cev,
                         n_events, j);
  };
  using Fused = std::integral_constant<bool, true>;
  using Last = std::integral_constant<bool, false>;
  for (int32_t j = 1; j < k; ++j) {
    if (between) between(ctx, 1);
    step(Fused{}, (uint32_t)j);
  }
  if (between) between(ctx, 2);
  step(Last{}, (uint32_t)k);
  if (between) between(ctx, -1);
  hipLaunchKernelGGL(k_batch_advance, dim3((n_events + 63) / 64), dim3(64), 0, s, ev,
                     n_events, (uint32_t)k);
}

void launch_gather_by_id(const Cells &cur, int64_t n_cells, double *x, double *y,
                         double *z, double *px, double *py, double *pz,
                         uint32_t binning_step, hipStream_t s) {
  if (n_cells <= 0) return;
  hipLaunchKernelGGL(k_gather_by_id, dim3(cell_blocks(n_cells)), dim3(kBlock), 0, s, cur,
                     (uint32_t)n_cells, x, y, z, px, py, pz, binning_step);
}

}  // namespace cuba
