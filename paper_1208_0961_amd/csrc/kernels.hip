// kernels.hip -- gfx950 kernels of the PIC Boltzmann step (arXiv:1208.0961).
//
// Per step, on the structure-of-arrays state kept in cell order:
//   count    stream + reflect each particle in registers, find its new cell,
//            count cells with wave-aggregated atomics        (HBM: 48 B read)
//   scan     exclusive prefix sum of the cell counts -> offsets and cursors
//   scatter  stream + reflect again (bit-identical), claim a slot in the new
//            cell, write the particle there                  (HBM: 52 B + 52 B)
//   collide  one wave64 per cell: ids to LDS, canonical (id) order by rank
//            counting, all n(n-1)/2 pair tests spread over the lanes with a
//            Philox block each, ballot-compaction of the pairs that can pass,
//            exact Eq. (3) test on those, greedy claim in pair order, then
//            the CM-frame kinematics of the claimed pairs   (ALU bound)
// plus the observe pass (slab sums of E and p_x) and state export by id.
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace cuba {

namespace {

constexpr int kBlock = 256;
constexpr uint32_t kFiltCap = 512;  // filtered pairs held before resolving

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Slot = old value of ctr[key] + rank of this lane among the active lanes
// of its wave with the same key.  The lanes are grouped by key with ballots
// first (ALU only); then every group leader issues its atomic in the same
// instruction, so the wave waits for one atomic round trip, not one per key.
__device__ __forceinline__ uint32_t aggregated_fetch_add(uint32_t *ctr, uint32_t key,
                                                         bool active) {
  const uint32_t lane = lane_id();
  const uint64_t below = (1ull << lane) - 1ull;
  uint32_t leader = lane, rank = 0, size = 0;
  uint64_t todo = __ballot(active);
  while (todo != 0) {
    const int l = __builtin_ctzll(todo);
    const uint32_t lkey = __shfl(key, l);
    const uint64_t group = __ballot(active && key == lkey);
    if (active && key == lkey) {
      leader = (uint32_t)l;
      rank = (uint32_t)__popcll(group & below);
      size = (uint32_t)__popcll(group);
    }
    todo &= ~group;
  }
  uint32_t base = 0;
  if (active && leader == lane) base = atomicAdd(&ctr[key], size);
  base = __shfl(base, (int)leader);
  return base + rank;
}

// Count-only variant: the leaders add their group sizes (no value returned).
__device__ __forceinline__ void aggregated_add(uint32_t *ctr, uint32_t key, bool active) {
  const uint32_t lane = lane_id();
  uint32_t leader = lane, size = 0;
  uint64_t todo = __ballot(active);
  while (todo != 0) {
    const int l = __builtin_ctzll(todo);
    const uint32_t lkey = __shfl(key, l);
    const uint64_t group = __ballot(active && key == lkey);
    if (active && key == lkey) {
      leader = (uint32_t)l;
      size = (uint32_t)__popcll(group);
    }
    todo &= ~group;
  }
  if (active && leader == lane) atomicAdd(&ctr[key], size);
}

// Workgroups are dispatched round-robin over the 8 XCDs of the MI355X
// (workgroup b runs on XCD b mod 8), each XCD with its own L2.
constexpr uint32_t kXcds = 8;

// Bijection on [0, nblocks) giving each XCD runs of kRun consecutive logical
// blocks, interleaved over the XCDs (balances work that varies along the
// block range while keeping neighbouring blocks on one L2).
template <uint32_t kRun>
__device__ __forceinline__ uint32_t xcd_runs(uint32_t b, uint32_t nblocks) {
  constexpr uint32_t kSuper = kXcds * kRun;
  const uint32_t full = nblocks / kSuper * kSuper;
  if (b >= full) return b;
  const uint32_t s = b / kSuper, r = b % kSuper;
  return s * kSuper + (r % kXcds) * kRun + r / kXcds;
}

__global__ __launch_bounds__(kBlock) void k_fill_u32(uint32_t *p, uint32_t v,
                                                     int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < count) p[i] = v;
}

__global__ __launch_bounds__(kBlock) void k_load(
    const double *__restrict__ x, const double *__restrict__ y,
    const double *__restrict__ z, const double *__restrict__ px,
    const double *__restrict__ py, const double *__restrict__ pz, SoA dst,
    int64_t n, Geometry g, DevStatus *status) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double a = x[i], b = y[i], c = z[i], qa = px[i], qb = py[i], qc = pz[i];
  dst.x[i] = a;
  dst.y[i] = b;
  dst.z[i] = c;
  dst.px[i] = qa;
  dst.py[i] = qb;
  dst.pz[i] = qc;
  dst.id[i] = (uint32_t)i;
  const bool ok = __builtin_isfinite(a) && __builtin_isfinite(b) &&
                  __builtin_isfinite(c) && __builtin_isfinite(qa) &&
                  __builtin_isfinite(qb) && __builtin_isfinite(qc) && a >= 0.0 &&
                  a <= g.L[0] && b >= 0.0 && b <= g.L[1] && c >= 0.0 &&
                  c <= g.L[2] && norm3(qa, qb, qc) > 0.0;
  if (!ok) atomicOr(&status->err, kErrRange);
}

template <bool kStream>
__global__ __launch_bounds__(kBlock) void k_count(SoA src, int64_t n, Geometry g,
                                                  uint32_t *counts) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const bool active = i < n;
  uint32_t c = 0;
  if (active) {
    double x = src.x[i], y = src.y[i], z = src.z[i];
    double px = src.px[i], py = src.py[i], pz = src.pz[i];
    advance<kStream>(g, x, y, z, px, py, pz);
    c = cell_id(g, x, y, z);
  }
  aggregated_add(counts, c, active);
}

template <bool kStream>
__global__ __launch_bounds__(kBlock) void k_scatter(SoA src, SoA dst, int64_t n,
                                                    Geometry g, uint32_t *cursor,
                                                    uint32_t *trace_cell) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const bool active = i < n;
  double x = 0, y = 0, z = 0, px = 0, py = 0, pz = 0;
  uint32_t id = 0, c = 0;
  if (active) {
    x = src.x[i];
    y = src.y[i];
    z = src.z[i];
    px = src.px[i];
    py = src.py[i];
    pz = src.pz[i];
    id = src.id[i];
    advance<kStream>(g, x, y, z, px, py, pz);
    c = cell_id(g, x, y, z);
  }
  const uint32_t slot = aggregated_fetch_add(cursor, c, active);
  if (active) {
    dst.x[slot] = x;
    dst.y[slot] = y;
    dst.z[slot] = z;
    dst.px[slot] = px;
    dst.py[slot] = py;
    dst.pz[slot] = pz;
    dst.id[slot] = id;
    if (trace_cell) trace_cell[id] = c;
  }
}

// Tile-local exclusive scan of counts (kScanTile per block, 8 per thread);
// clears the counts for the next step.
__global__ __launch_bounds__(kBlock) void k_scan_tiles(uint32_t *counts,
                                                       uint32_t *offsets,
                                                       uint32_t *tile_sums,
                                                       int64_t n_cells) {
  __shared__ uint32_t s_wave[kBlock / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * 8;
  const uint32_t lane = lane_id(), wave = threadIdx.x / 64;
  uint32_t v[8];
  uint32_t sum = 0;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int64_t idx = base + j;
    const uint32_t cnt = idx < n_cells ? counts[idx] : 0u;
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
    if (idx < n_cells) {
      offsets[idx] = excl + v[j];
      counts[idx] = 0u;
    }
  }
  if (threadIdx.x == kBlock - 1) tile_sums[blockIdx.x] = wave_off + incl;
}

// Adds the sum of all earlier tiles; copies the offsets into the cursors.
__global__ __launch_bounds__(kBlock) void k_scan_carry(uint32_t *offsets,
                                                       uint32_t *cursor,
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
    if (idx < n_cells) {
      const uint32_t o = offsets[idx] + carry;
      offsets[idx] = o;
      cursor[idx] = o;
    }
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0)
    offsets[n_cells] = carry + tile_sums[blockIdx.x];
}

// ---------------------------------------------------------------------------
// Collisions: one wave64 (one workgroup) per cell.
// ---------------------------------------------------------------------------
struct CellView {
  uint32_t c, n, base, t;
};

// Exact Eq. (3) test of the nf filtered pairs in s_filt (increasing pair
// index), then greedy claim in that order.  Entries are rewritten as
// flag | a << 10 | b.  claimed_bits holds, per lane, the claimed flags of
// canonical indices lane + 64 j.
template <bool kTrace>
__device__ __forceinline__ void resolve_filtered(
    uint32_t nf, const CellView &cv, const PairArgs &pa, const SoA &st,
    const uint16_t *s_perm, uint32_t *s_filt, uint32_t *s_claim,
    uint32_t &nclaim, uint32_t &claimed_bits, uint32_t &n_acc,
    const TraceArgs &tr, DevStatus *status) {
  const uint32_t lane = lane_id();
  __syncthreads();
  for (uint32_t i = lane; i < nf; i += 64) {
    const uint32_t k = s_filt[i];
    const Words4 w = philox10(k, cv.c, cv.t, 0u, pa.key0, pa.key1);
    const double u = uniform53(w.w0, w.w1);
    uint32_t a, b;
    pair_of_index(k, cv.n, a, b);
    const uint32_t ia = cv.base + s_perm[a], ib = cv.base + s_perm[b];
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
  __syncthreads();
  for (uint32_t i = 0; i < nf; ++i) {
    const uint32_t v = s_filt[i];
    if (v & 0x80000000u) {
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
  __syncthreads();
}

template <bool kTrace>
__global__ __launch_bounds__(64) void k_collide(const uint32_t *__restrict__ offsets,
                                                SoA st, uint32_t t, PairArgs pa,
                                                DevStatus *status, TraceArgs tr) {
  // s_buf holds the cell's ids while the canonical order is built; after
  // that its first half holds the filtered pairs and its second half the
  // claimed pairs.
  __shared__ __align__(16) uint32_t s_buf[kCellCap];
  __shared__ uint16_t s_perm[kCellCap];
  static_assert(kFiltCap + kCellCap / 2 <= kCellCap, "LDS aliasing");
  uint32_t *const s_id = s_buf;
  uint32_t *const s_filt = s_buf;
  uint32_t *const s_claim = s_buf + kFiltCap;

  const uint32_t lane = lane_id();
  CellView cv;
  cv.c = xcd_runs<8>(blockIdx.x, gridDim.x);
  cv.t = t;
  cv.base = offsets[cv.c];
  cv.n = offsets[cv.c + 1] - cv.base;
  const uint32_t n = cv.n;
  if (n > kCellCap) {
    if (lane == 0) atomicOr(&status->err, kErrOccupancy);
    return;
  }
  if (n < 2) {
    if (kTrace && n == 1 && lane == 0 && tr.perm) tr.perm[cv.base] = st.id[cv.base];
    return;
  }

  // ids to LDS, padded to a multiple of 4 with an id no particle has
  const uint32_t n4 = (n + 3u) & ~3u;
  for (uint32_t j = lane; j < n4; j += 64)
    s_id[j] = j < n ? st.id[cv.base + j] : 0xFFFFFFFFu;
  __syncthreads();

  // canonical order: the rank of each id among the cell's ids
  const uint4 *s_id4 = reinterpret_cast<const uint4 *>(s_id);
  for (uint32_t j = lane; j < n; j += 64) {
    const uint32_t me = s_id[j];
    uint32_t r = 0;
    for (uint32_t m = 0; m < n4 / 4; ++m) {
      const uint4 q = s_id4[m];
      r += (q.x < me) + (q.y < me) + (q.z < me) + (q.w < me);
    }
    s_perm[r] = (uint16_t)j;
    if (kTrace && tr.perm) tr.perm[cv.base + r] = me;
  }
  __syncthreads();

  // every pair k = 0 .. n(n-1)/2 - 1, lane-strided; pairs whose Philox word
  // w1 rules out acceptance (u >= w1 2^-32 > P22) are dropped at once, the
  // rest are compacted (in increasing k) for the exact test.  The main loop
  // takes two full rows of 64 pairs per iteration with no bounds checks.
  const uint32_t npairs = n * (n - 1u) / 2u;
  const uint64_t below = (1ull << lane) - 1ull;
  const uint32_t lim = pa.w1_max;
  uint32_t nf = 0, nclaim = 0, claimed_bits = 0, n_acc = 0;
  uint32_t k0 = 0;
  if (pa.any) {
    for (; k0 + 128u <= npairs; k0 += 128u) {
      const uint32_t ka = k0 + lane, kb = k0 + 64u + lane;
      const uint32_t wa = philox10_w1(ka, cv.c, t, 0u, pa.key0, pa.key1);
      const uint32_t wb = philox10_w1(kb, cv.c, t, 0u, pa.key0, pa.key1);
      const bool pass_a = wa <= lim, pass_b = wb <= lim;
      const uint64_t ma = __ballot(pass_a), mb = __ballot(pass_b);
      if ((ma | mb) != 0) {
        if (pass_a) s_filt[nf + (uint32_t)__popcll(ma & below)] = ka;
        nf += (uint32_t)__popcll(ma);
        if (pass_b) s_filt[nf + (uint32_t)__popcll(mb & below)] = kb;
        nf += (uint32_t)__popcll(mb);
        if (nf > kFiltCap - 128u) {
          resolve_filtered<kTrace>(nf, cv, pa, st, s_perm, s_filt, s_claim, nclaim,
                                   claimed_bits, n_acc, tr, status);
          nf = 0;
        }
      }
    }
    for (; k0 < npairs; k0 += 64u) {
      const uint32_t k = k0 + lane;
      bool pass = false;
      if (k < npairs) pass = philox10_w1(k, cv.c, t, 0u, pa.key0, pa.key1) <= lim;
      const uint64_t m = __ballot(pass);
      if (m != 0) {
        if (pass) s_filt[nf + (uint32_t)__popcll(m & below)] = k;
        nf += (uint32_t)__popcll(m);
        if (nf > kFiltCap - 64u) {
          resolve_filtered<kTrace>(nf, cv, pa, st, s_perm, s_filt, s_claim, nclaim,
                                   claimed_bits, n_acc, tr, status);
          nf = 0;
        }
      }
    }
  }
  if (nf != 0)
    resolve_filtered<kTrace>(nf, cv, pa, st, s_perm, s_filt, s_claim, nclaim,
                             claimed_bits, n_acc, tr, status);
  __syncthreads();

  // work counters: candidates are summed over the lanes that tested them
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) n_acc += __shfl_down(n_acc, o);
  if (lane == 0) {
    const uint32_t slot = cv.c % kCounterSlots;
    atomicAdd(&status->pairs[slot], (unsigned long long)npairs);
    atomicAdd(&status->cand[slot], (unsigned long long)n_acc);
    atomicAdd(&status->claims[slot], (unsigned long long)nclaim);
  }

  // kinematics of the claimed pairs (disjoint: one writer per particle)
  for (uint32_t i = lane; i < nclaim; i += 64) {
    const uint32_t v = s_claim[i];
    const uint32_t a = (v >> 10) & 1023u, b = v & 1023u;
    const uint32_t k = row_start(a, n) + (b - a - 1u);
    const Words4 w = philox10(k, cv.c, t, 1u, pa.key0, pa.key1);
    const double uc = uniform53(w.w0, w.w1);
    const double uphi = uniform53(w.w2, w.w3);
    const uint32_t ia = cv.base + s_perm[a], ib = cv.base + s_perm[b];
    double ax = st.px[ia], ay = st.py[ia], az = st.pz[ia];
    double bx = st.px[ib], by = st.py[ib], bz = st.pz[ib];
    scatter_pair(ax, ay, az, bx, by, bz, uc, uphi);
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

// ---------------------------------------------------------------------------
// Observe: per-slab sums of E and p_x.  Slab ix is the contiguous cell range
// [ix ny nz, (ix+1) ny nz), hence a contiguous particle range.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_observe_partial(
    const uint32_t *__restrict__ offsets, SoA st, uint32_t cells_per_slab,
    double *partial) {
  __shared__ double s_e[kBlock / 64], s_p[kBlock / 64];
  const uint32_t ix = blockIdx.x / kObsChunks, chunk = blockIdx.x % kObsChunks;
  const uint64_t lo = offsets[(uint64_t)ix * cells_per_slab];
  const uint64_t hi = offsets[(uint64_t)(ix + 1) * cells_per_slab];
  const uint64_t len = hi - lo;
  const uint64_t b0 = lo + len * chunk / kObsChunks;
  const uint64_t b1 = lo + len * (chunk + 1) / kObsChunks;
  double se = 0.0, sp = 0.0;
  for (uint64_t i = b0 + threadIdx.x; i < b1; i += kBlock) {
    const double px = st.px[i], py = st.py[i], pz = st.pz[i];
    se += norm3(px, py, pz);
    sp += px;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    se += __shfl_down(se, o);
    sp += __shfl_down(sp, o);
  }
  const uint32_t lane = lane_id(), wave = threadIdx.x / 64;
  if (lane == 0) {
    s_e[wave] = se;
    s_p[wave] = sp;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double te = 0.0, tp = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) {
      te += s_e[w];
      tp += s_p[w];
    }
    partial[2 * (size_t)blockIdx.x + 0] = te;
    partial[2 * (size_t)blockIdx.x + 1] = tp;
  }
}

__global__ __launch_bounds__(kBlock) void k_observe_final(const double *partial,
                                                          int32_t nx, double vol,
                                                          double *T00, double *T0x) {
  const int32_t ix = blockIdx.x * kBlock + threadIdx.x;
  if (ix >= nx) return;
  double te = 0.0, tp = 0.0;
  for (uint32_t ch = 0; ch < kObsChunks; ++ch) {
    te += partial[2 * ((size_t)ix * kObsChunks + ch) + 0];
    tp += partial[2 * ((size_t)ix * kObsChunks + ch) + 1];
  }
  T00[ix] = te / vol;
  T0x[ix] = tp / vol;
}

__global__ __launch_bounds__(kBlock) void k_gather_by_id(SoA st, int64_t n, double *x,
                                                         double *y, double *z,
                                                         double *px, double *py,
                                                         double *pz) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const uint32_t id = st.id[i];
  x[id] = st.x[i];
  y[id] = st.y[i];
  z[id] = st.z[i];
  px[id] = st.px[i];
  py[id] = st.py[i];
  pz[id] = st.pz[i];
}

inline unsigned grid_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
void launch_fill_u32(uint32_t *p, uint32_t v, int64_t count, hipStream_t s) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(count)), dim3(kBlock), 0, s, p, v, count);
}

void launch_load(const double *x, const double *y, const double *z,
                 const double *px, const double *py, const double *pz, SoA dst,
                 int64_t n, const Geometry &g, DevStatus *st, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_load, dim3(grid_for(n)), dim3(kBlock), 0, s, x, y, z, px, py,
                     pz, dst, n, g, st);
}

void launch_count(const SoA &src, int64_t n, const Geometry &g, bool stream,
                  uint32_t *counts, hipStream_t s) {
  if (n <= 0) return;
  if (stream)
    hipLaunchKernelGGL(k_count<true>, dim3(grid_for(n)), dim3(kBlock), 0, s, src, n, g,
                       counts);
  else
    hipLaunchKernelGGL(k_count<false>, dim3(grid_for(n)), dim3(kBlock), 0, s, src, n,
                       g, counts);
}

void launch_scan(uint32_t *counts, uint32_t *offsets, uint32_t *cursor,
                 uint32_t *tile_sums, int64_t n_cells, hipStream_t s) {
  const unsigned tiles = (unsigned)((n_cells + kScanTile - 1) / kScanTile);
  hipLaunchKernelGGL(k_scan_tiles, dim3(tiles), dim3(kBlock), 0, s, counts, offsets,
                     tile_sums, n_cells);
  hipLaunchKernelGGL(k_scan_carry, dim3(tiles), dim3(kBlock), 0, s, offsets, cursor,
                     (const uint32_t *)tile_sums, n_cells);
}

void launch_scatter(const SoA &src, SoA dst, int64_t n, const Geometry &g,
                    bool stream, uint32_t *cursor, uint32_t *trace_cell,
                    hipStream_t s) {
  if (n <= 0) return;
  if (stream)
    hipLaunchKernelGGL(k_scatter<true>, dim3(grid_for(n)), dim3(kBlock), 0, s, src, dst,
                       n, g, cursor, trace_cell);
  else
    hipLaunchKernelGGL(k_scatter<false>, dim3(grid_for(n)), dim3(kBlock), 0, s, src,
                       dst, n, g, cursor, trace_cell);
}

void launch_collide(const uint32_t *offsets, SoA st, int64_t n_cells, uint32_t t,
                    const PairArgs &pa, DevStatus *status, const TraceArgs *trace,
                    hipStream_t s) {
  if (n_cells <= 0) return;
  if (trace)
    hipLaunchKernelGGL(k_collide<true>, dim3((unsigned)n_cells), dim3(64), 0, s, offsets,
                       st, t, pa, status, *trace);
  else
    hipLaunchKernelGGL(k_collide<false>, dim3((unsigned)n_cells), dim3(64), 0, s,
                       offsets, st, t, pa, status, TraceArgs{});
}

void launch_observe(const uint32_t *offsets, const SoA &st, const Geometry &g,
                    double vol, double *partial, double *T00, double *T0x,
                    hipStream_t s) {
  const uint32_t nx = (uint32_t)g.n[0];
  const uint32_t cps = (uint32_t)g.n[1] * (uint32_t)g.n[2];
  hipLaunchKernelGGL(k_observe_partial, dim3(nx * kObsChunks), dim3(kBlock), 0, s,
                     offsets, st, cps, partial);
  hipLaunchKernelGGL(k_observe_final, dim3(grid_for(nx)), dim3(kBlock), 0, s,
                     (const double *)partial, (int32_t)nx, vol, T00, T0x);
}

void launch_gather_by_id(const SoA &st, int64_t n, double *x, double *y, double *z,
                         double *px, double *py, double *pz, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_gather_by_id, dim3(grid_for(n)), dim3(kBlock), 0, s, st, n, x, y,
                     z, px, py, pz);
}

}  // namespace cuba
