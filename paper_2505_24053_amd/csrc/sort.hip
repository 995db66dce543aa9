// Stage (b): association list.  Alg. 1 DuplicateWithKeys / SortByKeys /
// IdentifyFrustumRanges, arranged so the wide sort only touches tile ids:
//   1. stable LSD radix sort of the visible items by their 32-bit depth key
//      (the first pass compacts the visible items out of all items);
//   2. exclusive scan of the items' tile counts in depth order;
//   3. expansion of every item into (tile, item) entries in depth order,
//      balanced over entries (one binary search per 8 entries);
//   4. stable LSD radix sort of the entries by global tile id, so each tile's
//      run stays in (depth key, item) order;
//   5. run boundaries -> ranges[tile].
// Radix passes use 8-bit digits, 4096 keys per 256-lane block, LDS
// histograms and a wave-ballot match to rank equal digits stably.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "geer_common.h"

namespace geer {

constexpr int kBlock = 256;
constexpr int kPerThread = 16;
constexpr int kTileItems = kBlock * kPerThread;  // 4096 keys per block

__device__ __forceinline__ uint64_t lanemask_lt() {
  int lane = threadIdx.x & 63;
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// inclusive scan over a wave64 of u32
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
  int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    uint32_t y = __shfl_up(x, off);
    if (lane >= off) x += y;
  }
  return x;
}

// ------------------------------------------------------------------ scan --

__global__ __launch_bounds__(kBlock) void scan_reduce_kernel(const uint32_t* __restrict__ in, int64_t n,
                                                             uint32_t* __restrict__ sums) {
  int64_t base = (int64_t)blockIdx.x * kTileItems;
  uint32_t s = 0;
#pragma unroll 4
  for (int it = 0; it < kPerThread; ++it) {
    int64_t i = base + it * kBlock + threadIdx.x;
    if (i < n) s += in[i];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  __shared__ uint32_t red[kBlock / 64];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) sums[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// Exclusive scan of one 4096-item tile with a carried-in offset.
__global__ __launch_bounds__(kBlock) void scan_apply_kernel(const uint32_t* __restrict__ in, int64_t n,
                                                            const uint32_t* __restrict__ offs,
                                                            uint32_t* __restrict__ out) {
  int64_t base = (int64_t)blockIdx.x * kTileItems + (int64_t)threadIdx.x * kPerThread;
  uint32_t v[kPerThread];
  uint32_t tsum = 0;
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) {
    int64_t i = base + k;
    v[k] = i < n ? in[i] : 0u;
    tsum += v[k];
  }
  uint32_t incl = wave_incl_scan(tsum);
  __shared__ uint32_t wsum[kBlock / 64];
  int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 63) wsum[wv] = incl;
  __syncthreads();
  uint32_t wpre = 0;
  for (int w = 0; w < wv; ++w) wpre += wsum[w];
  uint32_t run = (offs ? offs[blockIdx.x] : 0u) + wpre + incl - tsum;
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) {
    int64_t i = base + k;
    if (i < n) out[i] = run;
    run += v[k];
  }
}

// ----------------------------------------------------------------- radix --

// Per-block digit histogram, written digit-major: hist[d * nblocks + b].
// With `filter`, items whose filter value is 0 are skipped (compaction pass).
// The element count is n_cap, or min(*dyn, n_cap) when a device-side count
// is given (capacity-sized launches that need no host read-back).
__device__ __forceinline__ int64_t dyn_count(int64_t n_cap, const unsigned long long* dyn) {
  return dyn ? min((int64_t)*dyn, n_cap) : n_cap;
}

__global__ __launch_bounds__(kBlock) void radix_hist_kernel(const uint32_t* __restrict__ keys,
                                                            const uint32_t* __restrict__ filter, int64_t n_cap,
                                                            const unsigned long long* __restrict__ dyn, int shift,
                                                            uint32_t* __restrict__ hist, int64_t nblocks) {
  const int64_t n = dyn_count(n_cap, dyn);
  __shared__ uint32_t cnt[256];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  int64_t base = (int64_t)blockIdx.x * kTileItems;
#pragma unroll 4
  for (int it = 0; it < kPerThread; ++it) {
    int64_t i = base + it * kBlock + threadIdx.x;
    if (i < n && (!filter || filter[i] != 0)) atomicAdd(&cnt[(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

// Stable scatter.  Items of a block are processed in 16 consecutive slices of
// 256; within a slice the rank of an item among equal digits is its rank in
// its wave (ballot match) plus the counts of the earlier waves.
__global__ __launch_bounds__(kBlock) void radix_scatter_kernel(
    const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in,
    const uint32_t* __restrict__ filter, int64_t n_cap, const unsigned long long* __restrict__ dyn, int shift,
    const uint32_t* __restrict__ hist_off, int64_t nblocks, uint32_t* __restrict__ keys_out,
    uint32_t* __restrict__ vals_out) {
  const int64_t n = dyn_count(n_cap, dyn);
  __shared__ uint32_t running[256];
  __shared__ uint32_t wcnt[2][4][256];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  running[tid] = hist_off[(int64_t)tid * nblocks + blockIdx.x];
#pragma unroll
  for (int w = 0; w < 4; ++w) { wcnt[0][w][tid] = 0; wcnt[1][w][tid] = 0; }
  __syncthreads();
  const uint64_t lt = lanemask_lt();
  int64_t base = (int64_t)blockIdx.x * kTileItems;
  for (int it = 0; it < kPerThread; ++it) {
    const int buf = it & 1;
    int64_t i = base + it * kBlock + tid;
    bool active = i < n && (!filter || filter[i] != 0);
    uint32_t key = active ? keys_in[i] : 0u;
    uint32_t val = active ? (vals_in ? vals_in[i] : (uint32_t)i) : 0u;
    uint32_t d = (key >> shift) & 255u;
    uint64_t m = __ballot(active);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      uint64_t bb = __ballot(active && ((d >> b) & 1u));
      m &= ((d >> b) & 1u) ? bb : ~bb;
    }
    uint32_t rank = (uint32_t)__popcll(m & lt);
    if (active && rank == 0) wcnt[buf][wv][d] = (uint32_t)__popcll(m);
    __syncthreads();
    if (active) {
      uint32_t pre = 0;
      for (int w = 0; w < wv; ++w) pre += wcnt[buf][w][d];
      uint32_t pos = running[d] + pre + rank;
      keys_out[pos] = key;
      vals_out[pos] = val;
    }
    uint32_t tot = wcnt[buf][0][tid] + wcnt[buf][1][tid] + wcnt[buf][2][tid] + wcnt[buf][3][tid];
    __syncthreads();
    running[tid] += tot;
#pragma unroll
    for (int w = 0; w < 4; ++w) wcnt[buf][w][tid] = 0;
  }
}

// ------------------------------------------------------------ expansion --

__global__ __launch_bounds__(kBlock) void gather_counts_kernel(const uint32_t* __restrict__ items, int64_t m_cap,
                                                               const unsigned long long* __restrict__ dyn,
                                                               const uint32_t* __restrict__ counts,
                                                               uint32_t* __restrict__ out) {
  const int64_t m = dyn_count(m_cap, dyn);
  int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j < m) out[j] = counts[items[j]];
  else if (j < m_cap) out[j] = 0u;
}

constexpr int kExpandPer = 8;

// Each lane expands kExpandPer consecutive entries (one binary search for the
// owner of its first entry), the block stages its 2048 entries in LDS and
// writes them back lane-striped so every store is coalesced.
__global__ __launch_bounds__(kBlock) void expand_kernel(const uint32_t* __restrict__ items,
                                                        const uint32_t* __restrict__ offs, int64_t m_cap,
                                                        const unsigned long long* __restrict__ dyn_m,
                                                        int64_t total_cap,
                                                        const unsigned long long* __restrict__ dyn_total,
                                                        const uint2* __restrict__ rects,
                                                        const ViewDev* __restrict__ views, int64_t n,
                                                        uint32_t* __restrict__ tiles_out,
                                                        uint32_t* __restrict__ items_out) {
  const int64_t m = dyn_count(m_cap, dyn_m);
  const int64_t total = dyn_count(total_cap, dyn_total);
  __shared__ uint32_t s_tile[kBlock * kExpandPer];
  __shared__ uint32_t s_item[kBlock * kExpandPer];
  const int64_t block0 = (int64_t)blockIdx.x * kBlock * kExpandPer;
  const int64_t e0 = block0 + (int64_t)threadIdx.x * kExpandPer;
  if (e0 < total) {
    // owner of e0: last j with offs[j] <= e0
    int64_t lo = 0, hi = m;
    while (hi - lo > 1) {
      int64_t mid = (lo + hi) >> 1;
      if ((int64_t)offs[mid] <= e0) lo = mid; else hi = mid;
    }
    int64_t j = lo;
    const int64_t e1 = min(e0 + kExpandPer, total);
    for (int64_t e = e0; e < e1; ++e) {
      while (j + 1 < m && (int64_t)offs[j + 1] <= e) ++j;
      const uint32_t item = items[j];
      const uint32_t local = (uint32_t)(e - (int64_t)offs[j]);
      const uint2 r = rects[item];
      const int tx0 = (int)(r.x & 0xffffu) >> 1, tx1 = (int)(r.x >> 16) >> 1;
      const int ty0 = (int)(r.y & 0xffffu) >> 1;
      const uint32_t wt = (uint32_t)(tx1 - tx0 + 1);
      const ViewDev& V = views[item / (uint32_t)n];
      const uint32_t ty = ty0 + local / wt, tx = tx0 + local % wt;
      const int s = (int)(e - block0);
      s_tile[s] = (uint32_t)V.tile_base + ty * (uint32_t)V.tiles_x + tx;
      s_item[s] = item;
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kExpandPer; ++k) {
    const int s = k * kBlock + threadIdx.x;
    const int64_t e = block0 + s;
    if (e < total) {
      tiles_out[e] = s_tile[s];
      items_out[e] = s_item[s];
    }
  }
}

__global__ __launch_bounds__(kBlock) void ranges_kernel(const uint32_t* __restrict__ tiles, int64_t total_cap,
                                                        const unsigned long long* __restrict__ dyn,
                                                        int64_t ntiles, uint32_t* __restrict__ ranges) {
  const int64_t total = dyn_count(total_cap, dyn);
  int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (total == 0) {
    for (int64_t t = e; t <= ntiles; t += (int64_t)gridDim.x * kBlock) ranges[t] = 0u;
    return;
  }
  if (e >= total) return;
  int64_t cur = tiles[e];
  int64_t prev = e > 0 ? (int64_t)tiles[e - 1] : -1;
  for (int64_t t = prev + 1; t <= cur; ++t) ranges[t] = (uint32_t)e;
  if (e == total - 1)
    for (int64_t t = cur + 1; t <= ntiles; ++t) ranges[t] = (uint32_t)total;
}

__global__ __launch_bounds__(kBlock) void fill_u32_kernel(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = v;
}

// list[total .. total + 8) = 0 with total read on the device (padding read by
// the render's 8-aligned batches); total is clamped to the capacity.
__global__ void pad_list_kernel(uint32_t* __restrict__ list, int64_t total_cap,
                                const unsigned long long* __restrict__ dyn) {
  const int64_t total = dyn_count(total_cap, dyn);
  if (threadIdx.x < 8) list[total + threadIdx.x] = 0u;
}

// Capacity guard of capacity-sized launches: stats[3] keeps the entry count;
// when it exceeds the capacity, the entry and visible counts are cleared so
// every later kernel sees an empty list (the frame renders as background and
// the host reports the overflow from stats[3]).
__global__ void capacity_guard_kernel(unsigned long long* __restrict__ stats, int64_t cap) {
  if (threadIdx.x == 0) {
    const unsigned long long e = stats[0];
    stats[3] = e;
    if (e > (unsigned long long)cap) {
      stats[0] = 0ull;
      stats[1] = 0ull;
    }
  }
}

// --------------------------------------------------------------- host side --

static inline unsigned grid_for(int64_t n, int64_t per) { return (unsigned)((n + per - 1) / per); }

int64_t scan_scratch_words(int64_t n) {
  int64_t words = 0;
  while (n > kTileItems) {
    n = (n + kTileItems - 1) / kTileItems;
    words += n + 1;
  }
  return words + 1;
}

// Exclusive scan of n u32 (in may equal out).  scratch: scan_scratch_words(n).
void scan_exclusive(hipStream_t st, const uint32_t* in, uint32_t* out, int64_t n, uint32_t* scratch) {
  if (n <= 0) return;
  if (n <= kTileItems) {
    hipLaunchKernelGGL(scan_apply_kernel, dim3(1), dim3(kBlock), 0, st, in, n, (const uint32_t*)nullptr, out);
    return;
  }
  int64_t nb = (n + kTileItems - 1) / kTileItems;
  uint32_t* sums = scratch;
  hipLaunchKernelGGL(scan_reduce_kernel, dim3((unsigned)nb), dim3(kBlock), 0, st, in, n, sums);
  scan_exclusive(st, sums, sums, nb, scratch + nb + 1);
  hipLaunchKernelGGL(scan_apply_kernel, dim3((unsigned)nb), dim3(kBlock), 0, st, in, n, (const uint32_t*)sums,
                     out);
}

int64_t radix_hist_words(int64_t n) { return 256 * ((n + kTileItems - 1) / kTileItems) + 1; }

// One stable 8-bit pass over n_cap keys (or the device count *dyn).
// hist: radix_hist_words(n_cap); scratch for its scan.
void radix_pass(hipStream_t st, const uint32_t* keys_in, const uint32_t* vals_in, const uint32_t* filter,
                int64_t n_cap, const unsigned long long* dyn, int shift, uint32_t* keys_out, uint32_t* vals_out,
                uint32_t* hist, uint32_t* scan_scratch) {
  if (n_cap <= 0) return;
  int64_t nb = (n_cap + kTileItems - 1) / kTileItems;
  hipLaunchKernelGGL(radix_hist_kernel, dim3((unsigned)nb), dim3(kBlock), 0, st, keys_in, filter, n_cap, dyn, shift,
                     hist, nb);
  scan_exclusive(st, hist, hist, 256 * nb, scan_scratch);
  hipLaunchKernelGGL(radix_scatter_kernel, dim3((unsigned)nb), dim3(kBlock), 0, st, keys_in, vals_in, filter, n_cap,
                     dyn, shift, (const uint32_t*)hist, nb, keys_out, vals_out);
}

void launch_gather_counts(hipStream_t st, const uint32_t* items, int64_t m_cap, const unsigned long long* dyn,
                          const uint32_t* counts, uint32_t* out) {
  if (m_cap <= 0) return;
  hipLaunchKernelGGL(gather_counts_kernel, dim3(grid_for(m_cap, kBlock)), dim3(kBlock), 0, st, items, m_cap, dyn,
                     counts, out);
}

void launch_expand(hipStream_t st, const uint32_t* items, const uint32_t* offs, int64_t m_cap,
                   const unsigned long long* dyn_m, int64_t total_cap, const unsigned long long* dyn_total,
                   const uint2* rects, const ViewDev* views, int64_t n, uint32_t* tiles_out, uint32_t* items_out) {
  if (total_cap <= 0) return;
  hipLaunchKernelGGL(expand_kernel, dim3(grid_for(total_cap, (int64_t)kBlock * kExpandPer)), dim3(kBlock), 0, st,
                     items, offs, m_cap, dyn_m, total_cap, dyn_total, rects, views, n, tiles_out, items_out);
}

void launch_ranges(hipStream_t st, const uint32_t* tiles, int64_t total_cap, const unsigned long long* dyn,
                   int64_t ntiles, uint32_t* ranges) {
  if (total_cap <= 0 && !dyn) {
    hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(ntiles + 1, kBlock)), dim3(kBlock), 0, st, ranges, ntiles + 1,
                       0u);
    return;
  }
  const int64_t g = std::max<int64_t>(total_cap, ntiles + 1);
  hipLaunchKernelGGL(ranges_kernel, dim3(grid_for(g, kBlock)), dim3(kBlock), 0, st, tiles, total_cap, dyn, ntiles,
                     ranges);
}

void launch_capacity_guard(hipStream_t st, unsigned long long* stats, int64_t cap) {
  hipLaunchKernelGGL(capacity_guard_kernel, dim3(1), dim3(64), 0, st, stats, cap);
}

void launch_pad_list(hipStream_t st, uint32_t* list, int64_t total_cap, const unsigned long long* dyn) {
  hipLaunchKernelGGL(pad_list_kernel, dim3(1), dim3(64), 0, st, list, total_cap, dyn);
}

void launch_fill_u32(hipStream_t st, uint32_t* p, int64_t n, uint32_t v) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, st, p, n, v);
}

}  // namespace geer
