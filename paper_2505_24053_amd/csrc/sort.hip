// Stage (b): association list.  Alg. 1 DuplicateWithKeys / SortByKeys /
// IdentifyFrustumRanges, arranged so the wide sort only touches tile ids:
//   1. stable LSD radix sort of the visible items by their 32-bit depth key
//      (the first pass compacts the visible items out of all items);
//   2. exclusive scan of the items' tile counts in depth order;
//   3. expansion of every item into (tile, item) entries in depth order,
//      balanced over entries (8 per lane; owners found through LDS), with
//      the contribution-cone cull marking the entries no ray can see;
//   4. stable LSD radix sort of the entries by global tile id, so each tile's
//      run stays in (depth key, item) order;
//   5. run boundaries -> ranges[tile].
// Radix passes use 8-bit digits, one kernel per pass with decoupled
// look-back (below).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "geer_common.h"
#include "geer_device.h"

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

// The element count is n_cap, or min(*dyn, n_cap) when a device-side count
// is given (capacity-sized launches that need no host read-back).
__device__ __forceinline__ int64_t dyn_count(int64_t n_cap, const unsigned long long* dyn) {
  return dyn ? min((int64_t)*dyn, n_cap) : n_cap;
}

// ------------------------------------------------------ gathered scan --
//
// Exclusive scan of the gathered values counts[items[j]] (j < m; 0 for
// m <= j < m_cap) in two kernels: the first gathers and sums each 4096-item
// tile, the second adds up the sums of the tiles before its own (at most
// kGatherScanTiles of them) and scans its tile.

constexpr int kGatherScanTiles = 4096;

__global__ __launch_bounds__(kBlock) void gather_reduce_kernel(const uint32_t* __restrict__ items, int64_t m_cap,
                                                               const unsigned long long* __restrict__ dyn,
                                                               const uint32_t* __restrict__ counts,
                                                               uint32_t* __restrict__ out,
                                                               uint32_t* __restrict__ sums) {
  const int64_t m = dyn_count(m_cap, dyn);
  const int64_t base = (int64_t)blockIdx.x * kTileItems;
  uint32_t it[kPerThread];
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) {  // independent loads first
    const int64_t i = base + k * kBlock + threadIdx.x;
    it[k] = i < m ? items[i] : 0u;
  }
  uint32_t s = 0u;
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) {
    const int64_t i = base + k * kBlock + threadIdx.x;
    const uint32_t v = i < m ? counts[it[k]] : 0u;
    if (i < m_cap) out[i] = v;
    s += v;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  __shared__ uint32_t red[kBlock / 64];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) sums[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// LDS slot of item i of a 4096-item tile: one word of padding per 16, so the
// 16 consecutive items of each thread start on distinct banks.
__device__ __forceinline__ int scan_slot(int i) { return i + (i >> 4); }

// kStaged: the tile goes through LDS so that global loads and stores are
// lane-striped (coalesced); worth its barrier from a few dozen tiles on.
template <bool kStaged>
__global__ __launch_bounds__(kBlock) void gathered_scan_kernel(const uint32_t* __restrict__ in, int64_t n,
                                                               const uint32_t* __restrict__ sums,
                                                               uint32_t* __restrict__ out) {
  __shared__ uint32_t s_v[kStaged ? kTileItems + kTileItems / 16 : 1];
  const int64_t tile0 = (int64_t)blockIdx.x * kTileItems;
  if (kStaged) {
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
      const int li = k * kBlock + threadIdx.x;
      s_v[scan_slot(li)] = tile0 + li < n ? in[tile0 + li] : 0u;
    }
  }
  // carried-in offset: the sums of tiles 0 .. blockIdx.x - 1
  uint32_t pre = 0u;
  for (int t = threadIdx.x; t < (int)blockIdx.x; t += kBlock) pre += sums[t];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) pre += __shfl_xor(pre, off);
  __shared__ uint32_t red[kBlock / 64], wsum[kBlock / 64];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = pre;
  __syncthreads();
  // each thread scans 16 consecutive items
  const int lbase = threadIdx.x * kPerThread;
  uint32_t v[kPerThread];
  uint32_t tsum = 0;
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) {
    if (kStaged) v[k] = s_v[scan_slot(lbase + k)];
    else v[k] = tile0 + lbase + k < n ? in[tile0 + lbase + k] : 0u;
    tsum += v[k];
  }
  const uint32_t incl = wave_incl_scan(tsum);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 63) wsum[wv] = incl;
  __syncthreads();
  uint32_t wpre = 0;
  for (int w = 0; w < wv; ++w) wpre += wsum[w];
  uint32_t run = red[0] + red[1] + red[2] + red[3] + wpre + incl - tsum;
  if (!kStaged) {
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
      if (tile0 + lbase + k < n) out[tile0 + lbase + k] = run;
      run += v[k];
    }
    return;
  }
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) {
    s_v[scan_slot(lbase + k)] = run;  // only this thread's slots: no barrier before
    run += v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) {
    const int li = k * kBlock + threadIdx.x;
    if (tile0 + li < n) out[tile0 + li] = s_v[scan_slot(li)];
  }
}

// ----------------------------------------------------------------- radix --
//
// Stable LSD radix sort with 8-bit digits, one kernel per pass ("onesweep"
// with decoupled look-back).  An upsweep kernel first counts the digits of
// every pass over the (filtered) input.  In a pass, block b takes the b-th
// chunk of keys (1024 to 4096 keys by sort size, os_per), ranks its keys
// stably (per wave: ballot match on the digit; across waves and slices:
// running counts in LDS), publishes its per-digit counts, and walks back
// over earlier blocks' published counts -- stopping at the first that
// already holds its inclusive prefix -- to find where its run of each digit
// starts.  Keys are then reordered by digit in LDS and written out as
// contiguous runs.  A status
// word is [flag:2 | count:30]; the look-back spin is bounded and reports a
// stall through an error word instead of hanging.  A block waits only on
// blocks with lower indices, and each XCD dispatches the workgroups of a
// launch in index order, so the lowest unfinished block is always resident
// and the walk always ends.  (A per-block atomic ticket would serialise:
// tickets come one at a time off one counter, which staggers the 692 blocks
// of a 2.8M-key pass over about 9 us.)

constexpr int kLookBack = 16;  // statuses read per look-back round
constexpr int kOSPerSmall = 4;                  // keys per thread below kOSSmallKeys keys
constexpr int64_t kOSSmallKeys = 1 << 18;
constexpr int kOSPer = 8;                       // keys per thread (mid-size sorts)
constexpr int kOSPerBig = 16;                   // keys per thread from kOSBigKeys keys on
constexpr int64_t kOSBigKeys = 1 << 20;
constexpr int kOSItems = kBlock * kOSPerSmall;  // 1024 keys per block: the smallest chunk

// Keys per thread of a sort of up to nmax keys: small sorts take small chunks
// (more blocks, each with a shorter chain of loads, ranking and scatter),
// large ones long chunks (longer runs of one digit per chunk).
__host__ __device__ __forceinline__ int os_per(int64_t nmax) {
  return nmax < kOSSmallKeys ? kOSPerSmall : nmax < kOSBigKeys ? kOSPer : kOSPerBig;
}
constexpr uint32_t kFlagAgg = 1u << 30, kFlagInc = 2u << 30, kValMask = (1u << 30) - 1u;
constexpr uint32_t kSpinLimit = 1u << 22;
constexpr int kWorkHead = 1024 + 64;            // histograms of 4 passes (padded)

__host__ __device__ __forceinline__ int64_t os_blocks(int64_t n, int items) { return (n + items - 1) / items; }

// Exclusive scan of one value per thread over a 256-lane block; also returns
// the block total.  Uses s_w[4].
__device__ __forceinline__ uint32_t block_excl_scan256(uint32_t x, uint32_t* s_w, uint32_t& total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t incl = wave_incl_scan(x);
  if (lane == 63) s_w[w] = incl;
  __syncthreads();
  uint32_t pre = 0;
  for (int q = 0; q < w; ++q) pre += s_w[q];
  total = s_w[0] + s_w[1] + s_w[2] + s_w[3];
  __syncthreads();
  return pre + incl - x;
}

// A key equal to kDropKey is not sorted when `drop` is set (entries the
// expansion found unable to contribute); the pass-0 output count is then
// added to *kept.
constexpr uint32_t kDropKey = 0xffffffffu;

__global__ __launch_bounds__(kBlock) void radix_upsweep_kernel(const uint32_t* __restrict__ keys,
                                                               const uint32_t* __restrict__ filter, int drop,
                                                               int64_t n_cap,
                                                               const unsigned long long* __restrict__ dyn,
                                                               int shift0, int bits, int npass,
                                                               uint32_t* __restrict__ ghist,
                                                               unsigned long long* __restrict__ kept) {
  const uint32_t dmask = (1u << bits) - 1u;
  const int64_t n = dyn_count(n_cap, dyn);
  __shared__ uint32_t h[4][256];
  __shared__ uint32_t s_kept;
#pragma unroll
  for (int p = 0; p < 4; ++p) h[p][threadIdx.x] = 0u;
  if (threadIdx.x == 0) s_kept = 0u;
  __syncthreads();
  uint32_t mine = 0u;
  // grid-stride; with many keys per thread, 8 keys per step with all their
  // loads in flight together
  constexpr int kUp = 8;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  if (n <= 2 * stride) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
      const uint32_t f = filter ? filter[i] : 1u;
      const uint32_t k = keys[i];
      if (f == 0u || (drop && k == kDropKey)) continue;
      ++mine;
      for (int p = 0; p < npass; ++p) atomicAdd(&h[p][(k >> (shift0 + bits * p)) & dmask], 1u);
    }
  } else {
    for (int64_t i0 = (int64_t)blockIdx.x * kBlock + threadIdx.x; i0 < n; i0 += kUp * stride) {
      uint32_t f[kUp], k[kUp];
#pragma unroll
      for (int u = 0; u < kUp; ++u) {
        const int64_t i = i0 + u * stride;
        const int64_t ic = i < n ? i : n - 1;
        f[u] = filter ? filter[ic] : 1u;
        k[u] = keys[ic];
      }
#pragma unroll
      for (int u = 0; u < kUp; ++u) {
        if (i0 + u * stride >= n || f[u] == 0u || (drop && k[u] == kDropKey)) continue;
        ++mine;
        for (int p = 0; p < npass; ++p) atomicAdd(&h[p][(k[u] >> (shift0 + bits * p)) & dmask], 1u);
      }
    }
  }
  if (kept && mine) atomicAdd(&s_kept, mine);
  __syncthreads();
  for (int p = 0; p < npass; ++p) {
    const uint32_t c = h[p][threadIdx.x];
    if (c) atomicAdd(&ghist[p * 256 + threadIdx.x], c);
  }
  if (kept && threadIdx.x == 0 && s_kept) atomicAdd(kept, (unsigned long long)s_kept);
}

template <int kPer>
__global__ __launch_bounds__(kBlock) void radix_onesweep_kernel(
    const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in, const uint32_t* __restrict__ filter,
    int drop, int64_t n_cap, const unsigned long long* __restrict__ dyn, int shift, uint32_t dmask,
    const uint32_t* __restrict__ ghist_p,
    uint32_t* __restrict__ status, uint32_t* __restrict__ status_next,
    uint32_t* __restrict__ keys_out, uint32_t* __restrict__ vals_out, unsigned long long* __restrict__ err) {
  __shared__ uint32_t s_cnt[4][256];  // per-wave running digit counts, then per-wave offsets
  __shared__ uint32_t s_loc[256];     // block-local start of each digit
  __shared__ uint32_t s_glob[256];    // global start of this block's run of each digit
  constexpr int kItems = kBlock * kPer;
  __shared__ uint32_t s_key[kItems], s_val[kItems];
  __shared__ uint32_t s_w[4];

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  // the grid is sized for the capacity: blocks past the live key count leave
  const int64_t n = dyn_count(n_cap, dyn);
  const int64_t blk = blockIdx.x;
  if (blk >= os_blocks(n, kItems)) return;
#pragma unroll
  for (int q = 0; q < 4; ++q) s_cnt[q][tid] = 0u;
  __syncthreads();
  if (status_next) status_next[blk * 256 + tid] = 0u;  // this row is clear for the next pass

  // stable ranks within the wave: wave w owns keys [base, base + 64 kPer).
  // Every slice's filter word, key and value are loaded first, from an index
  // clamped into [0, n) (n > 0 here), so the loads are independent and in
  // flight together; the ranking below only waits for them once.
  const int64_t base = blk * kItems + (int64_t)w * 64 * kPer;
  const uint64_t lt = lanemask_lt();
  uint32_t key[kPer], val[kPer], rank[kPer], flt[kPer];
#pragma unroll
  for (int sl = 0; sl < kPer; ++sl) {
    const int64_t i = base + sl * 64 + lane;
    const int64_t ic = i < n ? i : n - 1;
    flt[sl] = filter ? filter[ic] : 1u;
    key[sl] = keys_in[ic];
    val[sl] = vals_in ? vals_in[ic] : (uint32_t)i;
  }
  uint32_t act = 0u;
#pragma unroll
  for (int sl = 0; sl < kPer; ++sl) {
    const int64_t i = base + sl * 64 + lane;
    bool a = i < n && flt[sl] != 0u;
    if (drop) a = a && key[sl] != kDropKey;
    if (!a) key[sl] = 0u;
    if (!a) val[sl] = 0u;
    const uint32_t d = (key[sl] >> shift) & dmask;
    uint64_t m = __builtin_amdgcn_ballot_w64(a);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint64_t bb = __builtin_amdgcn_ballot_w64(((d >> b) & 1u) != 0u);
      m &= ((d >> b) & 1u) ? bb : ~bb;
    }
    const uint32_t r = (uint32_t)__popcll(m & lt);
    const uint32_t pre = a ? s_cnt[w][d] : 0u;  // every lane of a digit reads before its leader writes
    rank[sl] = pre + r;
    if (a && r == 0u) s_cnt[w][d] = pre + (uint32_t)__popcll(m);
    act |= (a ? 1u : 0u) << sl;
    // the wave's next slice reads these counts (LDS order within a wave)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  __syncthreads();

  // per digit (thread tid): wave offsets and the block's count
  const uint32_t c0 = s_cnt[0][tid], c1 = s_cnt[1][tid], c2 = s_cnt[2][tid], c3 = s_cnt[3][tid];
  const uint32_t tot = c0 + c1 + c2 + c3;
  s_cnt[0][tid] = 0u;
  s_cnt[1][tid] = c0;
  s_cnt[2][tid] = c0 + c1;
  s_cnt[3][tid] = c0 + c1 + c2;
  __hip_atomic_store(&status[blk * 256 + tid], kFlagAgg | tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);

  // decoupled look-back over the earlier blocks, kLookBack statuses per
  // round (independent loads in flight together): add aggregates from the
  // nearest block back until an inclusive prefix; stop at a block that has
  // not published yet and poll again from it.  Block 0's aggregate is its
  // inclusive prefix, so the walk also ends after it.
  uint32_t excl = 0u, spins = 0u;
  for (int64_t j = blk - 1; j >= 0;) {
    uint32_t v[kLookBack];
#pragma unroll
    for (int q = 0; q < kLookBack; ++q)
      v[q] = j - q >= 0 ? __hip_atomic_load(&status[(j - q) * 256 + tid], __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT)
                        : kFlagInc;
    int q = 0;
    bool done = false;
#pragma unroll
    for (int r = 0; r < kLookBack; ++r) {
      if (q != r) continue;
      const uint32_t f = v[r] & ~kValMask;
      if (f == 0u) continue;  // not published: poll from here again
      excl += v[r] & kValMask;
      if (f == kFlagInc) done = true;
      else q = r + 1;
    }
    if (done) break;
    j -= q;
    if (q < kLookBack) {
      if (++spins > kSpinLimit) {
        atomicOr(err, 1ull);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  __hip_atomic_store(&status[blk * 256 + tid], kFlagInc | (excl + tot), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);

  uint32_t gtotal, ltotal;
  const uint32_t gstart = block_excl_scan256(ghist_p[tid], s_w, gtotal);
  const uint32_t lstart = block_excl_scan256(tot, s_w, ltotal);
  s_glob[tid] = gstart + excl;
  s_loc[tid] = lstart;
  __syncthreads();

  // reorder by digit in LDS, then write contiguous runs
#pragma unroll
  for (int sl = 0; sl < kPer; ++sl) {
    if ((act >> sl) & 1u) {
      const uint32_t d = (key[sl] >> shift) & dmask;
      const uint32_t lp = s_loc[d] + s_cnt[w][d] + rank[sl];
      s_key[lp] = key[sl];
      s_val[lp] = val[sl];
    }
  }
  __syncthreads();
  for (uint32_t i = tid; i < ltotal; i += kBlock) {
    const uint32_t k = s_key[i];
    const uint32_t d = (k >> shift) & dmask;
    const uint32_t g = s_glob[d] + (i - s_loc[d]);
    keys_out[g] = k;
    vals_out[g] = s_val[i];
  }
}

// Partial digit histograms filled by a producer kernel: kHistCopies copies
// (block b adds to copy b % kHistCopies), each with 256 words per pass for
// up to kHistPasses passes and the count of kept keys at kHistKept.
constexpr int kHistCopies = 64;
constexpr int kHistPasses = 2;
constexpr int kHistKept = 256 * kHistPasses;
constexpr int kHistStride = kHistKept + 8;

int hist_parts_words() { return kHistCopies * kHistStride; }

// Writes the sort's work head and first status table: the pass histograms
// summed over the copies, zero elsewhere; *kept = the summed kept count.
__global__ __launch_bounds__(kBlock) void hist_prepare_kernel(uint32_t* __restrict__ work, int64_t nwords,
                                                              const uint32_t* __restrict__ hparts, int npass,
                                                              unsigned long long* __restrict__ kept) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= nwords) return;
  uint32_t v = 0u;
  if (i < 256 * npass) {
    for (int c = 0; c < kHistCopies; ++c) v += hparts[c * kHistStride + i];
  }
  work[i] = v;
  if (i == 0 && kept) {
    unsigned long long k = 0;
    for (int c = 0; c < kHistCopies; ++c) k += hparts[c * kHistStride + kHistKept];
    *kept = k;
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

// Corner directions of every 16x16 tile of every view (the expansion's
// culling cone), four float4 per tile: corner k in .xyz of entry k, the
// cone's validity in .w of entry 0.
__global__ __launch_bounds__(kBlock) void tile_cones_kernel(const ViewDev* __restrict__ views, int nviews,
                                                            const float2* __restrict__ dtab, int64_t ntiles,
                                                            float4* __restrict__ out, uint32_t* __restrict__ zero,
                                                            int64_t nzero) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t < nzero) zero[t] = 0u;  // a buffer the next kernels accumulate into
  if (t >= ntiles) return;
  int v = 0;
  while (v + 1 < nviews && t >= views[v + 1].tile_base) ++v;
  const ViewDev& V = views[v];
  const int lt = (int)(t - V.tile_base);
  const int ty = lt / V.tiles_x, tx = lt - ty * V.tiles_x;
  const QuadCone Q = block_cone(V, dtab, tx * kTile, ty * kTile, kTile);
#pragma unroll
  for (int k = 0; k < 4; ++k)
    out[4 * t + k] = make_float4(Q.d[k][0], Q.d[k][1], Q.d[k][2], k == 0 ? (Q.valid ? 1.0f : 0.0f) : 0.0f);
}

// floor(a / b), exact, for 0 < b and a quotient below 2^20 (here: a view
// index, < 4096, and a row of a rectangle, < 2^15): the float estimate has a
// relative error of a few 2^-24, so it is within one of the quotient, and one
// integer step each way corrects it (q b <= a + b < 2^32).
__device__ __forceinline__ uint32_t small_quotient(uint32_t a, uint32_t b) {
  uint32_t q = (uint32_t)((float)a * __builtin_amdgcn_rcpf((float)b));
  if (q * b > a) --q;
  else if (a - q * b >= b) ++q;
  return q;
}

// LDS slot of staged entry i: one word of padding per 32 so that lanes
// writing every kExpandPer-th entry hit distinct banks.
__device__ __forceinline__ int stage_slot(int i) { return i + (i >> 5); }

// Each lane expands kExpandPer consecutive entries; the block stages its
// 2048 entries in LDS and writes them back lane-striped so every store is
// coalesced.  With `cull`, an entry whose Gaussian's contribution cone meets
// no ray of its tile gets the tile id kDropKey and is left out by the tile
// sort.  Latency: one wave finds the owner of the block's first entry with a
// 64-way search (a few dependent loads instead of ~log2 m), the owners'
// offsets that can start inside the block are staged in LDS, where each lane
// finds and walks its owners; the tile ids of all the lane's entries are
// derived first, so each entry's tile cone is loaded one entry ahead of its
// test.
__global__ __launch_bounds__(kBlock) void expand_kernel(const uint32_t* __restrict__ items,
                                                        const uint32_t* __restrict__ offs, int64_t m_cap,
                                                        const unsigned long long* __restrict__ dyn_m,
                                                        int64_t total_cap,
                                                        const unsigned long long* __restrict__ dyn_total,
                                                        const uint2* __restrict__ rects,
                                                        const ViewDev* __restrict__ views, int64_t n,
                                                        const float4* __restrict__ tcones,
                                                        const Record* __restrict__ recs, Opts op, int cull,
                                                        uint32_t* __restrict__ tiles_out,
                                                        uint32_t* __restrict__ items_out,
                                                        uint32_t* __restrict__ hparts, int hpass, int hbits) {
  constexpr int kSpan = kBlock * kExpandPer;
  const int64_t m = dyn_count(m_cap, dyn_m);
  const int64_t total = dyn_count(total_cap, dyn_total);
  const int64_t block0 = (int64_t)blockIdx.x * kSpan;
  if (block0 >= total || m <= 0) return;  // uniform over the block
  __shared__ uint32_t s_tile[kSpan + kSpan / 32];  // slots spread by stage_slot
  __shared__ uint32_t s_item[kSpan + kSpan / 32];
  __shared__ uint32_t s_offs[kSpan + 1];  // offs[jlo + k]; past the last owner: 0xffffffff
  __shared__ uint32_t s_h[kHistPasses][256];  // this block's digit counts of the kept tile ids
  __shared__ uint32_t s_kept;
  __shared__ int64_t s_jlo;
  if (hpass) {
#pragma unroll
    for (int p = 0; p < kHistPasses; ++p) s_h[p][threadIdx.x] = 0u;
    if (threadIdx.x == 0) s_kept = 0u;
  }
  if (threadIdx.x < 64) {
    // owner of block0 (last j with offs[j] <= block0) in [lo, hi): each round
    // probes 64 evenly spaced offsets; offs is increasing and offs[0] = 0
    const int lane = threadIdx.x;
    int64_t lo = 0, hi = m;
    while (hi - lo > 1) {
      const int64_t step = (hi - lo + 63) / 64;
      const int64_t idx = lo + (int64_t)lane * step;
      const uint64_t le = __builtin_amdgcn_ballot_w64(idx < hi && (int64_t)offs[idx] <= block0);
      lo += (int64_t)(63 - __builtin_clzll(le)) * step;  // lane 0 always holds
      hi = min(lo + step, hi);
    }
    if (lane == 0) s_jlo = lo;
  }
  __syncthreads();
  // every owner of an entry of the block is one of jlo .. jlo + kSpan - 1
  const int64_t jlo = s_jlo;
  const int64_t S = min<int64_t>(kSpan + 1, m - jlo);
  for (int k = threadIdx.x; k < kSpan + 1; k += kBlock) s_offs[k] = k < S ? offs[jlo + k] : 0xffffffffu;
  __syncthreads();

  uint32_t my_kept = 0u, run_d = 0u, run_n = 0u;  // run of equal upper digits along this lane's entries
  const int64_t e0 = block0 + (int64_t)threadIdx.x * kExpandPer;
  const bool fixed = op.lambda_mode == 1;
  if (e0 < total) {
    const int cnt = (int)min<int64_t>(kExpandPer, total - e0);
    // local owner of e0: last k with s_offs[k] <= e0; it is at most
    // e0 - block0, since every owner covers at least one entry
    int lo = 0, hi = (int)min<int64_t>(S, (int64_t)threadIdx.x * kExpandPer + 1);
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if ((int64_t)s_offs[mid] <= e0) lo = mid; else hi = mid;
    }
    // tile ids and items of the lane's entries
    uint32_t tile[kExpandPer], item[kExpandPer];
    int jl = lo, cur = -1;
    uint32_t it = 0, tx = 0, ty = 0, tx0 = 0, tx1 = 0, row = 0, base = 0;
#pragma unroll
    for (int k = 0; k < kExpandPer; ++k) {
      tile[k] = kDropKey;
      item[k] = 0u;
      if (k < cnt) {
        const int64_t e = e0 + k;
        while ((int64_t)s_offs[jl + 1] <= e) ++jl;
        if (jl != cur) {
          cur = jl;
          it = items[jlo + jl];
          const uint32_t local = (uint32_t)(e - (int64_t)s_offs[jl]);
          const uint2 r = rects[it];
          tx0 = (r.x & 0xffffu) >> 1;
          tx1 = (r.x >> 16) >> 1;
          const uint32_t ty0 = (r.y & 0xffffu) >> 1;
          const uint32_t wt = tx1 - tx0 + 1u;
          const ViewDev& V = views[small_quotient(it, (uint32_t)n)];
          const uint32_t dy = small_quotient(local, wt);
          ty = ty0 + dy;
          tx = tx0 + (local - dy * wt);
          row = (uint32_t)V.tiles_x;
          base = (uint32_t)V.tile_base;
        } else if (++tx > tx1) {
          tx = tx0;
          ++ty;
        }
        tile[k] = base + ty * row + tx;
        item[k] = it;
      }
    }
    if (cull) {
      // the cone of entry k + 1 is loaded while entry k is tested
      float4 c0 = tcones[4 * (size_t)tile[0]], c1 = tcones[4 * (size_t)tile[0] + 1];
      float4 c2 = tcones[4 * (size_t)tile[0] + 2], c3 = tcones[4 * (size_t)tile[0] + 3];
      const float4* rp = reinterpret_cast<const float4*>(recs + item[0]);
      float4 p0 = rp[0], p1 = rp[1], p2 = rp[2], p3 = rp[3];
#pragma unroll
      for (int k = 0; k < kExpandPer; ++k) {
        if (k >= cnt) break;
        float4 n0 = c0, n1 = c1, n2 = c2, n3 = c3;
        if (k + 1 < cnt) {
          const float4* cp = tcones + 4 * (size_t)tile[k + 1];
          n0 = cp[0]; n1 = cp[1]; n2 = cp[2]; n3 = cp[3];
        }
        if (k > 0 && item[k] != item[k - 1]) {
          const float4* rq = reinterpret_cast<const float4*>(recs + item[k]);
          p0 = rq[0]; p1 = rq[1]; p2 = rq[2]; p3 = rq[3];
        }
        QuadCone Q;
        Q.d[0][0] = c0.x; Q.d[0][1] = c0.y; Q.d[0][2] = c0.z;
        Q.d[1][0] = c1.x; Q.d[1][1] = c1.y; Q.d[1][2] = c1.z;
        Q.d[2][0] = c2.x; Q.d[2][1] = c2.y; Q.d[2][2] = c2.z;
        Q.d[3][0] = c3.x; Q.d[3][1] = c3.y; Q.d[3][2] = c3.z;
        Q.valid = c0.w != 0.0f;
        if (!cone_meets_quad(p0, p1, p2, p3, Q, op.log2_amin, fixed)) tile[k] = kDropKey;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
      }
    }
#pragma unroll
    for (int k = 0; k < kExpandPer; ++k) {
      if (k >= cnt) break;
      const uint32_t t = tile[k];
      if (hpass && t != kDropKey) {
        ++my_kept;
        atomicAdd(&s_h[0][t & ((1u << hbits) - 1u)], 1u);
        if (hpass > 1) {
          const uint32_t d1 = t >> hbits;  // a kept tile id has at most 2 hbits bits
          if (d1 != run_d) {
            if (run_n) atomicAdd(&s_h[1][run_d], run_n);
            run_d = d1;
            run_n = 0u;
          }
          ++run_n;
        }
      }
      const int sl = stage_slot(threadIdx.x * kExpandPer + k);
      s_tile[sl] = t;
      s_item[sl] = item[k];
    }
  }
  if (hpass) {
    if (run_n) atomicAdd(&s_h[1][run_d], run_n);
    if (my_kept) atomicAdd(&s_kept, my_kept);
  }
  __syncthreads();
  if (hpass) {
    uint32_t* hp = hparts + (blockIdx.x % kHistCopies) * kHistStride;
    for (int p = 0; p < hpass; ++p) {
      const uint32_t c = s_h[p][threadIdx.x];
      if (c) atomicAdd(&hp[p * 256 + threadIdx.x], c);
    }
    if (threadIdx.x == 0 && s_kept) atomicAdd(&hp[kHistKept], s_kept);
  }
#pragma unroll
  for (int k = 0; k < kExpandPer; ++k) {
    const int sl = k * kBlock + threadIdx.x;
    const int64_t e = block0 + sl;
    if (e < total) {
      tiles_out[e] = s_tile[stage_slot(sl)];
      items_out[e] = s_item[stage_slot(sl)];
    }
  }
}

// Tile ranges of the sorted tile ids; with `list`, also list[total ..
// total + 8) = 0 (padding read by the render's window loads).
__global__ __launch_bounds__(kBlock) void ranges_kernel(const uint32_t* __restrict__ tiles, int64_t total_cap,
                                                        const unsigned long long* __restrict__ dyn,
                                                        int64_t ntiles, uint32_t* __restrict__ ranges,
                                                        uint32_t* __restrict__ list) {
  const int64_t total = dyn_count(total_cap, dyn);
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  const int64_t e0 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (list && e0 < 8) list[total + e0] = 0u;
  if (total == 0) {
    for (int64_t t = e0; t <= ntiles; t += stride) ranges[t] = 0u;
    return;
  }
  // grid-stride: the grid is bounded, however large the capacity
  for (int64_t e = e0; e < total; e += stride) {
    const int64_t cur = tiles[e];
    const int64_t prev = e > 0 ? (int64_t)tiles[e - 1] : -1;
    for (int64_t t = prev + 1; t <= cur; ++t) ranges[t] = (uint32_t)e;
    if (e == total - 1)
      for (int64_t t = cur + 1; t <= ntiles; ++t) ranges[t] = (uint32_t)total;
  }
}

__global__ __launch_bounds__(kBlock) void fill_u32_kernel(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = v;
}

// p1[0 .. n1) = 0 and p2[0 .. n2) = 0 in one launch.
__global__ __launch_bounds__(kBlock) void zero2_u32_kernel(uint32_t* __restrict__ p1, int64_t n1,
                                                           uint32_t* __restrict__ p2, int64_t n2) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n1) p1[i] = 0u;
  else if (i - n1 < n2) p2[i - n1] = 0u;
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

// Workspace of radix_sort, in u32 words: histograms, then two
// status tables of 256 words per 2048-key block.
int64_t radix_work_words(int64_t n_cap) { return kWorkHead + 2 * 256 * ((n_cap + kOSItems - 1) / kOSItems); }

// Stable sort of n0 keys (filtered; values = in_v, or the key index when
// in_v is null) by npass 8-bit digits from bit shift0.  Pass 0 reads (in_k,
// in_v) with the n0 count, the filter and (with drop) leaves out kDropKey
// keys, counting the rest into *kept when given; later passes read n1 keys
// (the filtered count, read on the device when dyn1 is given).  Passes write
// A, B, A, ...: the result is in A for odd npass, in B for even.
int64_t radix_zero_words(int64_t nmax) {
  const int items = kBlock * os_per(nmax);
  return kWorkHead + 256 * os_blocks(nmax, items);
}

void radix_sort(hipStream_t st, const uint32_t* in_k, const uint32_t* in_v, const uint32_t* filter, bool drop,
                int64_t n0_cap, const unsigned long long* dyn0, int64_t n1_cap, const unsigned long long* dyn1,
                int shift0, int npass, uint32_t* ak, uint32_t* av, uint32_t* bk, uint32_t* bv, uint32_t* work,
                unsigned long long* kept, unsigned long long* err, const uint32_t* hparts, int bits, bool zeroed) {
  if (n0_cap <= 0 || npass <= 0) return;
  const int64_t nmax = std::max(n0_cap, n1_cap);
  const int per = os_per(nmax);  // chunk size by sort size
  const int items = kBlock * per;
  const int64_t rows = 256 * os_blocks(nmax, items);
  const uint32_t dmask = (1u << bits) - 1u;
  uint32_t* ghist = work;
  uint32_t* stat[2] = {work + kWorkHead, work + kWorkHead + rows};
  if (hparts) {
    // the producer already counted the digits into partial histograms:
    // sum them into the histograms, clear the first status table
    hipLaunchKernelGGL(hist_prepare_kernel, dim3(grid_for(kWorkHead + rows, kBlock)), dim3(kBlock), 0, st, work,
                       (int64_t)kWorkHead + rows, hparts, npass, kept);
  } else {
    // histograms and the first status table start at zero
    if (!zeroed)
      hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(kWorkHead + rows, kBlock)), dim3(kBlock), 0, st, work,
                         (int64_t)kWorkHead + rows, 0u);
    // few blocks: every block adds its counts to the same 256 words per pass
    const unsigned ug = (unsigned)std::min<int64_t>(std::max<int64_t>(grid_for(n0_cap, kBlock), 1), 256);
    hipLaunchKernelGGL(radix_upsweep_kernel, dim3(ug), dim3(kBlock), 0, st, in_k, filter, drop ? 1 : 0, n0_cap,
                       dyn0, shift0, bits, npass, ghist, kept);
  }
  const uint32_t *sk = in_k, *sv = in_v;
  for (int p = 0; p < npass; ++p) {
    uint32_t* ok = (p % 2 == 0) ? ak : bk;
    uint32_t* ov = (p % 2 == 0) ? av : bv;
    const int64_t ncap = p == 0 ? n0_cap : n1_cap;
    const unsigned long long* dy = p == 0 ? dyn0 : dyn1;
    const unsigned nb = (unsigned)std::max<int64_t>(os_blocks(ncap, items), 1);
    auto kern = per == kOSPerBig ? radix_onesweep_kernel<kOSPerBig>
                : per == kOSPer      ? radix_onesweep_kernel<kOSPer>
                                     : radix_onesweep_kernel<kOSPerSmall>;
    hipLaunchKernelGGL(kern, dim3(nb), dim3(kBlock), 0, st, sk, sv, p == 0 ? filter : nullptr, (p == 0 && drop) ? 1 : 0,
                       ncap, dy, shift0 + bits * p, dmask, (const uint32_t*)(ghist + 256 * p), stat[p % 2],
                       p + 1 < npass ? stat[(p + 1) % 2] : nullptr, ok, ov, err);
    sk = ok;
    sv = ov;
  }
}

void launch_gather_counts(hipStream_t st, const uint32_t* items, int64_t m_cap, const unsigned long long* dyn,
                          const uint32_t* counts, uint32_t* out) {
  if (m_cap <= 0) return;
  hipLaunchKernelGGL(gather_counts_kernel, dim3(grid_for(m_cap, kBlock)), dim3(kBlock), 0, st, items, m_cap, dyn,
                     counts, out);
}

void gather_scan(hipStream_t st, const uint32_t* items, int64_t m_cap, const unsigned long long* dyn,
                 const uint32_t* counts, uint32_t* out, uint32_t* scratch) {
  if (m_cap <= 0) return;
  const int64_t nb = (m_cap + kTileItems - 1) / kTileItems;
  if (nb > kGatherScanTiles) {
    launch_gather_counts(st, items, m_cap, dyn, counts, out);
    scan_exclusive(st, out, out, m_cap, scratch);
    return;
  }
  hipLaunchKernelGGL(gather_reduce_kernel, dim3((unsigned)nb), dim3(kBlock), 0, st, items, m_cap, dyn, counts, out,
                     scratch);
  hipLaunchKernelGGL(nb >= 64 ? gathered_scan_kernel<true> : gathered_scan_kernel<false>, dim3((unsigned)nb),
                     dim3(kBlock), 0, st, out, m_cap, (const uint32_t*)scratch, out);
}

void launch_tile_cones(hipStream_t st, const ViewDev* views, int nviews, const float2* dtab, int64_t ntiles,
                       float4* out, uint32_t* zero, int64_t nzero) {
  if (ntiles <= 0 && nzero <= 0) return;
  hipLaunchKernelGGL(tile_cones_kernel, dim3(grid_for(std::max(ntiles, nzero), kBlock)), dim3(kBlock), 0, st, views,
                     nviews, dtab, ntiles, out, zero, nzero);
}

void launch_expand(hipStream_t st, const uint32_t* items, const uint32_t* offs, int64_t m_cap,
                   const unsigned long long* dyn_m, int64_t total_cap, const unsigned long long* dyn_total,
                   const uint2* rects, const ViewDev* views, int64_t n, const float4* tcones, const Record* recs,
                   const Opts& op, uint32_t* tiles_out, uint32_t* items_out, uint32_t* hparts, int hpass,
                   int hbits) {
  if (total_cap <= 0) return;
  hipLaunchKernelGGL(expand_kernel, dim3(grid_for(total_cap, (int64_t)kBlock * kExpandPer)), dim3(kBlock), 0, st,
                     items, offs, m_cap, dyn_m, total_cap, dyn_total, rects, views, n, tcones, recs, op,
                     op.cone_cull, tiles_out, items_out, hparts, hpass, hbits);
}

void launch_ranges(hipStream_t st, const uint32_t* tiles, int64_t total_cap, const unsigned long long* dyn,
                   int64_t ntiles, uint32_t* ranges, uint32_t* list) {
  if (total_cap <= 0 && !dyn) {
    hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(ntiles + 1, kBlock)), dim3(kBlock), 0, st, ranges, ntiles + 1,
                       0u);
    return;
  }
  const int64_t g = std::max<int64_t>(total_cap, ntiles + 1);
  hipLaunchKernelGGL(ranges_kernel, dim3(std::min<unsigned>(grid_for(g, kBlock), 8192u)), dim3(kBlock), 0, st, tiles,
                     total_cap, dyn, ntiles, ranges, list);
}

void launch_capacity_guard(hipStream_t st, unsigned long long* stats, int64_t cap) {
  hipLaunchKernelGGL(capacity_guard_kernel, dim3(1), dim3(64), 0, st, stats, cap);
}

void launch_zero2_u32(hipStream_t st, uint32_t* p1, int64_t n1, uint32_t* p2, int64_t n2) {
  if (n1 + n2 <= 0) return;
  hipLaunchKernelGGL(zero2_u32_kernel, dim3(grid_for(n1 + n2, kBlock)), dim3(kBlock), 0, st, p1, n1, p2, n2);
}

void launch_fill_u32(hipStream_t st, uint32_t* p, int64_t n, uint32_t v) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, st, p, n, v);
}

}  // namespace geer
