// Stage (b): association list.  Alg. 1 DuplicateWithKeys / SortByKeys /
// IdentifyFrustumRanges, arranged so the wide sort only touches tile ids:
//   1. stable LSD radix sort of the visible items by their 32-bit depth key
//      in four 8-bit passes: the first compacts the visible items out of all
//      items, the last also writes the exclusive scan of the items' tile
//      counts in depth order (the entry offsets);
//   2. expansion of every item into (tile, item) entries in depth order,
//      balanced over entries (4 per lane; owners found through LDS), with
//      the contribution-cone cull marking the entries no ray can see;
//   3. stable LSD radix sort of the entries by global tile id, so each tile's
//      run stays in (depth key, item) order; the first pass leaves out the
//      marked entries;
//   4. run boundaries -> ranges[tile].
// Every radix pass is one kernel with decoupled look-back (below).
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

// ----------------------------------------------------------------- radix --
//
// Stable LSD radix sort with 8-bit digits, one kernel per pass ("onesweep"
// with decoupled look-back).  The digit counts of every pass are known before
// the first pass: an upsweep kernel counts them over the (filtered) input,
// or the producer of the keys counted them into partial copies that each
// pass sums for itself.  In a pass, block b takes the b-th chunk of keys
// (1024 to 4096 keys by sort size, os_per), ranks its keys stably (per wave:
// ballot match on the digit; across waves and slices: running counts in
// LDS), publishes its per-digit counts, and walks back over earlier blocks'
// published counts -- stopping at the first that already holds its inclusive
// prefix -- to find where its run of each digit starts.  Keys are then
// reordered by digit in LDS and written out as contiguous runs.
//
// A status word is [flag:2 | count:30].  A weighted pass also carries each
// key's weight (wts[value]): its status words are 64 bits wide, the word
// above in the high half and the digit's weight sum (mod 2^32) in the low
// half, loaded and stored as one, and it writes for every output position the
// exclusive prefix sum of the weights in sorted order.  The depth order's last
// pass is weighted by the items' tile counts, so it also yields the entry
// offsets of the expansion.
//
// The look-back spin is bounded and reports a stall through an error word
// instead of hanging.  A block waits only on blocks with lower indices, and
// each XCD dispatches the workgroups of a launch in index order, so while
// the pass has the device to itself the lowest unfinished block is always
// resident and the walk always ends.  Kernels of other streams break that:
// higher blocks of several passes can hold every slot while they wait on
// lower blocks that are not dispatched.  Work that may run beside other
// streams (render plans) therefore numbers the chunks by atomic tickets taken
// as blocks start, so every block waited on is running.  (Tickets serialise:
// they come one at a time off one counter, which staggers the 692 blocks of a
// 2.8M-key pass over about 9 us, so eager forwards and training plans, one
// association at a time, go without.)

// Statuses read per look-back round.  Fewer loads per round beat a wider
// reach: every polling block re-reads its window, so wide windows flood the
// status table's lines (passes of 2.8M keys: 16 -> 30.4 us, 8 -> 27.9, 4 -> 26.7,
// 2 -> 27.8).
constexpr int kLookBack = 4;
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
// Work head: the digit counts of up to 4 passes, then the weighted counts of
// the last pass's digits (padded).
constexpr int kWorkHead = 5 * 256 + 64;
// Entries per expansion block: the weighted depth pass records the owner of
// every multiple of it, where an expansion block starts.
constexpr int kOwnerSpan = 1024;

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
// expansion found unable to contribute).
constexpr uint32_t kDropKey = 0xffffffffu;

// Digit counts (digits of `bits` bits from shift0) of every pass over the
// keys i < live count with filter[i] != 0 (every key without a filter; with
// drop, not kDropKey), added into ghist (npass rows of 256 words); with
// whist, the filter values summed per digit of the last pass are added into
// whist.
__global__ __launch_bounds__(kBlock) void radix_upsweep_kernel(const uint32_t* __restrict__ keys,
                                                               const uint32_t* __restrict__ filter, int drop,
                                                               int64_t n_cap,
                                                               const unsigned long long* __restrict__ dyn,
                                                               int shift0, int bits, int npass,
                                                               uint32_t* __restrict__ ghist,
                                                               uint32_t* __restrict__ whist) {
  const uint32_t dmask = (1u << bits) - 1u;
  const int64_t n = dyn_count(n_cap, dyn);
  __shared__ uint32_t h[4][256];
  __shared__ uint32_t hw[256];
#pragma unroll
  for (int p = 0; p < 4; ++p) h[p][threadIdx.x] = 0u;
  hw[threadIdx.x] = 0u;
  __syncthreads();
  const int lshift = shift0 + bits * (npass - 1);
  auto count = [&](uint32_t f, uint32_t k) {
    for (int p = 0; p < npass; ++p) atomicAdd(&h[p][(k >> (shift0 + bits * p)) & dmask], 1u);
    if (whist) atomicAdd(&hw[(k >> lshift) & dmask], f);
  };
  // grid-stride; with many keys per thread, 8 keys per step with all their
  // loads in flight together
  constexpr int kUp = 8;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  if (n <= 2 * stride) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
      const uint32_t f = filter ? filter[i] : 1u;
      const uint32_t k = keys[i];
      if (f != 0u && !(drop && k == kDropKey)) count(f, k);
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
      for (int u = 0; u < kUp; ++u)
        if (i0 + u * stride < n && f[u] != 0u && !(drop && k[u] == kDropKey)) count(f[u], k[u]);
    }
  }
  __syncthreads();
  for (int p = 0; p < npass; ++p) {
    const uint32_t c = h[p][threadIdx.x];
    if (c) atomicAdd(&ghist[p * 256 + threadIdx.x], c);
  }
  if (whist && hw[threadIdx.x]) atomicAdd(&whist[threadIdx.x], hw[threadIdx.x]);
}

// Partial digit histograms filled by a producer kernel: kHistCopies copies
// (block b adds to copy b % kHistCopies), each with 256 words per pass for
// up to kHistPasses passes; every pass of the sort sums the copies of its
// digits.
constexpr int kHistCopies = 16;
constexpr int kHistPasses = 2;
constexpr int kHistStride = 256 * kHistPasses + 64;

// Arguments of one radix pass.
struct PassArgs {
  const uint32_t* keys_in;
  const uint32_t* vals_in;  // null: the key's index
  const uint32_t* filter;   // null: every key; else only keys with filter[i] != 0
  int drop;                 // leave out kDropKey keys
  int64_t n_cap;
  const unsigned long long* dyn;  // live key count (null: n_cap)
  int shift;
  uint32_t dmask;  // digit = (key >> shift) & dmask, below 256
  const uint32_t* ghist;  // this pass's digit counts, summed over hcopies copies hstride words apart
  int hcopies, hstride;
  unsigned long long* kept_out;  // with it, block 0 stores the number of keys sorted
  const uint32_t* whist;  // weighted pass: weight totals per digit
  const uint32_t* wts;    // weighted pass: weight of value v (v < wts_n)
  int64_t wts_n;
  void* status;           // this pass's status table, one row per block
  void* status_next;      // the next pass's table (row b cleared by block b), or null
  int next_row_words;     // u32 words of a row of the next pass's table
  uint32_t* keys_out;     // null: keys are not written
  uint32_t* vals_out;
  uint32_t* wout;         // weighted pass: exclusive prefix of the weights in sorted order
  // weighted pass, or null: owners[b] = the output position whose weight run
  // [wout, wout + weight) holds b * kOwnerSpan, for b < owners_n
  uint32_t* owners;
  int64_t owners_n;
  unsigned long long* err;
  uint32_t* ticket;  // with it, a block's chunk is the ticket it takes off this counter (starts at 0)
  uint32_t spin_limit;  // polls of the look-back before it gives up
};

template <bool kW>
struct StatusWord;
template <>
struct StatusWord<false> {
  using T = uint32_t;
  __device__ static T make(uint32_t flag, uint32_t cnt, uint32_t) { return flag | cnt; }
  __device__ static uint32_t flag(T v) { return v & ~kValMask; }
  __device__ static uint32_t cnt(T v) { return v & kValMask; }
  __device__ static uint32_t wsum(T) { return 0u; }
};
template <>
struct StatusWord<true> {
  using T = unsigned long long;
  __device__ static T make(uint32_t flag, uint32_t cnt, uint32_t ws) {
    return ((unsigned long long)(flag | cnt) << 32) | ws;
  }
  __device__ static uint32_t flag(T v) { return (uint32_t)(v >> 32) & ~kValMask; }
  __device__ static uint32_t cnt(T v) { return (uint32_t)(v >> 32) & kValMask; }
  __device__ static uint32_t wsum(T v) { return (uint32_t)v; }
};

template <int kPer, bool kWeighted>
__global__ __launch_bounds__(kBlock) void radix_pass_kernel(const PassArgs a) {
  constexpr int kItems = kBlock * kPer;
  using SW = StatusWord<kWeighted>;
  using Stat = typename SW::T;
  __shared__ uint32_t s_cnt[4][256];  // per-wave running digit counts, then per-wave offsets
  __shared__ uint32_t s_loc[256];     // block-local start of each digit
  __shared__ uint32_t s_glob[256];    // global start of this block's run of each digit
  __shared__ uint32_t s_key[kItems], s_val[kItems];
  __shared__ uint32_t s_wt[kWeighted ? kItems : 1];  // weights, then their exclusive prefix
  __shared__ uint32_t s_wsum[kWeighted ? 256 : 1];   // the block's weight per digit
  __shared__ uint32_t s_wglob[kWeighted ? 256 : 1];  // weight before this block's run of each digit
  __shared__ uint32_t s_w[4];

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  // the grid is sized for the capacity: blocks past the live key count leave
  const int64_t n = dyn_count(a.n_cap, a.dyn);
  if ((int64_t)blockIdx.x >= os_blocks(n, kItems)) return;
  int64_t blk = blockIdx.x;
  if (a.ticket) {
    // chunks in the order blocks start: the walk then only ever waits on
    // blocks that are running, also when kernels of other streams share the
    // device (in-order dispatch holds within one kernel only).  Only the
    // blocks of live chunks take one: they are as many as the chunks.
    __shared__ uint32_t s_ticket;
    if (tid == 0) s_ticket = atomicAdd(a.ticket, 1u);
    __syncthreads();
    blk = s_ticket;
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) s_cnt[q][tid] = 0u;
  if (kWeighted) s_wsum[tid] = 0u;
  if (a.status_next) {  // this block's row of the next pass's table starts clear
    uint32_t* nx = (uint32_t*)a.status_next + blk * (int64_t)a.next_row_words;
    for (int i = tid; i < a.next_row_words; i += kBlock) nx[i] = 0u;
  }
  __syncthreads();
  // this pass's count of digit tid: the loads go out with the keys' and are
  // only summed after the look-back
  uint32_t gh[kHistCopies];
#pragma unroll
  for (int c = 0; c < kHistCopies; ++c) gh[c] = c < a.hcopies ? a.ghist[(int64_t)c * a.hstride + tid] : 0u;
  const uint32_t wh = kWeighted ? a.whist[tid] : 0u;

  // stable ranks within the wave: wave w owns keys [base, base + 64 kPer).
  // Every slice's filter word, key and value are loaded first, from an index
  // clamped into [0, n) (n > 0 here), so the loads are independent and in
  // flight together; the ranking below only waits for them once.
  const int64_t base = blk * kItems + (int64_t)w * 64 * kPer;
  const uint64_t lt = lanemask_lt();
  uint32_t key[kPer], val[kPer], rank[kPer], flt[kPer], wt[kPer];
#pragma unroll
  for (int sl = 0; sl < kPer; ++sl) {
    const int64_t i = base + sl * 64 + lane;
    const int64_t ic = i < n ? i : n - 1;
    flt[sl] = a.filter ? a.filter[ic] : 1u;
    key[sl] = a.keys_in[ic];
    val[sl] = a.vals_in ? a.vals_in[ic] : (uint32_t)i;
  }
  if (kWeighted) {
#pragma unroll
    for (int sl = 0; sl < kPer; ++sl) wt[sl] = a.wts[min<int64_t>(val[sl], a.wts_n - 1)];  // values are set
  }
  uint32_t act = 0u;
#pragma unroll
  for (int sl = 0; sl < kPer; ++sl) {
    const int64_t i = base + sl * 64 + lane;
    bool on = i < n && flt[sl] != 0u;
    if (a.drop) on = on && key[sl] != kDropKey;
    if (!on) {
      key[sl] = 0u;
      val[sl] = 0u;
      wt[sl] = 0u;
    }
    const uint32_t d = (key[sl] >> a.shift) & a.dmask;
    uint64_t m = __builtin_amdgcn_ballot_w64(on);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint64_t bb = __builtin_amdgcn_ballot_w64(((d >> b) & 1u) != 0u);
      m &= ((d >> b) & 1u) ? bb : ~bb;
    }
    const uint32_t r = (uint32_t)__popcll(m & lt);
    const uint32_t pre = on ? s_cnt[w][d] : 0u;  // every lane of a digit reads before its leader writes
    rank[sl] = pre + r;
    if (on && r == 0u) s_cnt[w][d] = pre + (uint32_t)__popcll(m);
    if (kWeighted && on) atomicAdd(&s_wsum[d], wt[sl]);
    act |= (on ? 1u : 0u) << sl;
    // the wave's next slice reads these counts (LDS order within a wave)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  __syncthreads();

  // per digit (thread tid): wave offsets and the block's count, published
  Stat* const status = (Stat*)a.status;
  const uint32_t c0 = s_cnt[0][tid], c1 = s_cnt[1][tid], c2 = s_cnt[2][tid], c3 = s_cnt[3][tid];
  const uint32_t tot = c0 + c1 + c2 + c3;
  const uint32_t bw = kWeighted ? s_wsum[tid] : 0u;
  s_cnt[0][tid] = 0u;
  s_cnt[1][tid] = c0;
  s_cnt[2][tid] = c0 + c1;
  s_cnt[3][tid] = c0 + c1 + c2;
  __hip_atomic_store(&status[blk * 256 + tid], SW::make(blk == 0 ? kFlagInc : kFlagAgg, tot, bw),
                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);

  // decoupled look-back over the earlier blocks, kLookBack statuses per
  // round (independent loads in flight together): add aggregates from the
  // nearest block back until an inclusive prefix; stop at a block that has
  // not published yet and poll again from it.  Block 0's aggregate is its
  // inclusive prefix, so the walk also ends after it.
  // Digits above the pass's digit mask hold no keys: their threads skip the
  // walk (every block's do), which spares the status table their polling.
  uint32_t excl = 0u, wexcl = 0u, spins = 0u;
  for (int64_t j = (uint32_t)tid <= a.dmask ? blk - 1 : -1; j >= 0;) {
    Stat v[kLookBack];
#pragma unroll
    for (int q = 0; q < kLookBack; ++q)
      v[q] = j - q >= 0 ? __hip_atomic_load(&status[(j - q) * 256 + tid], __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT)
                        : SW::make(kFlagInc, 0u, 0u);
    int q = 0;
    bool done = false;
#pragma unroll
    for (int r = 0; r < kLookBack; ++r) {
      if (q != r) continue;
      const uint32_t f = SW::flag(v[r]);
      if (f == 0u) continue;  // not published: poll from here again
      excl += SW::cnt(v[r]);
      wexcl += SW::wsum(v[r]);
      if (f == kFlagInc) done = true;
      else q = r + 1;
    }
    if (done) break;
    j -= q;
    if (q < kLookBack) {
      if (++spins > a.spin_limit) {
        atomicOr(a.err, 1ull);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  if (blk > 0)
    __hip_atomic_store(&status[blk * 256 + tid], SW::make(kFlagInc, excl + tot, wexcl + bw), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);

  // global starts of the digits (counts of smaller digits) and block-local ones
  uint32_t ghs = 0u;
#pragma unroll
  for (int c = 0; c < kHistCopies; ++c) ghs += gh[c];
  uint32_t gtotal, ltotal, wtotal;
  const uint32_t gstart = block_excl_scan256(ghs, s_w, gtotal);
  const uint32_t lstart = block_excl_scan256(tot, s_w, ltotal);
  s_glob[tid] = gstart + excl;
  s_loc[tid] = lstart;
  if (kWeighted) s_wglob[tid] = block_excl_scan256(wh, s_w, wtotal) + wexcl;
  if (a.kept_out && blk == 0 && tid == 0) *a.kept_out = gtotal;  // the keys this sort keeps
  __syncthreads();

  // reorder by digit in LDS, then write contiguous runs
#pragma unroll
  for (int sl = 0; sl < kPer; ++sl) {
    if ((act >> sl) & 1u) {
      const uint32_t d = (key[sl] >> a.shift) & a.dmask;
      const uint32_t lp = s_loc[d] + s_cnt[w][d] + rank[sl];
      s_key[lp] = key[sl];
      s_val[lp] = val[sl];
      if (kWeighted) s_wt[lp] = wt[sl];
    }
  }
  __syncthreads();
  uint32_t wt_total = 0u;
  if (kWeighted) {
    // exclusive prefix of the weights in the block's sorted order (in place;
    // thread t scans kPer consecutive positions)
    uint32_t v[kPer], s = 0u;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const uint32_t i = (uint32_t)(tid * kPer + k);
      v[k] = i < ltotal ? s_wt[i] : 0u;
      s += v[k];
    }
    uint32_t run = block_excl_scan256(s, s_w, wt_total);
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const uint32_t i = (uint32_t)(tid * kPer + k);
      if (i < ltotal) s_wt[i] = run;
      run += v[k];
    }
    __syncthreads();
  }
  // (a stalled look-back or inputs a stalled pass left behind can put g past
  // the keys; such keys are not written)
  for (uint32_t i = tid; i < ltotal; i += kBlock) {
    const uint32_t k = s_key[i];
    const uint32_t d = (k >> a.shift) & a.dmask;
    const uint32_t g = s_glob[d] + (i - s_loc[d]);
    if ((int64_t)g >= n) continue;
    if (a.keys_out) a.keys_out[g] = k;
    a.vals_out[g] = s_val[i];
    if (kWeighted) {
      const uint32_t o = s_wglob[d] + (s_wt[i] - s_wt[s_loc[d]]);
      a.wout[g] = o;
      if (a.owners) {
        // the expansion blocks whose first entry is one of this key's
        const uint32_t c = (i + 1 < ltotal ? s_wt[i + 1] : wt_total) - s_wt[i];
        for (uint64_t b = ((uint64_t)o + kOwnerSpan - 1) / kOwnerSpan;
             b * kOwnerSpan < (uint64_t)o + c && (int64_t)b < a.owners_n; ++b)
          a.owners[b] = g;
      }
    }
  }
}

int hist_parts_words() { return kHistCopies * kHistStride; }

int64_t owner_words(int64_t ecap) { return std::max<int64_t>(ecap, 1) / kOwnerSpan + 2; }

// ------------------------------------------------------------ expansion --

constexpr int kExpandPer = 4;
constexpr int kExpandSpan = kBlock * kExpandPer;  // entries per expansion block
constexpr int kConeStride = 5;                    // float4 per tile in the cull's table
constexpr int kWaveSlots = kExpandSpan / 4 + kExpandSpan / 128;  // staging slots of one wave

// Cone of every 16x16 tile of every view for the expansion's cull,
// kConeStride float4 per tile: corner direction k in .xyz of entry k and the
// cone's validity in .w of entry 0; entry 4 holds a centre direction c and a
// radius rho with |d - c| <= rho for every ray d of the tile (rho = -1 when
// the corners do not span the tile's rays, or rho would exceed 1).  The
// corners span the tile's rays, and the cap of angular radius
// max_k angle(c, corner k) < 90 degrees around c holds them and so their
// spherical hull; rho is rounded up.
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
    out[kConeStride * t + k] =
        make_float4(Q.d[k][0], Q.d[k][1], Q.d[k][2], k == 0 ? (Q.valid ? 1.0f : 0.0f) : 0.0f);
  float c[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) c[i] = (Q.d[0][i] + Q.d[1][i]) + (Q.d[2][i] + Q.d[3][i]);
  const float cn = sqrtf(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
  float rho = -1.0f;
  if (Q.valid && cn > 0.0f) {
#pragma unroll
    for (int i = 0; i < 3; ++i) c[i] = c[i] / cn;
    rho = 0.0f;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float dx = Q.d[k][0] - c[0], dy = Q.d[k][1] - c[1], dz = Q.d[k][2] - c[2];
      rho = fmaxf(rho, sqrtf(dx * dx + dy * dy + dz * dz));
    }
    rho = rho < 1.0f ? fmaf(rho, 0x1p-10f, rho) + 0x1p-20f : -1.0f;
  }
  out[kConeStride * t + 4] = make_float4(c[0], c[1], c[2], rho);
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
// 1024 entries in LDS and writes them back lane-striped so every store is
// coalesced.  With `cull`, an entry whose Gaussian's contribution cone meets
// no ray of its tile gets the tile id kDropKey and is left out by the tile
// sort.  The kernel is bound by chains of dependent loads, so blocks are
// small (many waves in flight) and the chains short: one wave finds the
// owner of the block's first entry with a 64-way search (a few dependent
// loads instead of ~log2 m); the offsets and items of the owners that can
// start inside the block are staged in LDS, where each lane finds and walks
// its owners; the tile ids of all the lane's entries are derived first, so
// their cull data are loaded together.
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
                                                        uint32_t* __restrict__ hparts, int hpass, int hbits,
                                                        int64_t nitems, uint32_t ntiles,
                                                        const uint32_t* __restrict__ owners) {
  constexpr int kSpan = kExpandSpan;
  static_assert(kSpan == kOwnerSpan, "the depth order records the owners of kOwnerSpan-entry blocks");
  const int64_t m = dyn_count(m_cap, dyn_m);
  const int64_t total = dyn_count(total_cap, dyn_total);
  const int64_t block0 = (int64_t)blockIdx.x * kSpan;
  if (block0 >= total || m <= 0) return;  // uniform over the block
  __shared__ uint32_t s_tile[kSpan + kSpan / 32];  // slots spread by stage_slot
  __shared__ uint32_t s_item[kSpan + kSpan / 32];
  __shared__ uint32_t s_offs[kSpan + 1];  // offs[jlo + k]; past the last owner: 0xffffffff
  __shared__ uint32_t s_own[kSpan + 1];   // items[jlo + k]
  __shared__ uint8_t s_keep[kSpan];        // verdicts of the exact cull test, per wave
  __shared__ uint32_t s_h[kHistPasses][256];  // this block's digit counts of the kept tile ids
  if (hpass) {
#pragma unroll
    for (int p = 0; p < kHistPasses; ++p) s_h[p][threadIdx.x] = 0u;
  }
  // owner of block0 (last j with offs[j] <= block0), recorded by the depth
  // order's weighted pass (clamped, so that a stalled sort's leftovers stay in
  // bounds); every owner of an entry of the block is one of jlo .. jlo + kSpan - 1
  const int64_t jlo = min<int64_t>(owners[blockIdx.x], m - 1);
  const int64_t S = min<int64_t>(kSpan + 1, m - jlo);
  for (int k = threadIdx.x; k < kSpan + 1; k += kBlock) {
    s_offs[k] = k < S ? offs[jlo + k] : 0xffffffffu;
    // item ids are clamped to the items there are, so that a depth order a
    // stalled sort left inconsistent cannot send the reads out of bounds
    s_own[k] = k < S ? (uint32_t)min<int64_t>(items[jlo + k], nitems - 1) : 0u;
  }
  __syncthreads();

  uint32_t run_d = 0u, run_n = 0u;  // run of equal upper digits along this lane's entries
  const int64_t e0 = block0 + (int64_t)threadIdx.x * kExpandPer;
  const bool fixed = op.lambda_mode == 1;
  // every lane of the block goes through the cull (its wave-wide queue);
  // lanes past the end have no entries
  const int cnt = e0 < total ? (int)min<int64_t>(kExpandPer, total - e0) : 0;
  {
    // local owner of e0: last k with s_offs[k] <= e0; it is at most
    // e0 - block0, since every owner covers at least one entry
    int lo = 0, hi = cnt > 0 ? (int)min<int64_t>(S, (int64_t)threadIdx.x * kExpandPer + 1) : 0;
    const int jmax = (int)S - 1;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if ((int64_t)s_offs[mid] <= e0) lo = mid; else hi = mid;
    }
    // tile ids and items of the lane's entries
    uint32_t tile[kExpandPer], item[kExpandPer];
    int jl = lo, cur = -1;
    uint32_t it = 0, tx = 0, ty = 0, tx0 = 0, tx1 = 0, ty1 = 0, row = 0, base = 0;
#pragma unroll
    for (int k = 0; k < kExpandPer; ++k) {
      tile[k] = kDropKey;
      item[k] = 0u;
      if (k < cnt) {
        const int64_t e = e0 + k;
        while (jl < jmax && (int64_t)s_offs[jl + 1] <= e) ++jl;
        if (jl != cur) {
          cur = jl;
          it = s_own[jl];
          const uint32_t local = (uint32_t)(e - (int64_t)s_offs[jl]);
          const uint2 r = rects[it];
          tx0 = (r.x & 0xffffu) >> 1;
          tx1 = (r.x >> 16) >> 1;
          const uint32_t ty0 = (r.y & 0xffffu) >> 1;
          ty1 = (r.y >> 16) >> 1;
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
        // an entry past its owner's rectangle (only offsets a stalled sort
        // left behind make one) is dropped, so every tile id stays in the grid
        const uint32_t tid_ = base + ty * row + tx;
        tile[k] = (ty <= ty1 && tid_ < ntiles) ? tid_ : kDropKey;
        item[k] = it;
      }
    }
    if (cull) {
      // (1) Every entry: a cheap conservative verdict from the tile's centre
      // ray.  With g = G d and h(d) = |g_xy| - tau g_z, a ray contributes only
      // if h(d) <= 0, and |h(d) - h(c)| <= L |d - c| with
      // L = (1 + tau) |G|_F; so h(c) > L rho means no ray of the tile
      // contributes.  The margin 2^-16 L covers the FP32 rounding of h(c)
      // (about 2^-20 L) and of the tables' directions.  Entries it cannot
      // settle go to (2).
      float4 cr[kExpandPer];
#pragma unroll
      for (int k = 0; k < kExpandPer; ++k)
        cr[k] = k < cnt && tile[k] != kDropKey ? tcones[kConeStride * (size_t)tile[k] + 4]
                                               : make_float4(0.0f, 0.0f, 0.0f, -1.0f);
      uint32_t survive = 0u, cur = 0xffffffffu;
      int cls = 0;  // the item's verdict: 0 no ray reaches alpha_min, 1 every tile kept, 2 per tile
      float G[9] = {}, tau = 0.0f, lip = 0.0f;
#pragma unroll
      for (int k = 0; k < kExpandPer; ++k) {
        if (k >= cnt) break;
        if (tile[k] == kDropKey) continue;
        if (item[k] != cur) {
          cur = item[k];
          const float4* rp = reinterpret_cast<const float4*>(recs + cur);
          // the cull reads the record's geometry and qmax, never its rgb (which
          // a batch's colour kernel may still be writing)
          const float4 p0 = rp[0], p1 = rp[1], p2 = rp[2];
          const float4 p3 = make_float4(0.0f, 0.0f, 0.0f, recs[cur].qmax);
          G[0] = p0.x; G[1] = p0.y; G[2] = p0.z; G[3] = p0.w;
          G[4] = p1.x; G[5] = p1.y; G[6] = p1.z; G[7] = p1.w; G[8] = p2.x;
          // the contribution threshold of the exact test, with its margins
          float Qc = (p2.z - op.log2_amin) * __builtin_amdgcn_rcpf(-p2.y);
          if (fixed) Qc = fminf(Qc, p3.w);
          Qc = fmaf(Qc, 0x1p-8f, Qc) + 0x1p-20f;
          cls = !(Qc > 0.0f) ? 0 : Qc >= 1.0f ? 1 : 2;
          if (cls == 2) {
            tau = __builtin_sqrtf(Qc * __builtin_amdgcn_rcpf(1.0f - Qc));
            float gg = 0.0f;
#pragma unroll
            for (int i = 0; i < 9; ++i) gg = fmaf(G[i], G[i], gg);
            lip = (1.0f + tau) * __builtin_sqrtf(gg);
          }
        }
        if (cls == 0) {
          tile[k] = kDropKey;
          continue;
        }
        if (cls == 1 || !(cr[k].w >= 0.0f)) continue;  // kept, as by the exact test
        const float gx = fmaf(G[2], cr[k].z, fmaf(G[1], cr[k].y, G[0] * cr[k].x));
        const float gy = fmaf(G[5], cr[k].z, fmaf(G[4], cr[k].y, G[3] * cr[k].x));
        const float gz = fmaf(G[8], cr[k].z, fmaf(G[7], cr[k].y, G[6] * cr[k].x));
        const float hc = __builtin_sqrtf(fmaf(gx, gx, gy * gy)) - tau * gz;
        if (hc > lip * (cr[k].w + 0x1p-16f)) tile[k] = kDropKey;
        else survive |= 1u << k;
      }
      // (2) The exact quad test of the entries (1) left open, compacted over
      // the wave so that every lane tests one: the wave's open entries are
      // queued in its staging slots, tested 64 at a time, and each verdict is
      // read back by the entry's lane.
      const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
      const uint32_t mine = (uint32_t)__popc(survive);
      const uint32_t incl = wave_incl_scan(mine);
      const uint32_t nq = __shfl(incl, 63);
      uint32_t* const qt = s_tile + wv * kWaveSlots;
      uint32_t* const qi = s_item + wv * kWaveSlots;
      uint8_t* const qk = s_keep + wv * (kExpandSpan / 4);
      uint32_t pos = incl - mine;
#pragma unroll
      for (int k = 0; k < kExpandPer; ++k) {
        if (!((survive >> k) & 1u)) continue;
        qt[pos] = tile[k];
        qi[pos] = item[k];
        ++pos;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      for (uint32_t r = 0; r < nq; r += 64) {  // nq is uniform over the wave
        const uint32_t q = r + (uint32_t)lane;
        if (q < nq) {
          const float4* cp = tcones + kConeStride * (size_t)qt[q];
          const float4* rq = reinterpret_cast<const float4*>(recs + qi[q]);
          const float4 c0 = cp[0], c1 = cp[1], c2 = cp[2], c3 = cp[3];
          const float4 p0 = rq[0], p1 = rq[1], p2 = rq[2];
          const float4 p3 = make_float4(0.0f, 0.0f, 0.0f, recs[qi[q]].qmax);
          QuadCone Q;
          Q.d[0][0] = c0.x; Q.d[0][1] = c0.y; Q.d[0][2] = c0.z;
          Q.d[1][0] = c1.x; Q.d[1][1] = c1.y; Q.d[1][2] = c1.z;
          Q.d[2][0] = c2.x; Q.d[2][1] = c2.y; Q.d[2][2] = c2.z;
          Q.d[3][0] = c3.x; Q.d[3][1] = c3.y; Q.d[3][2] = c3.z;
          Q.valid = c0.w != 0.0f;
          qk[q] = cone_meets_quad(p0, p1, p2, p3, Q, op.log2_amin, fixed) ? 1 : 0;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      pos = incl - mine;
#pragma unroll
      for (int k = 0; k < kExpandPer; ++k) {
        if (!((survive >> k) & 1u)) continue;
        if (!qk[pos]) tile[k] = kDropKey;
        ++pos;
      }
    }
#pragma unroll
    for (int k = 0; k < kExpandPer; ++k) {
      if (k >= cnt) break;
      const uint32_t t = tile[k];
      if (hpass && t != kDropKey) {
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
  if (hpass && run_n) atomicAdd(&s_h[1][run_d], run_n);
  __syncthreads();
  if (hpass) {
    uint32_t* hp = hparts + (blockIdx.x % kHistCopies) * kHistStride;
    for (int p = 0; p < hpass; ++p) {
      const uint32_t c = s_h[p][threadIdx.x];
      if (c) atomicAdd(&hp[p * 256 + threadIdx.x], c);
    }
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
                                                        uint32_t* __restrict__ list,
                                                        const unsigned long long* __restrict__ err) {
  // A sort that stalled leaves a list in no order: every tile's range is then
  // empty, so that nothing downstream reads the list (the outputs are
  // reported invalid anyway).  The sort's kernels have all ended, so every
  // block reads the same word.
  const bool bad = err && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0ull;
  const int64_t total = bad ? 0 : dyn_count(total_cap, dyn);
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  const int64_t e0 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (list && e0 < 8) list[total + e0] = 0u;
  if (total == 0) {
    for (int64_t t = e0; t <= ntiles; t += stride) ranges[t] = 0u;
    return;
  }
  // grid-stride: the grid is bounded, however large the capacity
  // tile ids are clamped into the grid, so that even a list a stalled sort
  // left inconsistent cannot send these writes out of bounds
  for (int64_t e = e0; e < total; e += stride) {
    const int64_t cur = min((int64_t)tiles[e], ntiles - 1);
    const int64_t prev = e > 0 ? min((int64_t)tiles[e - 1], ntiles - 1) : -1;
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

// Depth order of the visible items: an upsweep (digit counts of the four
// passes and the count-weighted counts of the last) and four passes.  Pass 0
// compacts the items with counts[i] != 0 out of all n0 items; passes 1 to 3
// read the live visible count (dyn1, or n1_cap).  Work layout (u32 words):
// the head, status table 0 (passes 0 and 2), status table 1 (pass 1, then the
// 64-bit rows of pass 3).
static int64_t depth_blocks(int64_t n0) { return os_blocks(n0, kBlock * os_per(n0)); }

int64_t depth_work_words(int64_t n0) { return kWorkHead + 3 * 256 * depth_blocks(std::max<int64_t>(n0, 1)); }

int64_t depth_zero_words(int64_t n0) { return kWorkHead + 256 * depth_blocks(std::max<int64_t>(n0, 1)); }

void depth_order(hipStream_t st, const uint32_t* keys, const uint32_t* counts, int64_t n0, int64_t n1_cap,
                 const unsigned long long* dyn1, uint32_t* work, bool zeroed, uint32_t* ka, uint32_t* va,
                 uint32_t* kb, uint32_t* vb, uint32_t* offs, uint32_t* owners, int64_t owners_n,
                 unsigned long long* err, bool tickets, uint32_t spin_limit) {
  if (n0 <= 0 || n1_cap <= 0) return;
  const int per = os_per(n0);
  const int items = kBlock * per;
  const int64_t nb0 = os_blocks(n0, items), nb1 = std::max<int64_t>(os_blocks(n1_cap, items), 1);
  uint32_t* ghist = work;
  uint32_t* whist = work + 4 * 256;
  uint32_t* tk = work + 5 * 256;  // the passes' tickets (in the head, so they start at zero)
  uint32_t* t0 = work + kWorkHead;
  uint32_t* t1 = t0 + 256 * nb0;
  if (!zeroed)
    hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(depth_zero_words(n0), kBlock)), dim3(kBlock), 0, st, work,
                       depth_zero_words(n0), 0u);
  const unsigned ug = (unsigned)std::min<int64_t>(std::max<int64_t>(grid_for(n0, kBlock), 1), 256);
  hipLaunchKernelGGL(radix_upsweep_kernel, dim3(ug), dim3(kBlock), 0, st, keys, counts, 0, n0,
                     (const unsigned long long*)nullptr, 0, 8, 4, ghist, whist);
  auto plain = per == kOSPerBig ? radix_pass_kernel<kOSPerBig, false>
               : per == kOSPer  ? radix_pass_kernel<kOSPer, false>
                                : radix_pass_kernel<kOSPerSmall, false>;
  auto weighted = per == kOSPerBig ? radix_pass_kernel<kOSPerBig, true>
                  : per == kOSPer  ? radix_pass_kernel<kOSPer, true>
                                   : radix_pass_kernel<kOSPerSmall, true>;
  PassArgs p{};
  p.spin_limit = spin_limit;
  p.hcopies = 1;
  p.dmask = 255u;
  p.next_row_words = 256;
  p.err = err;
  // pass 0: all items, the visible ones out (value = item index)
  p.keys_in = keys;
  p.filter = counts;
  p.n_cap = n0;
  p.ghist = ghist;
  p.status = t0;
  p.status_next = t1;
  p.keys_out = ka;
  p.vals_out = va;
  p.ticket = tickets ? tk : nullptr;
  hipLaunchKernelGGL(plain, dim3((unsigned)nb0), dim3(kBlock), 0, st, p);
  // passes 1 and 2 over the visible items: (ka, va) -> (kb, vb) -> (ka, va)
  p.filter = nullptr;
  p.n_cap = n1_cap;
  p.dyn = dyn1;
  for (int q = 1; q <= 2; ++q) {
    p.keys_in = q == 1 ? ka : kb;
    p.vals_in = q == 1 ? va : vb;
    p.shift = 8 * q;
    p.ghist = ghist + 256 * q;
    p.status = q == 1 ? t1 : t0;
    p.status_next = q == 1 ? t0 : t1;
    p.next_row_words = q == 1 ? 256 : 512;  // pass 3's rows are 64-bit
    p.keys_out = q == 1 ? kb : ka;
    p.vals_out = q == 1 ? vb : va;
    p.ticket = tickets ? tk + q : nullptr;
    hipLaunchKernelGGL(plain, dim3((unsigned)nb1), dim3(kBlock), 0, st, p);
  }
  // pass 3, weighted by the tile counts: items in depth order to vb, their
  // entry offsets to offs
  p.keys_in = ka;
  p.vals_in = va;
  p.shift = 24;
  p.ghist = ghist + 3 * 256;
  p.whist = whist;
  p.wts = counts;
  p.wts_n = n0;
  p.status = t1;
  p.status_next = nullptr;
  p.keys_out = nullptr;
  p.vals_out = vb;
  p.wout = offs;
  p.owners = owners;
  p.owners_n = owners_n;
  p.ticket = tickets ? tk + 3 : nullptr;
  hipLaunchKernelGGL(weighted, dim3((unsigned)nb1), dim3(kBlock), 0, st, p);
}

// Work of the expansion and the tile sort, u32 words: the expansion's partial
// histograms, the sort's head (digit counts when an upsweep counts them) and
// two status tables.  The first three parts must start at zero.
static int64_t tile_rows(int64_t ecap) {
  ecap = std::max<int64_t>(ecap, 1);
  return 256 * os_blocks(ecap, kBlock * os_per(ecap));
}

int64_t tile_zero_words(int64_t ecap) { return hist_parts_words() + kWorkHead + tile_rows(ecap); }

int64_t tile_work_words(int64_t ecap) { return tile_zero_words(ecap) + tile_rows(ecap); }

void tile_sort(hipStream_t st, const uint32_t* tin, const uint32_t* iin, int64_t ecap,
               const unsigned long long* dE, unsigned long long* kept, int passes, int bits, uint32_t* at,
               uint32_t* ai, uint32_t* bt, uint32_t* bi, uint32_t* twork, int hpass, unsigned long long* err,
               bool tickets, uint32_t spin_limit) {
  if (ecap <= 0 || passes <= 0) return;
  const int per = os_per(ecap);
  const unsigned nb = (unsigned)std::max<int64_t>(os_blocks(ecap, kBlock * per), 1);
  uint32_t* hparts = twork;
  uint32_t* head = hparts + hist_parts_words();
  uint32_t* t0 = head + kWorkHead;
  uint32_t* t1 = t0 + tile_rows(ecap);
  if (!hpass) {
    const unsigned ug = (unsigned)std::min<int64_t>(std::max<int64_t>(grid_for(ecap, kBlock), 1), 256);
    hipLaunchKernelGGL(radix_upsweep_kernel, dim3(ug), dim3(kBlock), 0, st, tin, (const uint32_t*)nullptr, 1, ecap,
                       dE, 0, bits, passes, head, (uint32_t*)nullptr);
  }
  auto kern = per == kOSPerBig ? radix_pass_kernel<kOSPerBig, false>
              : per == kOSPer  ? radix_pass_kernel<kOSPer, false>
                               : radix_pass_kernel<kOSPerSmall, false>;
  PassArgs p{};
  p.spin_limit = spin_limit;
  p.n_cap = ecap;
  p.dmask = (1u << bits) - 1u;
  p.hstride = kHistStride;
  p.hcopies = hpass ? kHistCopies : 1;
  p.next_row_words = 256;
  p.err = err;
  const uint32_t *sk = tin, *sv = iin;
  for (int q = 0; q < passes; ++q) {
    uint32_t* ok = (q % 2 == 0) ? at : bt;
    uint32_t* ov = (q % 2 == 0) ? ai : bi;
    // pass 0 reads the whole list and leaves the culled entries out, counting
    // the kept ones into *kept; later passes read those
    p.dyn = q == 0 ? dE : kept;
    p.drop = q == 0 ? 1 : 0;
    p.kept_out = q == 0 ? kept : nullptr;
    p.keys_in = sk;
    p.vals_in = sv;
    p.shift = bits * q;
    p.ghist = (hpass ? hparts : head) + 256 * q;
    p.status = (q % 2 == 0) ? t0 : t1;
    p.status_next = q + 1 < passes ? ((q % 2 == 0) ? t1 : t0) : nullptr;
    p.keys_out = ok;
    p.vals_out = ov;
    p.ticket = tickets ? head + 5 * 256 + q : nullptr;  // in the head, cleared with it
    hipLaunchKernelGGL(kern, dim3(nb), dim3(kBlock), 0, st, p);
    sk = ok;
    sv = ov;
  }
}

size_t tile_cone_bytes(int64_t ntiles) { return sizeof(float4) * kConeStride * (size_t)std::max<int64_t>(ntiles, 1); }

void launch_tile_cones(hipStream_t st, const ViewDev* views, int nviews, const float2* dtab, int64_t ntiles,
                       float4* out, uint32_t* zero, int64_t nzero) {
  if (ntiles <= 0 && nzero <= 0) return;
  hipLaunchKernelGGL(tile_cones_kernel, dim3(grid_for(std::max(ntiles, nzero), kBlock)), dim3(kBlock), 0, st, views,
                     nviews, dtab, ntiles, out, zero, nzero);
}

void launch_expand(hipStream_t st, const uint32_t* items, const uint32_t* offs, int64_t m_cap,
                   const unsigned long long* dyn_m, int64_t total_cap, const unsigned long long* dyn_total,
                   const uint2* rects, const ViewDev* views, int64_t n, const float4* tcones, const Record* recs,
                   const Opts& op, uint32_t* tiles_out, uint32_t* items_out, uint32_t* twork, int hpass,
                   int hbits, int64_t nitems, int64_t ntiles, const uint32_t* owners) {
  if (total_cap <= 0) return;
  hipLaunchKernelGGL(expand_kernel, dim3(grid_for(total_cap, kExpandSpan)), dim3(kBlock), 0, st, items, offs, m_cap,
                     dyn_m, total_cap, dyn_total, rects, views, n, tcones, recs, op, op.cone_cull, tiles_out,
                     items_out, twork, hpass, hbits, std::max<int64_t>(nitems, 1), (uint32_t)ntiles, owners);
}

void launch_ranges(hipStream_t st, const uint32_t* tiles, int64_t total_cap, const unsigned long long* dyn,
                   int64_t ntiles, uint32_t* ranges, uint32_t* list, const unsigned long long* err) {
  if (total_cap <= 0 && !dyn) {
    hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(ntiles + 1, kBlock)), dim3(kBlock), 0, st, ranges, ntiles + 1,
                       0u);
    return;
  }
  const int64_t g = std::max<int64_t>(total_cap, ntiles + 1);
  hipLaunchKernelGGL(ranges_kernel, dim3(std::min<unsigned>(grid_for(g, kBlock), 8192u)), dim3(kBlock), 0, st, tiles,
                     total_cap, dyn, ntiles, ranges, list, err);
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
