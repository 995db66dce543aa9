// Stage (c): per-ray front-to-back compositing (Alg. 1 render loop, Eq. color)
// with the closed-form ray opacity alpha = sigma exp(-kappa/2).
//
// Mapping: one 256-lane workgroup per 16x16 tile (camera sub-frustum), one
// wave64 per 8x8 half-tile, one lane per ray.  The workgroup walks its tile's
// depth-ordered list in batches of 256 entries: each lane fetches one entry's
// 64-byte record (vector loads, the next batch prefetched into registers
// while the current one blends) and stages it in LDS; wave ballots publish,
// per half-tile, which staged entries its rectangle meets.  Each wave then
// visits only its own hits, reading records from LDS as broadcasts, and skips
// the batch entirely once all of its rays have terminated; the tile stops
// when all four waves have.
//
// Per pair, kappa = |o_u x d_u|^2 / |d_u|^2 is evaluated in a canonical frame
// rotated so that o_u lies on its third axis (the canonical Gaussian is
// isotropic, so kappa is unchanged): with g = G d (G = r diag(1,1,-1) Q Wc),
// kappa = r^2 (gx^2 + gy^2) / |g|^2 and t* = r^2 gz / |g|^2.  This is the
// cross-product form with the rotation folded into the record; it keeps the
// first-order (not the squared) cancellation of the cross product.
#include <hip/hip_runtime.h>

#include "geer_common.h"
#include "geer_device.h"

namespace geer {

// One (ray, Gaussian) evaluation and blend, branch-free: lanes that already
// terminated compute too -- their SIMD lane is occupied either way -- but
// their blend weight is zero.  `done` is the wave's mask of terminated rays
// (wave-uniform, kept in scalar registers); a lane reads its own bit with an
// inverse ballot, so the bookkeeping costs no vector instructions.  The blend
// weight is the drop in transmittance, w = T - T(1 - alpha) (zero when the
// pair does not blend).  With kKeep the index one past the last blended
// entry is tracked for the backward replay.
template <bool kFixed, bool kKeep>
__device__ __forceinline__ void blend_one(const Record& R, float dx, float dy, float dz, const Opts& op, uint32_t e,
                                          uint64_t& done, float& T, float& cr, float& cg, float& cb, float& D,
                                          uint32_t& last) {
  const PairEval E = eval_pair(R, dx, dy, dz);
  // the contribution rule and the termination test as wave masks: each ballot
  // of a plain comparison is that comparison's lane mask
  uint64_t ok = ~done & __builtin_amdgcn_ballot_w64(E.gz > 0.0f) &
                __builtin_amdgcn_ballot_w64(E.a_raw >= op.alpha_min);
  if (kFixed) ok &= __builtin_amdgcn_ballot_w64(E.q <= R.qmax);
  const float a = fminf(E.a_raw, op.alpha_max);
  const float Tn = fmaf(-a, T, T);
  const uint64_t term = ok & __builtin_amdgcn_ballot_w64(Tn < op.t_min);
  const bool blend = __builtin_amdgcn_inverse_ballot_w64(ok & ~term);
  done |= term;
  const float Tnew = blend ? Tn : T;
  const float w = T - Tnew;
  T = Tnew;
  cr = fmaf(w, R.rgb[0], cr);
  cg = fmaf(w, R.rgb[1], cg);
  cb = fmaf(w, R.rgb[2], cb);
  D = fmaf(w * R.c1, E.gz * E.inv, D);
  if (kKeep) last = blend ? e + 1 : last;
}

constexpr int kBatch = 256;  // list entries staged per workgroup pass (one per lane)

template <bool kFixed, bool kKeep>
__global__ __launch_bounds__(256) void render_kernel(
    const ViewDev* __restrict__ views, int nviews, const float2* __restrict__ dtab,
    const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ list, const uint2* __restrict__ rects,
    const Record* __restrict__ recs, Opts op, float* __restrict__ rgb, float* __restrict__ depth,
    float* __restrict__ trans, uint32_t* __restrict__ nlast, float* __restrict__ tfinal,
    unsigned long long* __restrict__ stats) {
  __shared__ float4 s_rec[kBatch][4];     // 16 KB of records, one batch
  __shared__ uint64_t s_hit[4][kBatch / 64];  // per half-tile: which staged entries meet it

  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  int v = 0;
  while (v + 1 < nviews && tile >= views[v + 1].tile_base) ++v;
  const ViewDev& V = views[v];
  const int lt = tile - V.tile_base;
  const int tx = lt % V.tiles_x, ty = lt / V.tiles_x;
  const int tid = threadIdx.x;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;
  const int hx = 2 * tx + (wv & 1), hy = 2 * ty + (wv >> 1);
  const bool wave_live = hx < V.nhx && hy < V.nhy;  // half-tile inside a ragged image
  const int px = hx * kHalf + (lane & 7), py = hy * kHalf + (lane >> 3);
  const bool valid = wave_live && px < V.width && py < V.height;

  float dx, dy, dz;
  pixel_direction(V, dtab, px, py, dx, dy, dz);

  const uint32_t start = ranges[tile], end = ranges[tile + 1];
  float T = 1.0f, cr = 0.0f, cg = 0.0f, cb = 0.0f, D = 0.0f;
  uint32_t last = start;
  uint64_t evals = 0;
  uint64_t done = __ballot(!valid);  // wave mask of terminated (or absent) rays
  // the four half-tiles of this tile, for the per-entry hit bits
  const uint32_t hx0 = 2u * tx, hy0 = 2u * ty;

  // Prefetch of one batch into registers: entry start + k goes to lane k.
  float4 p0, p1, p2, p3;
  uint2 prc;
  auto fetch = [&](uint32_t b) {
    const uint32_t e = b + tid;
    if (e < end) {
      const uint32_t item = list[e];
      prc = rects[item];
      const float4* r = reinterpret_cast<const float4*>(recs + item);
      p0 = r[0]; p1 = r[1]; p2 = r[2]; p3 = r[3];
    } else {
      prc = make_uint2(1u, 0u);  // empty rectangle: meets no half-tile
    }
  };
  if (start < end) fetch(start);

  for (uint32_t base = start; base < end; base += kBatch) {
    // stage the prefetched batch (the barrier closing the previous pass made
    // the LDS free) and publish each half-tile's hit mask
    s_rec[tid][0] = p0; s_rec[tid][1] = p1; s_rec[tid][2] = p2; s_rec[tid][3] = p3;
    const uint32_t rx0 = prc.x & 0xffffu, rx1 = prc.x >> 16, ry0 = prc.y & 0xffffu, ry1 = prc.y >> 16;
    const bool cx0 = rx0 <= hx0 && hx0 <= rx1, cx1 = rx0 <= hx0 + 1 && hx0 + 1 <= rx1;
    const bool cy0 = ry0 <= hy0 && hy0 <= ry1, cy1 = ry0 <= hy0 + 1 && hy0 + 1 <= ry1;
    const uint64_t b00 = __ballot(cx0 && cy0), b10 = __ballot(cx1 && cy0);
    const uint64_t b01 = __ballot(cx0 && cy1), b11 = __ballot(cx1 && cy1);
    if (lane == 0) {
      s_hit[0][wv] = b00; s_hit[1][wv] = b10; s_hit[2][wv] = b01; s_hit[3][wv] = b11;
    }
    if (base + kBatch < end) fetch(base + kBatch);  // in flight while this batch blends
    __syncthreads();
    if (~done != 0) {
      const uint32_t nb = min((uint32_t)kBatch, end - base);
#pragma unroll
      for (int g = 0; g < kBatch / 64; ++g) {
        if ((uint32_t)(g * 64) >= nb) break;
        const uint64_t mv = s_hit[wv][g];  // same value in every lane: move it to SGPRs
        // (readfirstlane returns int: go through uint32_t so nothing sign-extends)
        uint64_t m = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(mv >> 32)) << 32) |
                     (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)mv);
        while (m) {
          const int k = g * 64 + __builtin_ctzll(m);
          m &= m - 1;
          Record R;
          float4* rr = reinterpret_cast<float4*>(&R);
          rr[0] = s_rec[k][0]; rr[1] = s_rec[k][1]; rr[2] = s_rec[k][2]; rr[3] = s_rec[k][3];
          evals += (uint64_t)__popcll(~done);
          blend_one<kFixed, kKeep>(R, dx, dy, dz, op, base + k, done, T, cr, cg, cb, D, last);
        }
      }
    }
    // every wave done -> the whole tile is done; the barrier also frees the LDS
    if (__syncthreads_and(~done == 0 ? 1 : 0)) break;
  }

  if (valid) {
    const int64_t hw = (int64_t)V.width * V.height;
    const int64_t p = (int64_t)py * V.width + px;
    float* out = rgb + 3 * (int64_t)V.pix_base;
    out[p] = cr;
    out[hw + p] = cg;
    out[2 * hw + p] = cb;
    const int64_t gp = (int64_t)V.pix_base + p;
    if (depth) depth[gp] = D;
    if (trans) trans[gp] = T;
    if (kKeep) {
      nlast[gp] = last;
      tfinal[gp] = T;
    }
  }
  if (stats && lane == 0 && evals) atomicAdd(&stats[0], (unsigned long long)evals);
}

void launch_render(hipStream_t st, bool fixed_lambda, int64_t ntiles, const ViewDev* views, int nviews,
                   const float2* dtab, const uint32_t* ranges, const uint32_t* list, const uint2* rects,
                   const Record* recs, const Opts& op, float* rgb, float* depth, float* trans, uint32_t* nlast,
                   float* tfinal, unsigned long long* stats) {
  if (ntiles <= 0) return;
  const bool keep = nlast != nullptr && tfinal != nullptr;
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3((unsigned)ntiles), dim3(256), 0, st, views, nviews, dtab, ranges, list, rects, recs,
                       op, rgb, depth, trans, nlast, tfinal, stats);
  };
  if (fixed_lambda) {
    if (keep) go(render_kernel<true, true>);
    else go(render_kernel<true, false>);
  } else {
    if (keep) go(render_kernel<false, true>);
    else go(render_kernel<false, false>);
  }
}

}  // namespace geer
