// Stage (c): per-ray front-to-back compositing (Alg. 1 render loop, Eq. color)
// with the closed-form ray opacity alpha = sigma exp(-kappa/2).
//
// Mapping: one 256-lane workgroup per 16x16 tile (camera sub-frustum), one
// wave64 per 8x8 half-tile, one lane per ray.  Each wave walks its tile's
// depth-ordered list on its own: the list index, the Gaussian's rectangle and
// its 64-byte record are wave-uniform (scalar loads into SGPRs, used directly
// as VALU operands), entries whose rectangle misses the wave's half-tile are
// skipped with a scalar branch, and the wave leaves the loop as soon as all of
// its rays have terminated.  No LDS, no barriers.
//
// Per pair, kappa = |o_u x d_u|^2 / |d_u|^2 is evaluated in a canonical frame
// rotated so that o_u lies on its third axis (the canonical Gaussian is
// isotropic, so kappa is unchanged): with g = G d (G = r diag(1,1,-1) Q Wc),
// kappa = r^2 (gx^2 + gy^2) / |g|^2 and t* = r^2 gz / |g|^2.  This is the
// cross-product form with the rotation folded into the record; it keeps the
// first-order (not the squared) cancellation of the cross product.
#include <hip/hip_runtime.h>

#include "geer_common.h"

namespace geer {

__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
  // Workgroups are dealt round-robin to the 8 XCDs; give each XCD a
  // contiguous band of tiles so neighbouring tiles share its L2.
  int q = nblocks >> 3, r = nblocks & 7, x = bid & 7;
  return x * q + min(x, r) + (bid >> 3);
}

// One (ray, Gaussian) evaluation and blend, branch-free: lanes that already
// terminated (or a disabled second slot) compute too -- their SIMD lane is
// occupied either way -- but their blend weight is zero.
template <bool kFixed>
__device__ __forceinline__ void blend_one(const Record& R, bool enable, float dx, float dy, float dz,
                                          const Opts& op, uint32_t e, bool& done, float& T, float& cr,
                                          float& cg, float& cb, float& D, uint32_t& last) {
  const float gx = fmaf(R.g[2], dz, fmaf(R.g[1], dy, R.g[0] * dx));
  const float gy = fmaf(R.g[5], dz, fmaf(R.g[4], dy, R.g[3] * dx));
  const float gz = fmaf(R.g[8], dz, fmaf(R.g[7], dy, R.g[6] * dx));
  const float mm = fmaf(gy, gy, gx * gx);
  const float ss = fmaf(gz, gz, mm);
  const float inv = __builtin_amdgcn_rcpf(ss);
  const float q = mm * inv;
  float a = __builtin_amdgcn_exp2f(fmaf(R.c0, q, R.lsig));
  bool ok = enable & !done & (gz > 0.0f) & (a >= op.alpha_min);
  if (kFixed) ok = ok & (q <= R.qmax);
  a = a < op.alpha_max ? a : op.alpha_max;
  const float Tn = T * (1.0f - a);
  const bool term = ok & (Tn < op.t_min);
  const bool blend = ok & !term;
  done = done | term;
  const float w = blend ? a * T : 0.0f;
  cr = fmaf(w, R.rgb[0], cr);
  cg = fmaf(w, R.rgb[1], cg);
  cb = fmaf(w, R.rgb[2], cb);
  D = fmaf(w * R.c1, gz * inv, D);
  T = blend ? Tn : T;
  last = blend ? e + 1 : last;
}

template <bool kFixed>
__global__ __launch_bounds__(256) void render_kernel(
    const ViewDev* __restrict__ views, int nviews, const float2* __restrict__ dtab,
    const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ list, const uint2* __restrict__ rects,
    const Record* __restrict__ recs, Opts op, float* __restrict__ rgb, float* __restrict__ depth,
    float* __restrict__ trans, uint32_t* __restrict__ nlast, float* __restrict__ tfinal,
    unsigned long long* __restrict__ stats) {
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  int v = 0;
  while (v + 1 < nviews && tile >= views[v + 1].tile_base) ++v;
  const ViewDev& V = views[v];
  const int lt = tile - V.tile_base;
  const int tx = lt % V.tiles_x, ty = lt / V.tiles_x;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int hx = 2 * tx + (wv & 1), hy = 2 * ty + (wv >> 1);
  if (hx >= V.nhx || hy >= V.nhy) return;  // half-tile outside a ragged image
  const int px = hx * kHalf + (lane & 7), py = hy * kHalf + (lane >> 3);
  const bool valid = px < V.width && py < V.height;

  const float2 cth = dtab[V.dx_off + min(px, V.width - 1)];  // (sin, cos) theta
  const float2 cph = dtab[V.dy_off + min(py, V.height - 1)]; // (sin, cos) phi
  float dx = cth.x * cph.y, dy = cth.y * cph.x, dz = cth.y * cph.y;
  const float dn = rsqrtf(dx * dx + dy * dy + dz * dz);
  dx *= dn; dy *= dn; dz *= dn;

  const uint32_t start = ranges[tile], end = ranges[tile + 1];
  float T = 1.0f, cr = 0.0f, cg = 0.0f, cb = 0.0f, D = 0.0f;
  uint32_t last = start;
  uint64_t evals = 0;
  bool done = !valid;
  const uint32_t hxu = (uint32_t)hx, hyu = (uint32_t)hy;

  // Batches of 8 list entries from an 8-aligned base (the list is padded with
  // a valid id): 8 ids -> 8 rectangles (all loads in flight together) -> mask
  // of entries meeting this half-tile -> their records two at a time, both
  // scalar loads issued before the single wait.
  for (uint32_t base = start & ~7u; base < end; base += 8) {
    const uint4 i0 = *reinterpret_cast<const uint4*>(list + base);
    const uint4 i1 = *reinterpret_cast<const uint4*>(list + base + 4);
    const uint32_t ids[8] = {i0.x, i0.y, i0.z, i0.w, i1.x, i1.y, i1.z, i1.w};
    uint2 rc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) rc[k] = rects[ids[k]];
    uint32_t mask = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const bool hit = (hxu >= (rc[k].x & 0xffffu)) & (hxu <= (rc[k].x >> 16)) & (hyu >= (rc[k].y & 0xffffu)) &
                       (hyu <= (rc[k].y >> 16));
      mask |= (uint32_t)hit << k;
    }
    const uint32_t lo = start > base ? start - base : 0u;
    const uint32_t hi = end - base < 8u ? end - base : 8u;
    mask &= (0xffu << lo) & (0xffu >> (8u - hi));
    while (mask) {
      const int k0 = __builtin_ctz(mask);
      mask &= mask - 1;
      const bool two = mask != 0;
      const int k1 = two ? __builtin_ctz(mask) : k0;
      mask &= two ? mask - 1 : mask;
      const Record R0 = recs[ids[k0]];
      const Record R1 = recs[ids[k1]];
      evals += (uint64_t)__popcll(__ballot(!done));
      blend_one<kFixed>(R0, true, dx, dy, dz, op, base + k0, done, T, cr, cg, cb, D, last);
      if (two) evals += (uint64_t)__popcll(__ballot(!done));
      blend_one<kFixed>(R1, two, dx, dy, dz, op, base + k1, done, T, cr, cg, cb, D, last);
    }
    if (__ballot(!done) == 0) break;
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
    if (nlast) nlast[gp] = last;
    if (tfinal) tfinal[gp] = T;
  }
  if (stats && lane == 0) atomicAdd(&stats[0], (unsigned long long)evals);
}

void launch_render(hipStream_t st, bool fixed_lambda, int64_t ntiles, const ViewDev* views, int nviews,
                   const float2* dtab, const uint32_t* ranges, const uint32_t* list, const uint2* rects,
                   const Record* recs, const Opts& op, float* rgb, float* depth, float* trans, uint32_t* nlast,
                   float* tfinal, unsigned long long* stats) {
  if (ntiles <= 0) return;
  if (fixed_lambda)
    hipLaunchKernelGGL(render_kernel<true>, dim3((unsigned)ntiles), dim3(256), 0, st, views, nviews, dtab, ranges,
                       list, rects, recs, op, rgb, depth, trans, nlast, tfinal, stats);
  else
    hipLaunchKernelGGL(render_kernel<false>, dim3((unsigned)ntiles), dim3(256), 0, st, views, nviews, dtab, ranges,
                       list, rects, recs, op, rgb, depth, trans, nlast, tfinal, stats);
}

}  // namespace geer
