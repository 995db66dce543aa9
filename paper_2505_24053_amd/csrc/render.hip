// Stage (c): per-ray front-to-back compositing (Alg. 1 render loop, Eq. color)
// with the closed-form ray opacity alpha = sigma exp(-kappa/2).
//
// Mapping: one wave64 per 8x8 half-tile (a quarter of a 16x16 camera
// sub-frustum), one lane per ray, each wave its own 64-lane workgroup so that
// nothing ties it to the other quarters of its tile.  The wave walks its
// tile's depth-ordered list in windows of 64 entries: lane k reads entry
// base + k's list slot and half-tile rectangle, and, when the rectangle meets
// this half-tile, its 64-byte record (the next window is prefetched into
// registers while the current one blends).  Lane k then tests whether the
// Gaussian's contribution cone reaches any ray of the half-tile at all (most
// rectangle hits of thin or small Gaussians do not); a ballot of the two
// tests gives the window's hits, staged in the wave's own 4 KB of LDS and
// visited in order, each record read as an LDS broadcast.  Skipped entries
// are exactly ones that would blend nothing, so the image is unchanged.  The
// wave stops as soon as all of its rays have terminated.
//
// Per pair, kappa = |o_u x d_u|^2 / |d_u|^2 is evaluated in a canonical frame
// rotated so that o_u lies on its third axis (the canonical Gaussian is
// isotropic, so kappa is unchanged): with g = G d (G = r diag(1,1,-1) Q Wc),
// kappa = r^2 (gx^2 + gy^2) / |g|^2 and t* = r^2 gz / |g|^2.  This is the
// cross-product form with the rotation folded into the record; it keeps the
// first-order (not the squared) cancellation of the cross product.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "geer_common.h"
#include "geer_device.h"

#ifndef RENDER_WAVES
#define RENDER_WAVES 2
#endif

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
__device__ __forceinline__ void blend_one(const Record& R, float dx, float dy, float dz, const Opts& op, int amax_bits,
                                          uint32_t e, uint64_t& done, float& T, float& cr, float& cg, float& cb,
                                          float& D, uint32_t& last) {
  const PairEval E = eval_pair(R, dx, dy, dz);
  // the contribution rule and the termination test as wave masks: each ballot
  // of a plain comparison is that comparison's lane mask
  uint64_t ok = ~done & __builtin_amdgcn_ballot_w64(E.gz > 0.0f) &
                __builtin_amdgcn_ballot_w64(E.a_raw >= op.alpha_min);
  if (kFixed) ok &= __builtin_amdgcn_ballot_w64(E.q <= R.qmax);
  // min(alpha_raw, alpha_max): both are >= +0, where the order of the bit
  // patterns is the order of the values (a NaN pattern also maps to alpha_max)
  const float a = __int_as_float(min(__float_as_int(E.a_raw), amax_bits));
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

constexpr int kWin = 64;  // list entries staged per wave pass (one per lane)

// DPP lane moves within each quad of 4 lanes.
template <int kCtrl>
__device__ __forceinline__ float qdpp(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), kCtrl, 0xF, 0xF, true));
}
template <int kCtrl>
__device__ __forceinline__ uint32_t qdpp_u(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kCtrl, 0xF, 0xF, true);
}
constexpr int kQuadPrev1 = 0x90;  // quad_perm [0, 0, 1, 2]: lane j reads lane j - 1
constexpr int kQuadPrev2 = 0x44;  // quad_perm [0, 1, 0, 1]: lane j reads lane j - 2
constexpr int kQuadXor1 = 0xB1;   // quad_perm [1, 0, 3, 2]
constexpr int kQuadXor2 = 0x4E;   // quad_perm [2, 3, 0, 1]

// Render of a heavy tile's 4x4 block of rays with all 64 lanes: lane
// 4 r + j holds ray r and, in each step, the j-th of the next four hits of
// the window, so a step composites four entries per ray.  The sequential
// front-to-back rule is kept exactly: the transmittance in front of hit j is
// T times the quad's exclusive prefix product of (1 - alpha) over the
// earlier contributing hits; the first hit whose blend would take it below
// T_min terminates the ray and excludes itself and the later hits.  Colour,
// depth and the last blended index are accumulated per lane and summed (or
// maximised) over the quad at the end; T advances by the quad's product.
template <bool kFixed, bool kKeep>
__device__ __forceinline__ void render_heavy_block(const WaveBlock& W, const ViewDev& V,
                                                   const float2* __restrict__ dtab, uint32_t start, uint32_t end,
                                                   const uint32_t* __restrict__ list, const uint2* __restrict__ rects,
                                                   const Record* __restrict__ recs, const Opts& op,
                                                   float4 (*s_rec)[4], float* __restrict__ rgb,
                                                   float* __restrict__ depth, float* __restrict__ trans,
                                                   uint32_t* __restrict__ nlast, float* __restrict__ tfinal,
                                                   uint64_t& evals_out) {
  const int lane = threadIdx.x & 63;
  const int j = lane & 3, r = lane >> 2;
  const uint32_t hx = (uint32_t)W.bx0 >> 3, hy = (uint32_t)W.by0 >> 3;
  const int px = W.bx0 + (r & 3), py = W.by0 + (r >> 2);
  const bool valid = px < V.width && py < V.height;
  float dx, dy, dz;
  pixel_direction(V, dtab, px, py, dx, dy, dz);
  const QuadCone Q = block_cone(V, dtab, W.bx0, W.by0, 4);
  float T = 1.0f, cr = 0.0f, cg = 0.0f, cb = 0.0f, D = 0.0f;
  uint32_t last = start;
  uint64_t evals = 0;
  uint64_t done = __builtin_amdgcn_ballot_w64(!valid);  // lanes of terminated (or absent) rays
  const int amax_bits = __float_as_int(op.alpha_max);
  const uint32_t below = (1u << j) - 1u;  // the quad's earlier lanes
  const int qsh = lane & ~3;              // this quad's bit offset in a wave mask

  // windows of 64 entries: lane k tests entry base + k (rectangle, then
  // contribution cone) and stages its record.  The next window is loaded
  // into registers while this one composites; its loads are unconditional
  // (a lane past the end reads the tile's first entry) so that they stay
  // plain register values.
  if (start >= end) {
    // an empty list (a heavy tile never has one): background
    if (valid && j == 0) {
      const int64_t hw = (int64_t)V.width * V.height;
      const int64_t p = (int64_t)py * V.width + px;
      float* out = rgb + 3 * (int64_t)V.pix_base;
      out[p] = 0.0f;
      out[hw + p] = 0.0f;
      out[2 * hw + p] = 0.0f;
      const int64_t gp = (int64_t)V.pix_base + p;
      if (depth) depth[gp] = 0.0f;
      if (trans) trans[gp] = 1.0f;
      if (kKeep) {
        nlast[gp] = start;
        tfinal[gp] = 1.0f;
      }
    }
    return;
  }
  float4 p0, p1, p2, p3;
  bool phit;
  {
    const uint32_t e = start + lane;
    const uint32_t item = list[e < end ? e : start];
    const uint2 rc = rects[item];
    phit = e < end && (rc.x & 0xffffu) <= hx && hx <= (rc.x >> 16) && (rc.y & 0xffffu) <= hy && hy <= (rc.y >> 16);
    const float4* rp = reinterpret_cast<const float4*>(recs + item);
    p0 = rp[0]; p1 = rp[1]; p2 = rp[2]; p3 = rp[3];
  }
  for (uint32_t base = start; base < end && ~done != 0; base += kWin) {
    if (phit && op.cone_cull) phit = cone_meets_quad(p0, p1, p2, p3, Q, op.log2_amin, kFixed);
    uint64_t m = __builtin_amdgcn_ballot_w64(phit);
    if (phit) {
      s_rec[lane][0] = p0; s_rec[lane][1] = p1; s_rec[lane][2] = p2; s_rec[lane][3] = p3;
    }
    {
      const uint32_t e = base + kWin + lane;
      const uint32_t item = list[e < end ? e : start];
      const uint2 rc = rects[item];
      phit = e < end && (rc.x & 0xffffu) <= hx && hx <= (rc.x >> 16) && (rc.y & 0xffffu) <= hy &&
             hy <= (rc.y >> 16);
      const float4* rp = reinterpret_cast<const float4*>(recs + item);
      p0 = rp[0]; p1 = rp[1]; p2 = rp[2]; p3 = rp[3];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    while (m != 0 && ~done != 0) {
      // the next (up to) four hits, in list order
      int kh[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        kh[q] = m != 0 ? __builtin_ctzll(m) : 64;
        m &= m - 1;
      }
      const int k = j == 0 ? kh[0] : (j == 1 ? kh[1] : (j == 2 ? kh[2] : kh[3]));
      // a lane without a hit reads the group's first hit (always staged this
      // window) so that everything it computes is finite; it blends nothing
      const bool has = k < 64;
      const int ks = has ? k : kh[0];
      Record R;
      float4* rr = reinterpret_cast<float4*>(&R);
      rr[0] = s_rec[ks][0]; rr[1] = s_rec[ks][1]; rr[2] = s_rec[ks][2]; rr[3] = s_rec[ks][3];
      const PairEval E = eval_pair(R, dx, dy, dz);
      const bool live = has && !__builtin_amdgcn_inverse_ballot_w64(done);
      evals += (uint64_t)__popcll(__builtin_amdgcn_ballot_w64(live));
      bool ok = live && E.gz > 0.0f && E.a_raw >= op.alpha_min;
      if (kFixed) ok = ok && E.q <= R.qmax;
      const float a = __int_as_float(min(__float_as_int(E.a_raw), amax_bits));
      const float f = ok ? 1.0f - a : 1.0f;
      // inclusive, then exclusive prefix product of f over the quad
      float incl = f;
      {
        const float t1 = qdpp<kQuadPrev1>(incl);
        incl = j >= 1 ? incl * t1 : incl;
        const float t2 = qdpp<kQuadPrev2>(incl);
        incl = j >= 2 ? incl * t2 : incl;
      }
      const float pex = qdpp<kQuadPrev1>(incl);
      const float Tj = j >= 1 ? T * pex : T;
      const float Tn = fmaf(-a, Tj, Tj);
      const bool term = ok && Tn < op.t_min;
      const uint32_t nib = (uint32_t)(__builtin_amdgcn_ballot_w64(term) >> qsh) & 0xFu;
      const bool blend = ok && !term && (nib & below) == 0u;
      const float w = blend ? Tj - Tn : 0.0f;
      cr = fmaf(w, R.rgb[0], cr);
      cg = fmaf(w, R.rgb[1], cg);
      cb = fmaf(w, R.rgb[2], cb);
      D = fmaf(w * R.c1, E.gz * E.inv, D);
      if (kKeep) last = blend ? base + (uint32_t)k + 1u : last;
      // T advances by the product of (1 - alpha) over the blended hits
      float g = blend ? f : 1.0f;
      g *= qdpp<kQuadXor1>(g);
      g *= qdpp<kQuadXor2>(g);
      T *= g;
      done |= __builtin_amdgcn_ballot_w64(nib != 0u);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  // sums (and the maximum blended index) over the quad
  cr += qdpp<kQuadXor1>(cr); cr += qdpp<kQuadXor2>(cr);
  cg += qdpp<kQuadXor1>(cg); cg += qdpp<kQuadXor2>(cg);
  cb += qdpp<kQuadXor1>(cb); cb += qdpp<kQuadXor2>(cb);
  D += qdpp<kQuadXor1>(D); D += qdpp<kQuadXor2>(D);
  if (kKeep) {
    last = max(last, qdpp_u<kQuadXor1>(last));
    last = max(last, qdpp_u<kQuadXor2>(last));
  }
  if (valid && j == 0) {
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
  evals_out += evals;
}

constexpr int kRenderWaves = RENDER_WAVES;  // independent waves per workgroup

template <bool kFixed, bool kKeep>
__global__ __launch_bounds__(64 * kRenderWaves) void render_kernel(
    const ViewDev* __restrict__ views, int nviews, const float2* __restrict__ dtab,
    const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ list, const uint2* __restrict__ rects,
    const Record* __restrict__ recs, Opts op, HeavyTiles heavy, float* __restrict__ rgb, float* __restrict__ depth,
    float* __restrict__ trans, uint32_t* __restrict__ nlast, float* __restrict__ tfinal,
    unsigned long long* __restrict__ stats) {
  __shared__ float4 s_all[kRenderWaves][kWin][4];  // each wave's own window of records
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  float4(*s_rec)[4] = s_all[wv];

  const int heavy_waves = kHeavySplit * heavy.hslots;
  const int wi = wave_index(blockIdx.x, gridDim.x, kRenderWaves, wv, heavy_waves);
  if (wi < heavy_waves) {
    // block wi % 16 of the listed heavy tiles wi / 16, wi / 16 + slots, ...
    uint64_t hevals = 0;
    const int nh = (int)min(*heavy.count, (unsigned long long)heavy.hmax);
    for (int h = wi / kHeavySplit; h < nh; h += heavy.hslots) {
      const WaveBlock Wh = heavy_block((int)heavy.list[h], wi % kHeavySplit, views, nviews);
      if (!Wh.live) continue;
      render_heavy_block<kFixed, kKeep>(Wh, views[Wh.v], dtab, ranges[Wh.tile], ranges[Wh.tile + 1], list, rects,
                                        recs, op, s_rec, rgb, depth, trans, nlast, tfinal, hevals);
    }
    add_evals<kRenderWaves>(stats, heavy.evals, hevals);
    return;
  }
  const WaveBlock W = ordinary_block(wi, heavy_waves, views, nviews, heavy.flag);
  if (!W.live) {
    add_evals<kRenderWaves>(stats, heavy.evals, 0);
    return;
  }
  const ViewDev& V = views[W.v];
  const int tile = W.tile;
  const uint32_t start = ranges[tile], end = ranges[tile + 1];
  const uint32_t hx = (uint32_t)W.bx0 >> 3, hy = (uint32_t)W.by0 >> 3;  // half-tile of the block
  const int lane = threadIdx.x & 63;
  const int px = W.bx0 + (lane & 7), py = W.by0 + (lane >> 3);
  const bool valid = px < V.width && py < V.height;

  float dx, dy, dz;
  pixel_direction(V, dtab, px, py, dx, dy, dz);

  const QuadCone Q = block_cone(V, dtab, W.bx0, W.by0, 8);
  float T = 1.0f, cr = 0.0f, cg = 0.0f, cb = 0.0f, D = 0.0f;
  uint32_t last = start;
  uint64_t evals = 0;
  uint64_t done = __builtin_amdgcn_ballot_w64(!valid);  // wave mask of terminated (or absent) rays
  const int amax_bits = __float_as_int(op.alpha_max);

  // Prefetch of one window into registers: entry base + k goes to lane k.
  // The loads are unconditional (a lane past the end reads the tile's first
  // entry), so the prefetched values stay plain register values.
  if (start >= end) {
    // empty tile: background
    if (valid) {
      const int64_t hw = (int64_t)V.width * V.height;
      const int64_t p = (int64_t)py * V.width + px;
      float* out = rgb + 3 * (int64_t)V.pix_base;
      out[p] = 0.0f;
      out[hw + p] = 0.0f;
      out[2 * hw + p] = 0.0f;
      const int64_t gp = (int64_t)V.pix_base + p;
      if (depth) depth[gp] = 0.0f;
      if (trans) trans[gp] = 1.0f;
      if (kKeep) {
        nlast[gp] = start;
        tfinal[gp] = 1.0f;
      }
    }
    add_evals<kRenderWaves>(stats, heavy.evals, 0);
    return;
  }
  float4 p0, p1, p2, p3;
  bool phit;
  auto fetch = [&](uint32_t b) {
    const uint32_t e = b + lane;
    const uint32_t item = list[e < end ? e : start];
    const uint2 rc = rects[item];
    phit = e < end && (rc.x & 0xffffu) <= hx && hx <= (rc.x >> 16) && (rc.y & 0xffffu) <= hy && hy <= (rc.y >> 16);
    const float4* r = reinterpret_cast<const float4*>(recs + item);
    p0 = r[0]; p1 = r[1]; p2 = r[2]; p3 = r[3];
  };
  fetch(start);

  for (uint32_t base = start; base < end && ~done != 0; base += kWin) {
    // entries whose rectangle meets the half-tile and whose contribution cone
    // reaches one of its rays
    if (phit && op.cone_cull) phit = cone_meets_quad(p0, p1, p2, p3, Q, op.log2_amin, kFixed);
    uint64_t m = __builtin_amdgcn_ballot_w64(phit);
    if (phit) {
      s_rec[lane][0] = p0; s_rec[lane][1] = p1; s_rec[lane][2] = p2; s_rec[lane][3] = p3;
    }
    if (base + kWin < end) fetch(base + kWin);  // in flight while this window blends
    // LDS traffic of one wave completes in order; the fences keep the
    // compiler from moving the window's reads above its writes (and the next
    // window's writes above these reads)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    while (m != 0 && ~done != 0) {
      const int k = __builtin_ctzll(m);
      m &= m - 1;
      Record R;
      float4* rr = reinterpret_cast<float4*>(&R);
      rr[0] = s_rec[k][0]; rr[1] = s_rec[k][1]; rr[2] = s_rec[k][2]; rr[3] = s_rec[k][3];
      evals += (uint64_t)__popcll(~done);
      blend_one<kFixed, kKeep>(R, dx, dy, dz, op, amax_bits, base + k, done, T, cr, cg, cb, D, last);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
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
  add_evals<kRenderWaves>(stats, heavy.evals, evals);
}

// Render with the splat opacity instead of the exact one (the render-time
// swap of the paper's local-affine ablation): alpha = sigma exp(-m / 2) with
// m = d^T C^-1 d the conic distance of the ray's BEAP angles from the mean's,
// C the local affine footprint.  The association stays the exact PBF one and
// nothing is culled beyond its half-tile rectangles, so a splat footprint
// reaching past the rectangle is cut there (the culling mismatch the swap
// exposes).  Ordinary 8x8 half-tile waves for every tile; depth accumulates
// the means' camera distances.  No backward state is kept.
__global__ __launch_bounds__(64 * kRenderWaves) void render_splat_kernel(
    const ViewDev* __restrict__ views, int nviews, const float2* __restrict__ dtab,
    const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ list, const uint2* __restrict__ rects,
    const Record* __restrict__ recs, Opts op, float* __restrict__ rgb, float* __restrict__ depth,
    float* __restrict__ trans) {
  __shared__ float4 s_all[kRenderWaves][kWin][4];
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  float4(*s_rec)[4] = s_all[wv];
  const int wi = wave_index(blockIdx.x, gridDim.x, kRenderWaves, wv, 0);
  const WaveBlock W = ordinary_block(wi, 0, views, nviews, nullptr);
  if (!W.live) return;
  const ViewDev& V = views[W.v];
  const uint32_t start = ranges[W.tile], end = ranges[W.tile + 1];
  const uint32_t hx = (uint32_t)W.bx0 >> 3, hy = (uint32_t)W.by0 >> 3;
  const int lane = threadIdx.x & 63;
  const int px = W.bx0 + (lane & 7), py = W.by0 + (lane >> 3);
  const bool valid = px < V.width && py < V.height;
  const float2 cth = dtab[V.dx_off + min(px, V.width - 1)];
  const float2 cph = dtab[V.dy_off + min(py, V.height - 1)];
  const float th = atan2f(cth.x, cth.y), ph = atan2f(cph.x, cph.y);
  const float PI = 3.14159265358979f;
  float T = 1.0f, cr = 0.0f, cg = 0.0f, cb = 0.0f, D = 0.0f;
  uint64_t done = __builtin_amdgcn_ballot_w64(!valid);
  for (uint32_t base = start; base < end && ~done != 0; base += kWin) {
    const uint32_t e = base + lane;
    bool hit = false;
    if (e < end) {
      const uint32_t item = list[e];
      const uint2 rc = rects[item];
      hit = (rc.x & 0xffffu) <= hx && hx <= (rc.x >> 16) && (rc.y & 0xffffu) <= hy && hy <= (rc.y >> 16);
      if (hit) {
        const float4* r = reinterpret_cast<const float4*>(recs + item);
        s_rec[lane][0] = r[0]; s_rec[lane][1] = r[1]; s_rec[lane][2] = r[2]; s_rec[lane][3] = r[3];
      }
    }
    uint64_t m = __builtin_amdgcn_ballot_w64(hit);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    while (m != 0 && ~done != 0) {
      const int k = __builtin_ctzll(m);
      m &= m - 1;
      Record R;
      float4* rr = reinterpret_cast<float4*>(&R);
      rr[0] = s_rec[k][0]; rr[1] = s_rec[k][1]; rr[2] = s_rec[k][2]; rr[3] = s_rec[k][3];
      float dt = th - R.g[0];
      dt = dt > PI ? dt - 2.0f * PI : (dt < -PI ? dt + 2.0f * PI : dt);
      const float dp = ph - R.g[1];
      const float q = fmaf(R.g[2] * dt, dt, fmaf(2.0f * R.g[3] * dt, dp, R.g[4] * dp * dp));
      const float a_raw = __builtin_amdgcn_exp2f(fmaf(-0.72134752044448170f, q, R.lsig));
      const uint64_t ok = ~done & __builtin_amdgcn_ballot_w64(a_raw >= op.alpha_min);
      const float a = fminf(a_raw, op.alpha_max);
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
      D = fmaf(w, R.c1, D);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
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
  }
}

// Flags tiles whose list is longer than 3x the mean over their own view's
// tiles (+64) as heavy and lists them (in any order).  A view has fewer than
// a third of its tiles above that bound, so hmax = ntiles / 3 + 1 slots never
// run out: the heavy set of a view depends on that view alone, whatever it is
// batched with.
__global__ __launch_bounds__(256) void mark_heavy_kernel(const uint32_t* __restrict__ ranges, int64_t ntiles,
                                                         const ViewDev* __restrict__ views, int nviews,
                                                         uint32_t* __restrict__ heavy_list,
                                                         uint32_t* __restrict__ heavy_flag,
                                                         unsigned long long* __restrict__ heavy_count, int hmax,
                                                         unsigned long long* __restrict__ evals) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (evals && t < kEvalSlots) evals[t * kEvalStride] = 0ull;  // the render's counters, cleared for it
  if (t >= ntiles) return;
  int v = 0;
  while (v + 1 < nviews && t >= views[v + 1].tile_base) ++v;
  const ViewDev& V = views[v];
  const int64_t vt = (int64_t)V.tiles_x * V.tiles_y;
  const uint32_t total = ranges[V.tile_base + vt] - ranges[V.tile_base];
  const uint32_t cnt = ranges[t + 1] - ranges[t];
  const uint64_t thr = 3ull * total / (uint64_t)vt + 64ull;
  uint32_t flag = 0u;
  if (cnt > thr) {
    const unsigned long long slot = atomicAdd(heavy_count, 1ull);
    if (slot < (unsigned long long)hmax) {
      heavy_list[slot] = (uint32_t)t;
      flag = 1u;
    }
  }
  heavy_flag[t] = flag;
}

int heavy_capacity(int64_t ntiles) { return (int)(ntiles / 3 + 1); }
// the list, padded to 128 bytes, then the render's evaluated-pair counters
int64_t heavy_evals_offset(int hmax) { return ((int64_t)hmax + 31) / 32 * 32; }
int64_t heavy_list_words(int64_t ntiles) {
  return heavy_evals_offset(heavy_capacity(ntiles)) + 2 * (int64_t)kEvalSlots * kEvalStride;
}
int heavy_slots(int hmax) { return std::min(hmax, 256); }

void launch_mark_heavy(hipStream_t st, const uint32_t* ranges, int64_t ntiles, const ViewDev* views, int nviews,
                       const HeavyTiles& h) {
  if (ntiles <= 0) return;
  hipLaunchKernelGGL(mark_heavy_kernel, dim3((unsigned)((ntiles + 255) / 256)), dim3(256), 0, st, ranges, ntiles,
                     views, nviews, h.list, h.flag, h.count, h.hmax, h.evals);
}

void launch_render_splat(hipStream_t st, int64_t ntiles, const ViewDev* views, int nviews, const float2* dtab,
                         const uint32_t* ranges, const uint32_t* list, const uint2* rects, const Record* recs,
                         const Opts& op, float* rgb, float* depth, float* trans) {
  if (ntiles <= 0) return;
  const unsigned grid = (unsigned)(4 * ntiles / kRenderWaves);
  hipLaunchKernelGGL(render_splat_kernel, dim3(grid), dim3(64 * kRenderWaves), 0, st, views, nviews, dtab, ranges,
                     list, rects, recs, op, rgb, depth, trans);
}

void launch_render(hipStream_t st, bool fixed_lambda, int64_t ntiles, const ViewDev* views, int nviews,
                   const float2* dtab, const uint32_t* ranges, const uint32_t* list, const uint2* rects,
                   const Record* recs, const Opts& op, const HeavyTiles& heavy, float* rgb, float* depth,
                   float* trans, uint32_t* nlast, float* tfinal, unsigned long long* stats) {
  if (ntiles <= 0) return;
  const bool keep = nlast != nullptr && tfinal != nullptr;
  // waves: 16 per heavy slot, 4 per tile (both multiples of kRenderWaves)
  const unsigned grid = (unsigned)((kHeavySplit * heavy.hslots + 4 * ntiles) / kRenderWaves);
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * kRenderWaves), 0, st, views, nviews, dtab, ranges, list, rects,
                       recs, op, heavy, rgb, depth, trans, nlast, tfinal, stats);
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
