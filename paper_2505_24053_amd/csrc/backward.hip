// Gradient of the render (App. C, two-stage propagation).
//
// Render backward (ray-wise, "RenderCUDA" stage): one wave per 8x8 half-tile
// as in the forward, walking the tile's list back to front in windows of 64
// entries from the largest saved last-blended index of its rays, with the
// forward's rectangle and contribution-cone skips.  A pair is replayed only
// if the forward blended it (same evaluation functions, bit-identical
// decisions); the transmittance before it is recovered as T / (1 - alpha)
// (no per-sample state is stored).  Per pair:
//   dL/dc     = alpha T G,           dL/dalpha = T (c - C_behind) . G,
//   dL/dkappa = -alpha / 2 dL/dalpha,
// and, in the canonical frame rotated so that o_u = (0, 0, r) (u' = Q Wc d,
// g = r (u'x, u'y, -u'z), ss = |g|^2, mm = gx^2 + gy^2), the corrected-sign
// chain  dkappa/do_u = d_u x g_m,  dkappa/dd_u = -(2 kappa/|d_u|^2) d_u
// + g_m x o_u  (g_m = 2 m_u / |d_u|^2, m_u = o_u x d_u) reads
//   dkappa/do_u' = (2 r / ss) (gx gz, gy gz, mm),
//   dkappa/du'   = (2 r / ss) (r^2 / ss) (gz^2 gx, gz^2 gy, mm gz).
// Each wave reduces its 16 per-pair partials (dlog sigma, dc[3], do_u'[3],
// du' d^T [9]) with a value-splitting butterfly (17 shuffles) and 16 lanes
// add them to the item's accumulator.
//
// Preprocess backward (Gaussian-wise, "PreprocessCUDA" stage): one lane per
// Gaussian, summing over views: dWc = Q^T dP', do_u = Q^T do_u';
// dW = dWc Rc + do_u (o - mu)^T (Eq. b9), dmu = -W^T do_u (mean gradient) plus
// the SH view-direction term; ds_k = -sum_j dW_kj R_jk / s_k^2 (Eq. scaling);
// dq through the four dW/dq matrices (Eq. rotation) and the normalisation.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "geer_common.h"
#include "geer_device.h"

namespace geer {

constexpr int kWinB = 64;  // list entries staged per wave pass
constexpr int kAcc = 16;  // accumulator floats per (Gaussian, view) item

// Lane exchanges for the reduction: DPP within rows of 16 lanes, and the
// gfx950 row swaps across rows.
template <int kCtrl>
__device__ __forceinline__ float dpp(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), kCtrl, 0xF, 0xF, true));
}
// A quad or row permute that leaves the lanes' own values where the source
// lane is outside the rule's reach (bound_ctrl off: the old value stays).
template <int kCtrl>
__device__ __forceinline__ float qdppb(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(x), __float_as_int(x), kCtrl, 0xF, 0xF, false));
}
constexpr int kDppXor1 = 0xB1;         // quad_perm [1, 0, 3, 2]
constexpr int kDppXor2 = 0x4E;         // quad_perm [2, 3, 0, 1]
constexpr int kDppRowMirror = 0x140;   // lane i <-> 15 - i within each row of 16
constexpr int kDppHalfMirror = 0x141;  // lane i <-> 7 - i within each half row of 8

// a + b after swapping lanes 32..63 of a with lanes 0..31 of b: lanes below
// 32 get a summed over the lane pair (i, i + 32), the others b.
__device__ __forceinline__ float swap32_add(float a, float b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
// The same with rows of 16: rows 0 and 2 get a summed over (i, i + 16), rows 1 and 3 b.
__device__ __forceinline__ float swap16_add(float a, float b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Sum v[0..15] over the wave (every lane active) by value splitting: at
// each level a lane keeps half of its values and adds its partner's partial
// sums of them (partners differ in the level's lane bit and agree in the
// bits already split on; the mirrors pair lane i with 15 - i and 7 - i).
// Lanes with (lane & 3) == 0 end up holding the total of value index idx
// and add it to dst[idx].
__device__ __forceinline__ void wave_reduce16_add(const float v[16], float* __restrict__ dst) {
  const int lane = threadIdx.x & 63;
  const bool h32 = lane & 32, h16 = lane & 16, h8 = lane & 8, h4 = lane & 4;
  float a8[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) a8[j] = swap32_add(v[j], v[8 + j]);  // lanes >= 32 hold values 8..15
  float a4[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) a4[j] = swap16_add(a8[j], a8[4 + j]);  // odd rows hold the upper half
  float a2[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const float send = h8 ? a4[j] : a4[2 + j];
    const float keep = h8 ? a4[2 + j] : a4[j];
    a2[j] = keep + dpp<kDppRowMirror>(send);
  }
  float a1 = (h4 ? a2[1] : a2[0]) + dpp<kDppHalfMirror>(h4 ? a2[0] : a2[1]);
  a1 += dpp<kDppXor1>(a1);
  a1 += dpp<kDppXor2>(a1);
  const int idx = (h32 ? 8 : 0) + (h16 ? 4 : 0) + (h8 ? 2 : 0) + (h4 ? 1 : 0);
  if ((lane & 3) == 0 && a1 != 0.0f) unsafeAtomicAdd(dst + idx, a1);
}

// Row rotations (DPP row_ror) for the heavy blocks' reduction: within a row
// of 16 lanes, lane i reads lane (i - n) mod 16.
constexpr int kDppRor4 = 0x124, kDppRor8 = 0x128, kDppRor12 = 0x12C;
// Quad permutes for the heavy blocks' scans: lane j of a quad reads lane
// j - 1 (j - 2), and lane 3.
constexpr int kQuadPrev1 = 0x90;  // quad_perm [0, 0, 1, 2]
constexpr int kQuadPrev2 = 0x44;  // quad_perm [0, 1, 0, 1]
constexpr int kQuadLast = 0xFF;   // quad_perm [3, 3, 3, 3]

// Sum v[0..15] over the 16 lanes that share lane & 3 (the rays of one hit in
// a heavy block), by value splitting on lane bits 5, 4, 3 and 2: the row
// swaps for bits 5 and 4, row_ror 8 for bit 3 (the xor within a row), and
// for bit 2 row_ror 12 (lane i + 4) or row_ror 4 (lane i - 4).  Lane i ends
// with value (i >> 2) & 15, summed.
__device__ __forceinline__ float quad_reduce16(const float v[16]) {
  const int lane = threadIdx.x & 63;
  const bool h8 = lane & 8, h4 = lane & 4;
  float a8[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) a8[j] = swap32_add(v[j], v[8 + j]);
  float a4[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) a4[j] = swap16_add(a8[j], a8[4 + j]);
  float a2[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const float send = h8 ? a4[j] : a4[2 + j];
    const float keep = h8 ? a4[2 + j] : a4[j];
    a2[j] = keep + dpp<kDppRor8>(send);
  }
  const float send = h4 ? a2[0] : a2[1];
  const float from_up = dpp<kDppRor12>(send), from_down = dpp<kDppRor4>(send);
  return (h4 ? a2[1] : a2[0]) + (h4 ? from_down : from_up);
}

// Back-to-front replay of a heavy tile's 4x4 block with all 64 lanes: lane
// 4 r + j holds ray r and, in each step, the j-th of the next four hits of
// the window, back to front.  The sequential replay is kept: the
// transmittance in front of hit j is T divided by the quad's inclusive
// prefix product of (1 - alpha) over the replayed hits, and the colour behind
// it is the quad's exclusive prefix composition of the maps
// cb -> alpha c + (1 - alpha) cb applied to the colour behind the step.  The
// 16 partials of each hit are summed over its 16 rays (quad_reduce16) and
// added by one lane each.
template <bool kFixed>
__device__ __forceinline__ void backward_heavy_block(const WaveBlock& W, const ViewDev* __restrict__ views,
                                                     const float2* __restrict__ dtab,
                                                     const uint32_t* __restrict__ ranges,
                                                     const uint32_t* __restrict__ list,
                                                     const uint2* __restrict__ rects, const Record* __restrict__ recs,
                                                     const Opts& op, const uint32_t* __restrict__ nlast,
                                                     const float* __restrict__ tfinal,
                                                     const float* __restrict__ dl_drgb, float* __restrict__ acc,
                                                     float4 (*s_rec)[4], uint32_t* s_item, uint64_t& evals) {
  const ViewDev& V = views[W.v];
  const int tile = W.tile;
  const uint32_t hx = (uint32_t)W.bx0 >> 3, hy = (uint32_t)W.by0 >> 3;
  const int lane = threadIdx.x & 63;
  const int j = lane & 3, r = lane >> 2;
  const int px = W.bx0 + (r & 3), py = W.by0 + (r >> 2);
  const bool valid = px < V.width && py < V.height;
  float dx, dy, dz;
  pixel_direction(V, dtab, px, py, dx, dy, dz);
  const QuadCone Q = block_cone(V, dtab, W.bx0, W.by0, 4);

  const uint32_t start = ranges[tile];
  const int64_t hw = (int64_t)V.width * V.height;
  const int64_t p = (int64_t)py * V.width + px;
  const int64_t gp = (int64_t)V.pix_base + p;
  float T = 1.0f, G0 = 0.0f, G1 = 0.0f, G2 = 0.0f;
  uint32_t last = start;
  if (valid) {
    T = tfinal[gp];
    last = nlast[gp];
    const float* g = dl_drgb + 3 * (int64_t)V.pix_base;
    G0 = g[p];
    G1 = g[hw + p];
    G2 = g[2 * hw + p];
  }
  float cb0 = 0.0f, cb1 = 0.0f, cb2 = 0.0f;  // colour of everything behind the step

  uint32_t top = last;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) top = max(top, (uint32_t)__shfl_xor((int)top, off));

  float4 p0, p1, p2, p3;
  uint32_t pitem = 0;
  bool phit = false;
  auto fetch = [&](uint32_t b, uint32_t e_end) {
    const uint32_t e = b + lane;
    phit = false;
    if (e < e_end) {
      pitem = list[e];
      const uint2 rc = rects[pitem];
      phit = (rc.x & 0xffffu) <= hx && hx <= (rc.x >> 16) && (rc.y & 0xffffu) <= hy && hy <= (rc.y >> 16);
      if (phit) {
        const float4* rp = reinterpret_cast<const float4*>(recs + pitem);
        p0 = rp[0]; p1 = rp[1]; p2 = rp[2]; p3 = rp[3];
      }
    }
  };
  uint32_t bend = top;
  uint32_t bbase = bend > start + kWinB ? bend - kWinB : start;
  if (start < top) fetch(bbase, bend);

  while (bend > start) {
    if (phit && op.cone_cull) phit = cone_meets_quad(p0, p1, p2, p3, Q, op.log2_amin, kFixed);
    uint64_t m = __builtin_amdgcn_ballot_w64(phit);
    if (phit) {
      s_rec[lane][0] = p0; s_rec[lane][1] = p1; s_rec[lane][2] = p2; s_rec[lane][3] = p3;
      s_item[lane] = pitem;
    }
    const uint32_t base = bbase;
    bend = bbase;
    bbase = bend > start + kWinB ? bend - kWinB : start;
    if (bend > start) fetch(bbase, bend);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    while (m != 0) {
      // the next (up to) four hits, back to front
      int kh[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        kh[q] = m != 0 ? 63 - __builtin_clzll(m) : -1;
        if (m != 0) m &= ~(1ull << kh[q]);
      }
      const int k = j == 0 ? kh[0] : (j == 1 ? kh[1] : (j == 2 ? kh[2] : kh[3]));
      // a lane without a hit reads the group's first hit so that everything
      // it computes is finite; it replays nothing
      const bool has = k >= 0;
      const int ks = has ? k : kh[0];
      Record R;
      float4* rr = reinterpret_cast<float4*>(&R);
      rr[0] = s_rec[ks][0]; rr[1] = s_rec[ks][1]; rr[2] = s_rec[ks][2]; rr[3] = s_rec[ks][3];
      const PairEval E = eval_pair(R, dx, dy, dz);
      const uint32_t e = base + (uint32_t)ks;
      const bool in_range = valid & has & (e < last);
      evals += (uint64_t)__popcll(__builtin_amdgcn_ballot_w64(in_range));
      const bool on = in_range & pair_contributes<kFixed>(R, E, op);
      const float a = clamp_alpha(E.a_raw, op);
      const bool clamped = !(E.a_raw < op.alpha_max);
      // per-slot map cb -> A cb + B of the hit (identity when not replayed)
      const float fa = on ? 1.0f - a : 1.0f;
      float Ai = fa, B0 = on ? a * R.rgb[0] : 0.0f, B1 = on ? a * R.rgb[1] : 0.0f, B2 = on ? a * R.rgb[2] : 0.0f;
      // inclusive prefix over the quad (slot 0 is the furthest back): the
      // later map after the earlier one, x -> A2 (A1 x + B1) + B2
      {
        const float pA = qdppb<kQuadPrev1>(Ai), pB0 = qdppb<kQuadPrev1>(B0), pB1 = qdppb<kQuadPrev1>(B1),
                    pB2 = qdppb<kQuadPrev1>(B2);
        if (j >= 1) {
          B0 = fmaf(Ai, pB0, B0);
          B1 = fmaf(Ai, pB1, B1);
          B2 = fmaf(Ai, pB2, B2);
          Ai *= pA;
        }
        const float qA = qdppb<kQuadPrev2>(Ai), qB0 = qdppb<kQuadPrev2>(B0), qB1 = qdppb<kQuadPrev2>(B1),
                    qB2 = qdppb<kQuadPrev2>(B2);
        if (j >= 2) {
          B0 = fmaf(Ai, qB0, B0);
          B1 = fmaf(Ai, qB1, B1);
          B2 = fmaf(Ai, qB2, B2);
          Ai *= qA;
        }
      }
      // exclusive prefix (the maps of the hits behind this one) applied to the step's colour
      const float eA = qdppb<kQuadPrev1>(Ai), eB0 = qdppb<kQuadPrev1>(B0), eB1 = qdppb<kQuadPrev1>(B1),
                  eB2 = qdppb<kQuadPrev1>(B2);
      const float c0 = j >= 1 ? fmaf(eA, cb0, eB0) : cb0;
      const float c1 = j >= 1 ? fmaf(eA, cb1, eB1) : cb1;
      const float c2 = j >= 1 ? fmaf(eA, cb2, eB2) : cb2;
      // transmittance in front of this hit: T over the inclusive product of (1 - alpha)
      const float Tb = T * __builtin_amdgcn_rcpf(Ai);
      const float w = on ? a * Tb : 0.0f;
      float part[kAcc];
      part[1] = w * G0;
      part[2] = w * G1;
      part[3] = w * G2;
      const float dla = on ? Tb * ((R.rgb[0] - c0) * G0 + (R.rgb[1] - c1) * G1 + (R.rgb[2] - c2) * G2) : 0.0f;
      const float dlk = clamped ? 0.0f : -0.5f * a * dla;  // dL/dkappa
      part[0] = clamped ? 0.0f : dla * a;                  // dL/dlog(sigma)
      const float rr_ = __builtin_amdgcn_sqrtf(R.c1);
      const float f = 2.0f * rr_ * E.inv * dlk;
      part[4] = f * E.gx * E.gz;
      part[5] = f * E.gy * E.gz;
      part[6] = f * E.mm;
      const float h = f * (R.c1 * E.inv);
      const float gz2 = E.gz * E.gz;
      const float du0 = h * gz2 * E.gx, du1 = h * gz2 * E.gy, du2 = h * E.mm * E.gz;
      part[7] = du0 * dx; part[8] = du0 * dy; part[9] = du0 * dz;
      part[10] = du1 * dx; part[11] = du1 * dy; part[12] = du1 * dz;
      part[13] = du2 * dx; part[14] = du2 * dy; part[15] = du2 * dz;
      // the step's state for the next one: the whole quad's map and product
      T *= __builtin_amdgcn_rcpf(qdppb<kQuadLast>(Ai));
      cb0 = fmaf(qdppb<kQuadLast>(Ai), cb0, qdppb<kQuadLast>(B0));
      cb1 = fmaf(qdppb<kQuadLast>(Ai), cb1, qdppb<kQuadLast>(B1));
      cb2 = fmaf(qdppb<kQuadLast>(Ai), cb2, qdppb<kQuadLast>(B2));
      const float sum = quad_reduce16(part);
      if (has && sum != 0.0f) unsafeAtomicAdd(acc + (int64_t)s_item[ks] * kAcc + ((lane >> 2) & 15), sum);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

constexpr int kBackWaves = 2;  // independent waves per workgroup

// Back-to-front replay of one block of rays (8x8, or 4x4 in heavy tiles).
template <bool kFixed>
__device__ __forceinline__ void backward_block(const WaveBlock& W, const ViewDev* __restrict__ views,
                                               const float2* __restrict__ dtab, const uint32_t* __restrict__ ranges,
                                               const uint32_t* __restrict__ list, const uint2* __restrict__ rects,
                                               const Record* __restrict__ recs, const Opts& op,
                                               const uint32_t* __restrict__ nlast, const float* __restrict__ tfinal,
                                               const float* __restrict__ dl_drgb, float* __restrict__ acc,
                                               float4 (*s_rec)[4], uint32_t* s_item, uint64_t& evals) {
  const ViewDev& V = views[W.v];
  const int tile = W.tile;
  const uint32_t hx = (uint32_t)W.bx0 >> 3, hy = (uint32_t)W.by0 >> 3;  // half-tile of the block
  const int lane = threadIdx.x & 63;
  const int lb = W.bs == 8 ? 3 : 2;
  const int px = W.bx0 + (lane & (W.bs - 1)), py = W.by0 + (lane >> lb);
  const bool valid = lane < W.bs * W.bs && px < V.width && py < V.height;
  float dx, dy, dz;
  pixel_direction(V, dtab, px, py, dx, dy, dz);
  const QuadCone Q = block_cone(V, dtab, W.bx0, W.by0, W.bs);

  const uint32_t start = ranges[tile];
  const int64_t hw = (int64_t)V.width * V.height;
  const int64_t p = (int64_t)py * V.width + px;
  const int64_t gp = (int64_t)V.pix_base + p;
  float T = 1.0f, G0 = 0.0f, G1 = 0.0f, G2 = 0.0f;
  uint32_t last = start;
  if (valid) {
    T = tfinal[gp];
    last = nlast[gp];
    const float* g = dl_drgb + 3 * (int64_t)V.pix_base;
    G0 = g[p];
    G1 = g[hw + p];
    G2 = g[2 * hw + p];
  }
  float cb0 = 0.0f, cb1 = 0.0f, cb2 = 0.0f;  // colour of everything behind, as seen just in front of it

  // this wave replays [start, max over its rays of last)
  uint32_t top = last;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) top = max(top, (uint32_t)__shfl_xor((int)top, off));

  float4 p0, p1, p2, p3;
  uint32_t pitem = 0;
  bool phit = false;
  auto fetch = [&](uint32_t b, uint32_t e_end) {
    const uint32_t e = b + lane;
    phit = false;
    if (e < e_end) {
      pitem = list[e];
      const uint2 rc = rects[pitem];
      phit = (rc.x & 0xffffu) <= hx && hx <= (rc.x >> 16) && (rc.y & 0xffffu) <= hy && hy <= (rc.y >> 16);
      if (phit) {
        const float4* r = reinterpret_cast<const float4*>(recs + pitem);
        p0 = r[0]; p1 = r[1]; p2 = r[2]; p3 = r[3];
      }
    }
  };
  uint32_t bend = top;
  uint32_t bbase = bend > start + kWinB ? bend - kWinB : start;
  if (start < top) fetch(bbase, bend);

  while (bend > start) {
    if (phit && op.cone_cull) phit = cone_meets_quad(p0, p1, p2, p3, Q, op.log2_amin, kFixed);
    uint64_t m = __builtin_amdgcn_ballot_w64(phit);
    if (phit) {
      s_rec[lane][0] = p0; s_rec[lane][1] = p1; s_rec[lane][2] = p2; s_rec[lane][3] = p3;
      s_item[lane] = pitem;
    }
    const uint32_t base = bbase;
    // prefetch the window in front of this one
    bend = bbase;
    bbase = bend > start + kWinB ? bend - kWinB : start;
    if (bend > start) fetch(bbase, bend);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    while (m != 0) {
      const int k = 63 - __builtin_clzll(m);  // back to front
      m &= ~(1ull << k);
      const uint32_t e = base + (uint32_t)k;
      Record R;
      float4* rr = reinterpret_cast<float4*>(&R);
      rr[0] = s_rec[k][0]; rr[1] = s_rec[k][1]; rr[2] = s_rec[k][2]; rr[3] = s_rec[k][3];
      const PairEval E = eval_pair(R, dx, dy, dz);
      const bool in_range = valid & (e < last);
      evals += (uint64_t)__popcll(__builtin_amdgcn_ballot_w64(in_range));
      const bool on = in_range & pair_contributes<kFixed>(R, E, op);
      if (__ballot(on) == 0) continue;
      const float a = clamp_alpha(E.a_raw, op);
      const bool clamped = !(E.a_raw < op.alpha_max);
      const float Tb = on ? T * __builtin_amdgcn_rcpf(1.0f - a) : T;  // transmittance in front of this Gaussian
      const float w = on ? a * Tb : 0.0f;
      float part[kAcc];
      part[1] = w * G0;
      part[2] = w * G1;
      part[3] = w * G2;
      const float dla = on ? Tb * ((R.rgb[0] - cb0) * G0 + (R.rgb[1] - cb1) * G1 + (R.rgb[2] - cb2) * G2) : 0.0f;
      cb0 = on ? fmaf(a, R.rgb[0] - cb0, cb0) : cb0;
      cb1 = on ? fmaf(a, R.rgb[1] - cb1, cb1) : cb1;
      cb2 = on ? fmaf(a, R.rgb[2] - cb2, cb2) : cb2;
      T = Tb;
      const float dlk = clamped ? 0.0f : -0.5f * a * dla;  // dL/dkappa
      part[0] = clamped ? 0.0f : dla * a;                  // dL/dlog(sigma)
      const float r = __builtin_amdgcn_sqrtf(R.c1);
      const float f = 2.0f * r * E.inv * dlk;               // dL/dkappa * 2 r / ss
      part[4] = f * E.gx * E.gz;
      part[5] = f * E.gy * E.gz;
      part[6] = f * E.mm;
      const float h = f * (R.c1 * E.inv);
      const float gz2 = E.gz * E.gz;
      const float du0 = h * gz2 * E.gx, du1 = h * gz2 * E.gy, du2 = h * E.mm * E.gz;
      part[7] = du0 * dx; part[8] = du0 * dy; part[9] = du0 * dz;
      part[10] = du1 * dx; part[11] = du1 * dy; part[12] = du1 * dz;
      part[13] = du2 * dx; part[14] = du2 * dy; part[15] = du2 * dz;
      wave_reduce16_add(part, acc + (int64_t)s_item[k] * kAcc);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}


template <bool kFixed>
__global__ __launch_bounds__(64 * kBackWaves) void render_backward_kernel(
    const ViewDev* __restrict__ views, int nviews, const float2* __restrict__ dtab,
    const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ list, const uint2* __restrict__ rects,
    const Record* __restrict__ recs, Opts op, HeavyTiles heavy, const uint32_t* __restrict__ nlast,
    const float* __restrict__ tfinal, const float* __restrict__ dl_drgb, float* __restrict__ acc,
    unsigned long long* __restrict__ evals_total, unsigned long long* __restrict__ eval_slots) {
  __shared__ float4 s_rec_all[kBackWaves][kWinB][4];  // each wave's own window
  __shared__ uint32_t s_item_all[kBackWaves][kWinB];
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  float4(*s_rec)[4] = s_rec_all[wv];
  uint32_t* s_item = s_item_all[wv];
  const int heavy_waves = kHeavySplit * heavy.hslots;
  const int wi = wave_index(blockIdx.x, gridDim.x, kBackWaves, wv, heavy_waves);
  // one block for an ordinary wave; for a heavy wave, block wi % 16 of the
  // listed heavy tiles wi / 16, wi / 16 + slots, ... (one call site, so the
  // replay is inlined once)
  const bool hw = wi < heavy_waves;
  const int nh = hw ? (int)min(*heavy.count, (unsigned long long)heavy.hmax) : 0;
  uint64_t evals = 0;  // (ray, entry) pairs replayed, as the forward counts them
  for (int h = wi / kHeavySplit;; h += heavy.hslots) {
    if (hw && h >= nh) break;
    if (hw) {
      const WaveBlock W = heavy_block((int)heavy.list[h], wi % kHeavySplit, views, nviews);
      if (W.live)
        backward_heavy_block<kFixed>(W, views, dtab, ranges, list, rects, recs, op, nlast, tfinal, dl_drgb, acc,
                                     s_rec, s_item, evals);
      continue;
    }
    const WaveBlock W = ordinary_block(wi, heavy_waves, views, nviews, heavy.flag);
    if (W.live)
      backward_block<kFixed>(W, views, dtab, ranges, list, rects, recs, op, nlast, tfinal, dl_drgb, acc, s_rec, s_item,
                             evals);
    break;
  }
  add_evals<kBackWaves>(evals_total, eval_slots, evals);
}

// ------------------------------------------------------------------------
// Gaussian-wise stage

// sum_k w_k grad B_k (x, y, z): the derivatives of the real SH basis (the
// same ones sh_basis gives) contracted with w, without a derivative table.
template <int kDeg>
__device__ __forceinline__ void sh_grad_dot(float x, float y, float z, const float w[16], float gv[3]) {
  gv[0] = gv[1] = gv[2] = 0.0f;
  if (kDeg < 1) return;
  const float C1 = 0.4886025119029199f;
  gv[0] -= C1 * w[3];
  gv[1] -= C1 * w[1];
  gv[2] += C1 * w[2];
  if (kDeg < 2) return;
  const float C20 = 1.0925484305920792f, C21 = -1.0925484305920792f, C22 = 0.31539156525252005f,
              C23 = -1.0925484305920792f, C24 = 0.5462742152960396f;
  const float xx = x * x, yy = y * y, zz = z * z;
  gv[0] += C20 * y * w[4] - 2.0f * C22 * x * w[6] + C23 * z * w[7] + 2.0f * C24 * x * w[8];
  gv[1] += C20 * x * w[4] + C21 * z * w[5] - 2.0f * C22 * y * w[6] - 2.0f * C24 * y * w[8];
  gv[2] += C21 * y * w[5] + 4.0f * C22 * z * w[6] + C23 * x * w[7];
  if (kDeg < 3) return;
  const float C30 = -0.5900435899266435f, C31 = 2.890611442640554f, C32 = -0.4570457994644658f,
              C33 = 0.3731763325901154f, C34 = -0.4570457994644658f, C35 = 1.445305721320277f,
              C36 = -0.5900435899266435f;
  gv[0] += C30 * 6.0f * x * y * w[9] + C31 * y * z * w[10] - 2.0f * C32 * x * y * w[11] -
           6.0f * C33 * x * z * w[12] + C34 * (4.0f * zz - 3.0f * xx - yy) * w[13] + 2.0f * C35 * x * z * w[14] +
           C36 * (3.0f * xx - 3.0f * yy) * w[15];
  gv[1] += C30 * (3.0f * xx - 3.0f * yy) * w[9] + C31 * x * z * w[10] + C32 * (4.0f * zz - xx - 3.0f * yy) * w[11] -
           6.0f * C33 * y * z * w[12] - 2.0f * C34 * x * y * w[13] - 2.0f * C35 * y * z * w[14] -
           6.0f * C36 * x * y * w[15];
  gv[2] += C31 * x * y * w[10] + 8.0f * C32 * y * z * w[11] + C33 * (6.0f * zz - 3.0f * xx - 3.0f * yy) * w[12] +
           8.0f * C34 * x * z * w[13] + C35 * (xx - yy) * w[14];
}

// Colour part of one view's Gaussian-wise backward: the SH coefficients'
// gradient into dsh and the view-direction term into dmu.  dc: dL/dc of the
// item's channels, zero where the forward clamped the colour (its record's
// rgb = max(raw, 0) is > 0 exactly when raw > 0).  The direction term is the
// gradient of sum_k w_k B_k with w_k = sum_c coef_kc dc_c, so each basis
// derivative is used once and no derivative table is kept.
template <int kDeg, typename ShPtr>
__device__ __forceinline__ void colour_grad(int64_t n, int64_t g, const float mu[3], ShPtr sh,
                                            const ViewDev& V, const float dc[3], float* dsh, float dmu[3]) {
  constexpr int K = (kDeg + 1) * (kDeg + 1);
  const float dv[3] = {mu[0] - V.campos[0], mu[1] - V.campos[1], mu[2] - V.campos[2]};
  const float dist = sqrtf(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
  const float vd[3] = {dv[0] / dist, dv[1] / dist, dv[2] / dist};
  float B[16];
  sh_basis(kDeg, vd, B, nullptr);
  float w[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    w[k] = 0.0f;
    if (k >= K) continue;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      dsh[k * 3 + c] += B[k] * dc[c];
      w[k] += sh[(int64_t)(k * 3 + c) * n + g] * dc[c];
    }
  }
  float gv[3];
  sh_grad_dot<kDeg>(vd[0], vd[1], vd[2], w, gv);
  const float vg = vd[0] * gv[0] + vd[1] * gv[1] + vd[2] * gv[2];
#pragma unroll
  for (int j = 0; j < 3; ++j) dmu[j] += (gv[j] - vd[j] * vg) / dist;
}

// dL/dc of an item's channels, zero where the forward clamped its colour.
__device__ __forceinline__ void colour_dc(const Record& R, float a1, float a2, float a3, float dc[3]) {
  dc[0] = R.rgb[0] > 0.0f ? a1 : 0.0f;
  dc[1] = R.rgb[1] > 0.0f ? a2 : 0.0f;
  dc[2] = R.rgb[2] > 0.0f ? a3 : 0.0f;
}

// The Gaussian-wise backward (App. C, second stage): per view the forward's
// association and frame are recomputed and the item's 16 ray-wise partials
// are pulled back to the mean, scale, rotation, opacity and (with kColour)
// the SH coefficients and the view direction.
template <int kDeg, bool kColour>
__global__ __launch_bounds__(256) void preprocess_backward_kernel(
    int64_t n, int32_t n_views, const float* __restrict__ mean, const float* __restrict__ scale,
    const float* __restrict__ quat, const float* __restrict__ opacity, const float* __restrict__ sh,
    const ViewDev* __restrict__ views, Opts op, const float* __restrict__ lam_tab, const float* __restrict__ edges,
    const uint32_t* __restrict__ counts, const float* __restrict__ acc, const Record* __restrict__ recs,
    int accumulate, float* __restrict__ g_mean, float* __restrict__ g_scale, float* __restrict__ g_quat,
    float* __restrict__ g_opacity, float* __restrict__ g_sh) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const float mu[3] = {mean[g], mean[n + g], mean[2 * n + g]};
  const float s[3] = {scale[g], scale[n + g], scale[2 * n + g]};
  const float q[4] = {quat[g], quat[n + g], quat[2 * n + g], quat[3 * n + g]};
  const float sigma = opacity[g];
  constexpr int K = (kDeg + 1) * (kDeg + 1);
  float dmu[3] = {0, 0, 0}, dW[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, dsig = 0.0f;
  float dsh[K * 3];
#pragma unroll
  for (int i = 0; i < K * 3; ++i) dsh[i] = 0.0f;
  float R[9], qh[4] = {1, 0, 0, 0}, qn = 1.0f;
  bool any = false;
  // views in groups of 8: the group's tile counts are loaded together, and
  // only the views where the Gaussian is visible (its accumulator written
  // by the ray-wise backward) are read
  uint32_t vis = 0u;
  for (int v = 0; v < n_views; ++v) {
    if ((v & 7) == 0) {
      vis = 0u;
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (v + k < n_views && counts[(int64_t)(v + k) * n + g] != 0u) vis |= 1u << k;
    }
    if (!((vis >> (v & 7)) & 1u)) continue;
    const int64_t item = (int64_t)v * n + g;
    const float4* ap = reinterpret_cast<const float4*>(acc + item * kAcc);
    const float4 A0 = ap[0], A1 = ap[1], A2 = ap[2], A3 = ap[3];
    const float a[16] = {A0.x, A0.y, A0.z, A0.w, A1.x, A1.y, A1.z, A1.w,
                         A2.x, A2.y, A2.z, A2.w, A3.x, A3.y, A3.z, A3.w};
    bool nz = false;
#pragma unroll
    for (int i = 0; i < 16; ++i) nz |= a[i] != 0.0f;
    if (!nz) continue;
    const ViewDev& Vw = views[v];
    AssocOut As;
    associate(mu, s, q, sigma, Vw, op, lam_tab, edges, As);
    Frame3 F;
    canonical_frame(As, s, F);
    any = true;
#pragma unroll
    for (int i = 0; i < 9; ++i) R[i] = As.R[i];
    qh[0] = As.qh[0]; qh[1] = As.qh[1]; qh[2] = As.qh[2]; qh[3] = As.qh[3];
    qn = As.qn;
    const float* Q0 = F.e1;
    const float* Q1 = F.e2;
    const float* Q2 = F.nn;
    // dWc = Q^T dP',  do_u = Q^T do_u'
    float dWc[9], dou[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
#pragma unroll
      for (int i = 0; i < 3; ++i) dWc[k * 3 + i] = Q0[k] * a[7 + i] + Q1[k] * a[10 + i] + Q2[k] * a[13 + i];
      dou[k] = Q0[k] * a[4] + Q1[k] * a[5] + Q2[k] * a[6];
    }
    // Wc = W Rc^T  =>  dW += dWc Rc ;  o_u = W (o - mu)  =>  dW += do_u (o - mu)^T
    const float om[3] = {Vw.campos[0] - mu[0], Vw.campos[1] - mu[1], Vw.campos[2] - mu[2]};
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        dW[k * 3 + j] += dWc[k * 3 + 0] * Vw.Rc[0 * 3 + j] + dWc[k * 3 + 1] * Vw.Rc[1 * 3 + j] +
                         dWc[k * 3 + 2] * Vw.Rc[2 * 3 + j] + dou[k] * om[j];
    // dmu = -W^T do_u, W[k][j] = R[j][k] / s_k
#pragma unroll
    for (int j = 0; j < 3; ++j)
      dmu[j] -= R[j * 3 + 0] / s[0] * dou[0] + R[j * 3 + 1] / s[1] * dou[1] + R[j * 3 + 2] / s[2] * dou[2];
    dsig += a[0] / sigma;
    if (kColour) {
      float dc[3];
      colour_dc(recs[item], a[1], a[2], a[3], dc);
      colour_grad<kDeg>(n, g, mu, sh, Vw, dc, dsh, dmu);
    }
  }
  float ds[3] = {0, 0, 0}, dq[4] = {0, 0, 0, 0};
  if (any) {
    // W[i][j] = R[j][i] / s_i  =>  ds_i = -sum_j dW_ij R_ji / s_i^2
#pragma unroll
    for (int i = 0; i < 3; ++i)
      ds[i] = -(dW[i * 3 + 0] * R[0 * 3 + i] + dW[i * 3 + 1] * R[1 * 3 + i] + dW[i * 3 + 2] * R[2 * 3 + i]) /
              (s[i] * s[i]);
    // X_ij = dW_ij / s_i, contracted with the four dW/dq matrices of the unit quaternion
    float X[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) X[i * 3 + j] = dW[i * 3 + j] / s[i];
    const float qr = qh[0], qi = qh[1], qj = qh[2], qk = qh[3];
    float dh[4];
    dh[0] = 2.0f * (X[1] * qk - X[2] * qj - X[3] * qk + X[5] * qi + X[6] * qj - X[7] * qi);
    dh[1] = 2.0f * (X[1] * qj + X[2] * qk + X[3] * qj - 2.0f * X[4] * qi + X[5] * qr + X[6] * qk - X[7] * qr -
                    2.0f * X[8] * qi);
    dh[2] = 2.0f * (-2.0f * X[0] * qj + X[1] * qi - X[2] * qr + X[3] * qi + X[5] * qk + X[6] * qr + X[7] * qk -
                    2.0f * X[8] * qj);
    dh[3] = 2.0f * (-2.0f * X[0] * qk + X[1] * qr + X[2] * qi - X[3] * qr - 2.0f * X[4] * qk + X[5] * qj +
                    X[6] * qi + X[7] * qj);
    const float proj = dh[0] * qr + dh[1] * qi + dh[2] * qj + dh[3] * qk;
#pragma unroll
    for (int c = 0; c < 4; ++c) dq[c] = (dh[c] - qh[c] * proj) / qn;
  }
  auto put = [&](float* dst, int64_t idx, float val) { dst[idx] = accumulate ? dst[idx] + val : val; };
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    put(g_mean, j * n + g, dmu[j]);
    put(g_scale, j * n + g, ds[j]);
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) put(g_quat, c * n + g, dq[c]);
  put(g_opacity, g, dsig);
  if (kColour) {
#pragma unroll
    for (int k = 0; k < K * 3; ++k) put(g_sh, (int64_t)k * n + g, dsh[k]);
  }
}

// The colour part of the Gaussian-wise backward for a batch of views, after
// a preprocess_backward_kernel launched without it: the SH coefficients'
// gradient is written (or, with accumulate, added) and the view-direction
// term added to g_mean.  Kept out of the geometric kernel for batches: the
// coefficients, their gradients and the basis derivatives would otherwise
// share its registers over every view.  A channel's clamp is read from the
// forward's colour (rgb = max(raw, 0) > 0 exactly when raw > 0), and the
// direction term is the gradient of sum_k w_k B_k with
// w_k = sum_c coef_kc dL/dc_c, so each basis derivative is used once.
template <int kDeg>
__global__ __launch_bounds__(256) void colour_backward_kernel(int64_t n, int32_t n_views,
                                                              const float* __restrict__ mean,
                                                              const float* __restrict__ sh,
                                                              const ViewDev* __restrict__ views,
                                                              const uint32_t* __restrict__ counts,
                                                              const float* __restrict__ acc,
                                                              const Record* __restrict__ recs, int accumulate,
                                                              float* __restrict__ g_mean, float* __restrict__ g_sh) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const float mu[3] = {mean[g], mean[n + g], mean[2 * n + g]};
  constexpr int K = (kDeg + 1) * (kDeg + 1);
  float dmu[3] = {0, 0, 0};
  float dsh[K * 3];
#pragma unroll
  for (int i = 0; i < K * 3; ++i) dsh[i] = 0.0f;
  // the coefficients are read in every view (from cache), not held across
  // the view loop beside the gradients
  const volatile float* shv = sh;
  for (int v = 0; v < n_views; ++v) {
    const int64_t item = (int64_t)v * n + g;
    if (counts[item] == 0u) continue;
    const float4 A0 = reinterpret_cast<const float4*>(acc + item * kAcc)[0];
    float dc[3];
    colour_dc(recs[item], A0.y, A0.z, A0.w, dc);
    if (dc[0] == 0.0f && dc[1] == 0.0f && dc[2] == 0.0f) continue;
    colour_grad<kDeg>(n, g, mu, shv, views[v], dc, dsh, dmu);
  }
#pragma unroll
  for (int j = 0; j < 3; ++j) g_mean[j * n + g] += dmu[j];
#pragma unroll
  for (int k = 0; k < K * 3; ++k) g_sh[(int64_t)k * n + g] = accumulate ? g_sh[(int64_t)k * n + g] + dsh[k] : dsh[k];
}

// Clears the accumulators of the items visible in their view (tile count
// above zero); the others are never written by the ray-wise backward and
// never read by the Gaussian-wise one.
__global__ __launch_bounds__(256) void zero_acc_kernel(float* __restrict__ acc, const uint32_t* __restrict__ counts,
                                                       int64_t nitems, unsigned long long* __restrict__ counters) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (counters && i <= kEvalSlots) counters[i * kEvalStride] = 0ull;  // the replay's pair counters and total
  if (i >= nitems || counts[i] == 0u) return;
  float4* a = reinterpret_cast<float4*>(acc + i * kAcc);
  const float4 z = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  a[0] = z; a[1] = z; a[2] = z; a[3] = z;
}

void launch_zero_acc(hipStream_t st, float* acc, const uint32_t* counts, int64_t nitems,
                     unsigned long long* counters) {
  const int64_t n = std::max<int64_t>(nitems, counters ? kEvalSlots + 1 : 0);
  if (n > 0)
    hipLaunchKernelGGL(zero_acc_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, acc, counts, nitems,
                       counters);
}

void launch_render_backward(hipStream_t st, bool fixed_lambda, int64_t ntiles, int32_t n_views, const ViewDev* views,
                            const float2* dtab, const Opts& op, const HeavyTiles& heavy, const uint32_t* ranges,
                            const uint32_t* list, const uint2* rects, const Record* recs, const uint32_t* nlast,
                            const float* tfinal, const float* dl_drgb, float* acc, unsigned long long* counters) {
  if (ntiles <= 0) return;
  // waves: 16 per heavy slot, 4 per tile (both multiples of kBackWaves)
  const unsigned grid = (unsigned)((kHeavySplit * heavy.hslots + 4 * ntiles) / kBackWaves);
  unsigned long long* total = counters ? counters + kEvalSlots * kEvalStride : nullptr;
  if (fixed_lambda)
    hipLaunchKernelGGL(render_backward_kernel<true>, dim3(grid), dim3(64 * kBackWaves), 0, st, views, n_views, dtab,
                       ranges, list, rects, recs, op, heavy, nlast, tfinal, dl_drgb, acc, total, counters);
  else
    hipLaunchKernelGGL(render_backward_kernel<false>, dim3(grid), dim3(64 * kBackWaves), 0, st, views, n_views, dtab,
                       ranges, list, rects, recs, op, heavy, nlast, tfinal, dl_drgb, acc, total, counters);
}

void launch_preprocess_backward(hipStream_t st, int64_t n, int32_t n_views, int32_t sh_degree, const float* mean,
                                const float* scale, const float* quat, const float* opacity, const float* sh,
                                const ViewDev* views, const float* edges, const float* lam_tab, const Opts& op,
                                const uint32_t* counts, const float* acc, const Record* recs, int accumulate,
                                float* g_mean, float* g_scale, float* g_quat, float* g_opacity, float* g_sh) {
  if (n <= 0) return;
  const dim3 grid((unsigned)((n + 255) / 256));
  // one view: the colour part in the same pass; a batch of views: a second kernel
#define GEER_PB(D)                                                                                                 \
  do {                                                                                                             \
    if (n_views == 1 || D == 0) {                                                                                  \
      hipLaunchKernelGGL((preprocess_backward_kernel<D, true>), grid, dim3(256), 0, st, n, n_views, mean, scale,  \
                         quat, opacity, sh, views, op, lam_tab, edges, counts, acc, recs, accumulate, g_mean,       \
                         g_scale, g_quat, g_opacity, g_sh);                                                        \
    } else {                                                                                                       \
      hipLaunchKernelGGL((preprocess_backward_kernel<D, false>), grid, dim3(256), 0, st, n, n_views, mean, scale, \
                         quat, opacity, sh, views, op, lam_tab, edges, counts, acc, recs, accumulate, g_mean,       \
                         g_scale, g_quat, g_opacity, g_sh);                                                        \
      hipLaunchKernelGGL(colour_backward_kernel<D>, grid, dim3(256), 0, st, n, n_views, mean, sh, views, counts,  \
                         acc, recs, accumulate, g_mean, g_sh);                                                    \
    }                                                                                                              \
  } while (0)
  switch (sh_degree) {
    case 0: GEER_PB(0); break;
    case 1: GEER_PB(1); break;
    case 2: GEER_PB(2); break;
    default: GEER_PB(3); break;
  }
#undef GEER_PB
}

void launch_backward(hipStream_t st, bool fixed_lambda, int64_t ntiles, int64_t n, int32_t n_views,
                     int32_t sh_degree, const float* mean, const float* scale, const float* quat,
                     const float* opacity, const float* sh, const ViewDev* views, const float2* dtab,
                     const float* edges, const float* lam_tab, const Opts& op, const HeavyTiles& heavy,
                     const uint32_t* ranges, const uint32_t* list, const uint2* rects, const Record* recs,
                     const uint32_t* counts, const uint32_t* nlast, const float* tfinal, const float* dl_drgb,
                     float* acc, int accumulate, float* g_mean, float* g_scale, float* g_quat, float* g_opacity,
                     float* g_sh, unsigned long long* counters) {
  launch_zero_acc(st, acc, counts, n * n_views, counters);
  launch_render_backward(st, fixed_lambda, ntiles, n_views, views, dtab, op, heavy, ranges, list, rects, recs, nlast,
                         tfinal, dl_drgb, acc, counters);
  launch_preprocess_backward(st, n, n_views, sh_degree, mean, scale, quat, opacity, sh, views, edges, lam_tab, op,
                             counts, acc, recs, accumulate, g_mean, g_scale, g_quat, g_opacity, g_sh);
}

}  // namespace geer
