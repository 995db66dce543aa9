// Stage (a): per-Gaussian preprocessing and particle bounding frustum (PBF).
//
// One lane per Gaussian; the lane loops over the views of the batch so the
// scene is read from HBM once per batch.  For every (Gaussian, view) item it
// writes the half-tile rectangle, tile count and depth key (the association,
// bit-exact IEEE single arithmetic in a fixed order, no contraction) and the
// 64-byte render record (radiometric, free-form FP32).  A single view gets
// its colour in the same pass; a batch of views gets it from a second kernel
// (one lane per item), so that the association runs without the
// coefficients' registers.
//
// PBF (Sec. 3.2, App. D.1): with M = Rc R S and mu_c = Rc mu + t, a plane
// through the camera y axis x = c z is tangent to the lambda-ellipsoid iff
// T22 c^2 - 2 T02 c + T00 = 0, T = lambda^2 Sigma_c - mu_c mu_c^T
// (Eq. solve_tan, pbf-cov3d); likewise T22 c^2 - 2 T12 c + T11 = 0 for planes
// through the x axis.  The discriminants are evaluated in the cancellation
// free form lambda^2 (|mu0 m2 - mu2 m0|^2 - lambda^2 |m0 x m2|^2) (m_a = row a
// of M).  Theta roots are mapped through the xi = 1 mirror tan(theta/2)
// (Eq. aabb) as homogeneous pairs, and the interval is the pair of mirrored
// candidates that brackets the centre's mirrored angle; an arc through the
// back direction becomes two pieces clipped to the field of view.  Phi uses
// tan(phi) directly; a Gaussian straddling z = 0 gives the complement of the
// root interval.  Bounds are padded outward by 2^-14 (1 + |x|) and compared
// with the half-tile edge tables (closed intervals).
#include <hip/hip_runtime.h>

#include "geer_common.h"
#include "geer_device.h"

namespace geer {

// Adds the block's sums of association entries and visible items to
// totals[0] and totals[1] (every thread of the 256-thread block calls it).
__device__ __forceinline__ void block_add_totals(unsigned long long e, unsigned long long vis,
                                                 unsigned long long* totals) {
  __shared__ unsigned long long red[2][4];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    e += __shfl_xor(e, off);
    vis += __shfl_xor(vis, off);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();  // the previous call's reads of red are done
  if (lane == 0) { red[0][wv] = e; red[1][wv] = vis; }
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned long long te = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    const unsigned long long tv = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    if (te) atomicAdd(&totals[0], te);
    if (tv) atomicAdd(&totals[1], tv);
  }
}

// The real SH basis functions of one band (degree) in direction (x, y, z),
// the terms of that band in the full basis.  No contraction, so the values
// do not depend on the code they are inlined into.
template <int kBand>
__device__ __forceinline__ void sh_band(float x, float y, float z, float B[7]) {
#pragma clang fp contract(off)
  if (kBand == 0) {
    B[0] = 0.28209479177387814f;
  } else if (kBand == 1) {
    const float C1 = 0.4886025119029199f;
    B[0] = -C1 * y; B[1] = C1 * z; B[2] = -C1 * x;
  } else if (kBand == 2) {
    const float xx = x * x, yy = y * y, zz = z * z;
    B[0] = 1.0925484305920792f * x * y;
    B[1] = -1.0925484305920792f * y * z;
    B[2] = 0.31539156525252005f * (2.0f * zz - xx - yy);
    B[3] = -1.0925484305920792f * x * z;
    B[4] = 0.5462742152960396f * (xx - yy);
  } else {
    const float xx = x * x, yy = y * y, zz = z * z;
    B[0] = -0.5900435899266435f * y * (3.0f * xx - yy);
    B[1] = 2.890611442640554f * x * y * z;
    B[2] = -0.4570457994644658f * y * (4.0f * zz - xx - yy);
    B[3] = 0.3731763325901154f * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
    B[4] = -0.4570457994644658f * x * (4.0f * zz - xx - yy);
    B[5] = 1.445305721320277f * z * (xx - yy);
    B[6] = -0.5900435899266435f * x * (xx - 3.0f * yy);
  }
}

// Adds band kBand of Gaussian g's colour in direction (x, y, z) to acc --
// the one per-view sequence of operations of both colour paths, so that a
// view renders the same bits alone and in a batch.
template <int kBand, int kDeg>
__device__ __forceinline__ void add_band(int64_t n, int64_t g, const float* __restrict__ sh, float x, float y,
                                         float z, float acc[3]) {
  if (kBand > kDeg) return;
  constexpr int k0 = kBand * kBand, kn = 2 * kBand + 1;
  float B[7];
  sh_band<kBand>(x, y, z, B);
#pragma unroll
  for (int i = 0; i < kn; ++i)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[c] = fmaf(B[i], sh[(int64_t)((k0 + i) * 3 + c) * n + g], acc[c]);
}

// Unit direction from view V's camera centre to the mean.
__device__ __forceinline__ void view_direction(const ViewDev& V, const float mu[3], float& x, float& y, float& z) {
#pragma clang fp contract(off)
  const float dv[3] = {mu[0] - V.campos[0], mu[1] - V.campos[1], mu[2] - V.campos[2]};
  const float dinv = rsqrtf(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
  x = dv[0] * dinv;
  y = dv[1] * dinv;
  z = dv[2] * dinv;
}

template <int kDeg, bool kColour>
__global__ __launch_bounds__(256) void preprocess_kernel(
    int64_t n, int32_t n_views, const float* __restrict__ mean, const float* __restrict__ scale,
    const float* __restrict__ quat, const float* __restrict__ opacity, const float* __restrict__ sh,
    const ViewDev* __restrict__ views, Opts op, const float* __restrict__ lam_tab,
    const float* __restrict__ edges, Record* __restrict__ recs, uint2* __restrict__ rects,
    uint32_t* __restrict__ keys, uint32_t* __restrict__ counts, unsigned long long* __restrict__ totals,
    int totals_stride, const unsigned long long* __restrict__ err_in) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // the sticky stall flag of earlier forwards, returned with this one's counts
  if (err_in && g == 0) totals[7] = *err_in;
  const bool in = g < n;
  unsigned long long my_entries = 0, my_visible = 0;
  float mu[3], s[3], q[4], sigma = 0.0f;
  if (in) {
    mu[0] = mean[g]; mu[1] = mean[n + g]; mu[2] = mean[2 * n + g];
    s[0] = scale[g]; s[1] = scale[n + g]; s[2] = scale[2 * n + g];
    q[0] = quat[g]; q[1] = quat[n + g]; q[2] = quat[2 * n + g]; q[3] = quat[3 * n + g];
    sigma = opacity[g];
  }
  for (int v = 0; v < n_views; ++v) {
    // with a totals stride every view has its own counters: flush the sums of the previous view
    if (totals_stride && v > 0) {
      block_add_totals(my_entries, my_visible, totals + (int64_t)(v - 1) * totals_stride);
      my_entries = my_visible = 0;
    }
    if (!in) continue;
    {
      const ViewDev& V = views[v];
      int64_t item = (int64_t)v * n + g;
      AssocOut A;
      associate(mu, s, q, sigma, V, op, lam_tab, edges, A);
      keys[item] = A.key;
      if (!A.visible) {
        counts[item] = 0;
        rects[item] = make_uint2(pack16(1, 0), pack16(1, 0));
        continue;
      }
      uint32_t cnt = (uint32_t)((A.hx1 / 2 - A.hx0 / 2 + 1) * (A.hy1 / 2 - A.hy0 / 2 + 1));
      counts[item] = cnt;
      rects[item] = make_uint2(pack16(A.hx0, A.hx1), pack16(A.hy0, A.hy1));
      my_entries += cnt;
      my_visible += 1;

      // ---- render record (radiometric) ----
      Frame3 F;
      canonical_frame(A, s, F);
      Record rec;
#pragma unroll
      for (int ii = 0; ii < 3; ++ii) {
        const float a0 = F.e1[0] * F.Wc[0 * 3 + ii] + F.e1[1] * F.Wc[1 * 3 + ii] + F.e1[2] * F.Wc[2 * 3 + ii];
        const float a1 = F.e2[0] * F.Wc[0 * 3 + ii] + F.e2[1] * F.Wc[1 * 3 + ii] + F.e2[2] * F.Wc[2 * 3 + ii];
        const float a2 = F.ou[0] * F.Wc[0 * 3 + ii] + F.ou[1] * F.Wc[1 * 3 + ii] + F.ou[2] * F.Wc[2 * 3 + ii];
        rec.g[0 * 3 + ii] = F.r * a0;
        rec.g[1 * 3 + ii] = F.r * a1;
        rec.g[2 * 3 + ii] = -a2;
      }
      rec.c0 = -0.72134752044448170f * F.r2;  // -log2(e) / 2 * r^2
      rec.lsig = __log2f(sigma);
      rec.c1 = F.r2;
      rec.qmax = op.lambda_mode == 1 ? op.kmax_fixed / F.r2 : INFINITY;
      if (kColour) {
        // the view-dependent colour (Eq. color's c_i): SH expansion in the
        // direction from the camera centre to the mean, + 1/2, clamped at 0
        float x, y, z;
        view_direction(V, mu, x, y, z);
        float acc[3] = {0.5f, 0.5f, 0.5f};
        add_band<0, kDeg>(n, g, sh, x, y, z, acc);
        add_band<1, kDeg>(n, g, sh, x, y, z, acc);
        add_band<2, kDeg>(n, g, sh, x, y, z, acc);
        add_band<3, kDeg>(n, g, sh, x, y, z, acc);
#pragma unroll
        for (int c = 0; c < 3; ++c) rec.rgb[c] = fmaxf(acc[c], 0.0f);
      } else {
        rec.rgb[0] = rec.rgb[1] = rec.rgb[2] = 0.0f;  // colour_kernel fills it in
      }
      if (op.splat) {
        // splat record: the mean's BEAP angles and the conic of the local
        // affine footprint C = J Sigma_c J^T + dilation (C^-1 = [a b; b c]),
        // log2(sigma), the mean's camera distance as the depth
        float tc, pc;
        beap_angles(A.mc[0], A.mc[1], A.mc[2], tc, pc);
        float c00, c01, c11;
        splat_cov(A.mc, A.A, s, c00, c01, c11);
        c00 += V.dil_t;
        c11 += V.dil_p;
        const float det = c00 * c11 - c01 * c01;
        const float idet = det > 0.0f ? 1.0f / det : 0.0f;
#pragma unroll
        for (int k = 0; k < 9; ++k) rec.g[k] = 0.0f;
        rec.g[0] = tc;
        rec.g[1] = pc;
        rec.g[2] = c11 * idet;
        rec.g[3] = -c01 * idet;
        rec.g[4] = c00 * idet;
        rec.c0 = 0.0f;
        rec.c1 = sqrtf(A.mc[0] * A.mc[0] + A.mc[1] * A.mc[1] + A.mc[2] * A.mc[2]);
        rec.qmax = INFINITY;
      }
      float4* dst = reinterpret_cast<float4*>(recs + item);
      const float4* src = reinterpret_cast<const float4*>(&rec);
      dst[0] = src[0]; dst[1] = src[1]; dst[2] = src[2]; dst[3] = src[3];
    }
  }
  block_add_totals(my_entries, my_visible,
                   totals + (totals_stride ? (int64_t)(n_views - 1) * totals_stride : 0));
}

// The colour of every visible (Gaussian, view) item of a batch, for a
// preprocess launched without it: one lane per item, the views of one
// Gaussian on neighbouring lanes, so their loads of its SH coefficients are
// the same addresses.  Kept out of the association kernel for batches of
// views: there the coefficients' registers would halve its occupancy.
template <int kDeg>
__global__ __launch_bounds__(256) void colour_kernel(int64_t n, int32_t n_views, const float* __restrict__ mean,
                                                     const float* __restrict__ sh, const ViewDev* __restrict__ views,
                                                     const uint32_t* __restrict__ counts,
                                                     Record* __restrict__ recs) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * n_views) return;
  const int64_t g = t / n_views;
  const int v = (int)(t - g * n_views);
  const int64_t item = (int64_t)v * n + g;
  if (counts[item] == 0u) return;
  const float mu[3] = {mean[g], mean[n + g], mean[2 * n + g]};
  float x, y, z;
  view_direction(views[v], mu, x, y, z);
  float acc[3] = {0.5f, 0.5f, 0.5f};
  add_band<0, kDeg>(n, g, sh, x, y, z, acc);
  add_band<1, kDeg>(n, g, sh, x, y, z, acc);
  add_band<2, kDeg>(n, g, sh, x, y, z, acc);
  add_band<3, kDeg>(n, g, sh, x, y, z, acc);
  Record* r = recs + item;
#pragma unroll
  for (int c = 0; c < 3; ++c) r->rgb[c] = fmaxf(acc[c], 0.0f);
}

void launch_colour(hipStream_t st, int64_t n, int32_t n_views, int32_t sh_degree, const float* mean,
                   const float* sh, const ViewDev* views, const uint32_t* counts, Record* recs) {
  if (n == 0 || n_views == 1 || sh_degree == 0) return;  // the association kernel gave the colour
  const dim3 grid((unsigned)((n * n_views + 255) / 256));
  switch (sh_degree) {
    case 1: hipLaunchKernelGGL(colour_kernel<1>, grid, dim3(256), 0, st, n, n_views, mean, sh, views, counts, recs); break;
    case 2: hipLaunchKernelGGL(colour_kernel<2>, grid, dim3(256), 0, st, n, n_views, mean, sh, views, counts, recs); break;
    default: hipLaunchKernelGGL(colour_kernel<3>, grid, dim3(256), 0, st, n, n_views, mean, sh, views, counts, recs); break;
  }
}

void launch_preprocess(hipStream_t st, int64_t n, int32_t n_views, int32_t sh_degree, const float* mean,
                       const float* scale, const float* quat, const float* opacity, const float* sh,
                       const ViewDev* views, const Opts& op, const float* lam_tab, const float* edges,
                       Record* recs, uint2* rects, uint32_t* keys, uint32_t* counts,
                       unsigned long long* totals, int totals_stride, const unsigned long long* err_in,
                       bool defer_colour) {
  if (n == 0) return;
  const dim3 grid((unsigned)((n + 255) / 256));
  // one view: the colour in the same pass; a batch of views: a second kernel
#define GEER_PRE(D)                                                                                               \
  do {                                                                                                            \
    if (n_views == 1 || D == 0) {                                                                                 \
      hipLaunchKernelGGL((preprocess_kernel<D, true>), grid, dim3(256), 0, st, n, n_views, mean, scale, quat,    \
                         opacity, sh, views, op, lam_tab, edges, recs, rects, keys, counts, totals, totals_stride, \
                         err_in);                                                                                 \
    } else {                                                                                                      \
      hipLaunchKernelGGL((preprocess_kernel<D, false>), grid, dim3(256), 0, st, n, n_views, mean, scale, quat,   \
                         opacity, sh, views, op, lam_tab, edges, recs, rects, keys, counts, totals, totals_stride, \
                         err_in);                                                                                 \
      if (!defer_colour)                                                                                          \
        launch_colour(st, n, n_views, D, mean, sh, views, counts, recs);                                          \
    }                                                                                                             \
  } while (0)
  switch (sh_degree) {
    case 0: GEER_PRE(0); break;
    case 1: GEER_PRE(1); break;
    case 2: GEER_PRE(2); break;
    default: GEER_PRE(3); break;
  }
#undef GEER_PRE
}

}  // namespace geer
