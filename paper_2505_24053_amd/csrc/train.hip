// Training step around the renderer (Alg. "3DGEER Initialization and Training
// Framework": the Adam step on the loss gradient, and the periodic
// refinement that adds and removes Gaussians, driven by view-space mean
// gradients instead of screen-space ones).
//
// Parameters are kept raw, as the optimiser sees them: mean, log scale,
// unnormalised quaternion, opacity logit, SH coefficients.  The renderer
// reads the activated scale exp(log s) and opacity sigmoid(logit), which the
// Adam kernel writes after every update, so the scene it renders is always
// the one the optimiser holds.  Both kernels are HBM-bound streaming passes,
// one lane per Gaussian, every parameter row read and written coalesced.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "geer_common.h"

namespace geer {

// Parameter rows of a scene with K SH coefficients per channel: mean 3, log
// scale 3, quaternion 4, opacity logit 1, SH 3K (row r at raw[r n ...]).

// The renderer's activated scale and opacity from the raw rows.
__global__ __launch_bounds__(256) void activate_kernel(int64_t n, const float* __restrict__ raw,
                                                       float* __restrict__ scale_out, float* __restrict__ opac_out) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  for (int a = 0; a < 3; ++a) scale_out[(int64_t)a * n + g] = expf(raw[(int64_t)(3 + a) * n + g]);
  opac_out[g] = 1.0f / (1.0f + expf(-raw[10 * n + g]));
}

void launch_activate(hipStream_t st, int64_t n, const float* raw, float* scale_out, float* opac_out) {
  if (n > 0)
    hipLaunchKernelGGL(activate_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, raw, scale_out,
                       opac_out);
}

// One fused Adam step.  grad rows are the renderer's gradients with respect
// to the activated parameters (linear scale, opacity); they are chained
// through the activations (d/dlog s = s d/ds, d/dlogit = sigma (1 - sigma)
// d/dsigma), moments updated (m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2)
// and the parameter moved by lr m_hat / (sqrt(v_hat) + eps) with the bias
// corrections c1 = 1 / (1 - b1^t), c2 = 1 / (1 - b2^t).  Gaussians with an
// all-zero gradient (not seen by any ray) keep their moments' decay too, as
// Adam does.  The norm of the mean gradient is added to accum and 1 to
// count when it is non-zero (the densification statistics).
template <int K>
__global__ __launch_bounds__(256) void adam_kernel(int64_t n, float* __restrict__ raw, const float* __restrict__ g_mean,
                                                   const float* __restrict__ g_scale, const float* __restrict__ g_quat,
                                                   const float* __restrict__ g_opac, const float* __restrict__ g_sh,
                                                   float* __restrict__ mom1, float* __restrict__ mom2,
                                                   float* __restrict__ scale_out, float* __restrict__ opac_out,
                                                   float* __restrict__ accum, float* __restrict__ count, AdamParams ap) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  constexpr int NR = 11 + 3 * K;
  float gm2 = 0.0f;
#pragma unroll 1
  for (int r = 0; r < NR; ++r) {
    const int64_t i = (int64_t)r * n + g;
    float p = raw[i];
    float gr, lr;
    if (r < 3) {
      gr = g_mean[(int64_t)r * n + g];
      gm2 = fmaf(gr, gr, gm2);
      lr = ap.lr[0];
    } else if (r < 6) {
      gr = g_scale[(int64_t)(r - 3) * n + g] * expf(p);  // d/dlog s = s d/ds
      lr = ap.lr[1];
    } else if (r < 10) {
      gr = g_quat[(int64_t)(r - 6) * n + g];
      lr = ap.lr[2];
    } else if (r == 10) {
      const float sg = 1.0f / (1.0f + expf(-p));
      gr = g_opac[g] * sg * (1.0f - sg);  // d/dlogit = sigma (1 - sigma) d/dsigma
      lr = ap.lr[3];
    } else {
      gr = g_sh[(int64_t)(r - 11) * n + g];
      lr = ap.lr[4];
    }
    const float m = fmaf(ap.b1, mom1[i], ap.omb1 * gr);
    const float v = fmaf(ap.b2, mom2[i], ap.omb2 * gr * gr);
    mom1[i] = m;
    mom2[i] = v;
    p -= lr * (m * ap.c1) / (sqrtf(v * ap.c2) + ap.eps);
    raw[i] = p;
    if (r >= 3 && r < 6) scale_out[(int64_t)(r - 3) * n + g] = expf(p);
    if (r == 10) opac_out[g] = 1.0f / (1.0f + expf(-p));
  }
  if (accum && gm2 > 0.0f) {
    accum[g] += sqrtf(gm2);
    count[g] += 1.0f;
  }
}

// Refinement decisions (3DGS-style) from the statistics, per Gaussian:
// pruned when its opacity logit is below prune_logit; else, when the mean
// gradient norm averaged over the steps that saw it reaches grad_threshold,
// cloned (two copies) if its largest log scale is at most split_log_scale,
// split (two smaller ones) otherwise.  Output count per Gaussian: 0, 1 or 2.
__global__ __launch_bounds__(256) void densify_count_kernel(int64_t n, const float* __restrict__ raw,
                                                            const float* __restrict__ accum,
                                                            const float* __restrict__ count, DensifyParams dp,
                                                            uint32_t* __restrict__ nout, uint32_t* __restrict__ kind) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  uint32_t k = 0u;  // 0 prune, 1 keep, 2 clone, 3 split
  if (!(raw[10 * n + g] < dp.prune_logit)) {
    k = 1u;
    const float c = count[g];
    if (c > 0.0f && accum[g] / c >= dp.grad_threshold) {
      const float ls = fmaxf(fmaxf(raw[3 * n + g], raw[4 * n + g]), raw[5 * n + g]);
      k = ls > dp.split_log_scale ? 3u : 2u;
    }
  }
  kind[g] = k;
  nout[g] = k == 0u ? 0u : (k == 1u ? 1u : 2u);
}

// Writes the refined scene at the scanned offsets.  A kept Gaussian is
// copied with its moments; a clone is copied twice, the copy with zero
// moments; a split Gaussian becomes two, each with mean mu + R S xi (xi the
// caller's standard normal draws, noise[c * 3 + a][g] for child c and axis a),
// log scale reduced by log(1.6), the other parameters copied, zero moments.
// The statistics of every output start at zero.
template <int K>
__global__ __launch_bounds__(256) void densify_apply_kernel(int64_t n, const float* __restrict__ raw,
                                                            const float* __restrict__ mom1,
                                                            const float* __restrict__ mom2,
                                                            const uint32_t* __restrict__ kind,
                                                            const uint32_t* __restrict__ offs,
                                                            const float* __restrict__ noise, int64_t n_out,
                                                            float* __restrict__ raw_o, float* __restrict__ mom1_o,
                                                            float* __restrict__ mom2_o, float* __restrict__ scale_o,
                                                            float* __restrict__ opac_o, float* __restrict__ accum_o,
                                                            float* __restrict__ count_o, float split_shrink) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const uint32_t k = kind[g];
  if (k == 0u) return;
  constexpr int NR = 11 + 3 * K;
  const int64_t o0 = offs[g];
  const int nc = k == 1u ? 1 : 2;
  // split children: mean offsets R S xi
  float off[2][3] = {{0, 0, 0}, {0, 0, 0}};
  if (k == 3u) {
    float q[4] = {raw[6 * n + g], raw[7 * n + g], raw[8 * n + g], raw[9 * n + g]};
    const float qn = sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const float r = q[0] / qn, i = q[1] / qn, j = q[2] / qn, kk = q[3] / qn;
    const float R[9] = {1.0f - 2.0f * (j * j + kk * kk), 2.0f * (i * j - r * kk), 2.0f * (i * kk + r * j),
                        2.0f * (i * j + r * kk), 1.0f - 2.0f * (i * i + kk * kk), 2.0f * (j * kk - r * i),
                        2.0f * (i * kk - r * j), 2.0f * (j * kk + r * i), 1.0f - 2.0f * (i * i + j * j)};
    const float s[3] = {expf(raw[3 * n + g]), expf(raw[4 * n + g]), expf(raw[5 * n + g])};
    for (int c = 0; c < 2; ++c) {
      const float xi0 = s[0] * noise[(int64_t)(c * 3 + 0) * n + g];
      const float xi1 = s[1] * noise[(int64_t)(c * 3 + 1) * n + g];
      const float xi2 = s[2] * noise[(int64_t)(c * 3 + 2) * n + g];
      for (int a = 0; a < 3; ++a) off[c][a] = R[a * 3 + 0] * xi0 + R[a * 3 + 1] * xi1 + R[a * 3 + 2] * xi2;
    }
  }
  for (int c = 0; c < nc; ++c) {
    const int64_t o = o0 + c;
    const bool fresh = (k == 2u && c == 1) || k == 3u;  // new Gaussians start with zero moments
#pragma unroll 1
    for (int r = 0; r < NR; ++r) {
      float p = raw[(int64_t)r * n + g];
      if (k == 3u && r < 3) p += off[c][r];
      if (k == 3u && r >= 3 && r < 6) p -= split_shrink;
      raw_o[(int64_t)r * n_out + o] = p;
      mom1_o[(int64_t)r * n_out + o] = fresh ? 0.0f : mom1[(int64_t)r * n + g];
      mom2_o[(int64_t)r * n_out + o] = fresh ? 0.0f : mom2[(int64_t)r * n + g];
      if (r >= 3 && r < 6) scale_o[(int64_t)(r - 3) * n_out + o] = expf(p);
      if (r == 10) opac_o[o] = 1.0f / (1.0f + expf(-p));
    }
    accum_o[o] = 0.0f;
    count_o[o] = 0.0f;
  }
}

void launch_adam(hipStream_t st, int64_t n, int sh_degree, float* raw, const float* g_mean, const float* g_scale,
                 const float* g_quat, const float* g_opac, const float* g_sh, float* m, float* v, float* scale_out,
                 float* opac_out, float* accum, float* count, const AdamParams& ap) {
  if (n <= 0) return;
  const dim3 grid((unsigned)((n + 255) / 256));
#define GEER_ADAM(D)                                                                                              \
  hipLaunchKernelGGL(adam_kernel<(D + 1) * (D + 1)>, grid, dim3(256), 0, st, n, raw, g_mean, g_scale, g_quat, g_opac, \
                     g_sh, m, v, scale_out, opac_out, accum, count, ap)
  switch (sh_degree) {
    case 0: GEER_ADAM(0); break;
    case 1: GEER_ADAM(1); break;
    case 2: GEER_ADAM(2); break;
    default: GEER_ADAM(3); break;
  }
#undef GEER_ADAM
}

void launch_densify_count(hipStream_t st, int64_t n, const float* raw, const float* accum, const float* count,
                          const DensifyParams& dp, uint32_t* nout, uint32_t* kind) {
  if (n <= 0) return;
  hipLaunchKernelGGL(densify_count_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, raw, accum, count,
                     dp, nout, kind);
}

void launch_densify_apply(hipStream_t st, int64_t n, int sh_degree, const float* raw, const float* m, const float* v,
                          const uint32_t* kind, const uint32_t* offs, const float* noise, int64_t n_out, float* raw_o,
                          float* m_o, float* v_o, float* scale_o, float* opac_o, float* accum_o, float* count_o,
                          float split_shrink) {
  if (n <= 0) return;
  const dim3 grid((unsigned)((n + 255) / 256));
#define GEER_DA(D)                                                                                                 \
  hipLaunchKernelGGL(densify_apply_kernel<(D + 1) * (D + 1)>, grid, dim3(256), 0, st, n, raw, m, v, kind, offs, noise, \
                     n_out, raw_o, m_o, v_o, scale_o, opac_o, accum_o, count_o, split_shrink)
  switch (sh_degree) {
    case 0: GEER_DA(0); break;
    case 1: GEER_DA(1); break;
    case 2: GEER_DA(2); break;
    default: GEER_DA(3); break;
  }
#undef GEER_DA
}

}  // namespace geer
