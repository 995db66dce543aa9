// L1 photometric loss over the valid rays of one view and its gradient, with
// a weight w (1 for a single view; 1/V for one view of a V-view batch whose
// loss is the mean of the views' losses):
//   L = w sum_{valid rays, channels} |rgb - target| / (3 n_valid),
//   dL/drgb = w sign(rgb - target) / (3 n_valid) on valid rays, 0 elsewhere.
// Block partial sums are reduced by one block in a fixed order, so the loss
// is deterministic.
#include <hip/hip_runtime.h>

#include <stdint.h>

namespace geer {

constexpr int kLossBlock = 256;
constexpr int kLossPer = 8;

__global__ __launch_bounds__(kLossBlock) void l1_partial_kernel(int64_t P, const float* __restrict__ rgb,
                                                                const float* __restrict__ target,
                                                                const uint8_t* __restrict__ mask,
                                                                float2* __restrict__ partial) {
  float s = 0.0f, c = 0.0f;
  const int64_t base = (int64_t)blockIdx.x * kLossBlock * kLossPer;
#pragma unroll
  for (int k = 0; k < kLossPer; ++k) {
    const int64_t p = base + (int64_t)k * kLossBlock + threadIdx.x;
    if (p < P && mask[p]) {
      c += 1.0f;
      s += fabsf(rgb[p] - target[p]) + fabsf(rgb[P + p] - target[P + p]) + fabsf(rgb[2 * P + p] - target[2 * P + p]);
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    s += __shfl_xor(s, off);
    c += __shfl_xor(c, off);
  }
  __shared__ float2 red[kLossBlock / 64];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = make_float2(s, c);
  __syncthreads();
  if (threadIdx.x == 0) {
    float2 t = red[0];
    for (int w = 1; w < kLossBlock / 64; ++w) { t.x += red[w].x; t.y += red[w].y; }
    partial[blockIdx.x] = t;
  }
}

__global__ __launch_bounds__(kLossBlock) void l1_finalize_kernel(int64_t nblocks, const float2* __restrict__ partial,
                                                                 double weight, float* __restrict__ loss,
                                                                 float* __restrict__ scale) {
  __shared__ double rs[kLossBlock], rc[kLossBlock];
  double s = 0.0, c = 0.0;
  for (int64_t b = threadIdx.x; b < nblocks; b += kLossBlock) {
    s += partial[b].x;
    c += partial[b].y;
  }
  rs[threadIdx.x] = s;
  rc[threadIdx.x] = c;
  __syncthreads();
  for (int w = kLossBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      rs[threadIdx.x] += rs[threadIdx.x + w];
      rc[threadIdx.x] += rc[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double n = rc[0];
    *loss = n > 0 ? (float)(weight * rs[0] / (3.0 * n)) : 0.0f;
    *scale = n > 0 ? (float)(weight / (3.0 * n)) : 0.0f;
  }
}

__global__ __launch_bounds__(kLossBlock) void l1_grad_kernel(int64_t P, const float* __restrict__ rgb,
                                                             const float* __restrict__ target,
                                                             const uint8_t* __restrict__ mask,
                                                             const float* __restrict__ scale,
                                                             float* __restrict__ dl) {
  const int64_t p = (int64_t)blockIdx.x * kLossBlock + threadIdx.x;
  if (p >= P) return;
  const float sc = mask[p] ? *scale : 0.0f;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float d = rgb[c * P + p] - target[c * P + p];
    dl[c * P + p] = d > 0.0f ? sc : (d < 0.0f ? -sc : 0.0f);
  }
}

int64_t l1_partial_count(int64_t P) { return (P + kLossBlock * kLossPer - 1) / (kLossBlock * kLossPer); }

// Sum of n floats in index order (one lane), e.g. the per-view losses of a batch.
__global__ void sum_f32_kernel(int n, const float* __restrict__ in, float* __restrict__ out) {
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += in[i];
    *out = (float)s;
  }
}

void launch_sum_f32(hipStream_t st, int n, const float* in, float* out) {
  hipLaunchKernelGGL(sum_f32_kernel, dim3(1), dim3(64), 0, st, n, in, out);
}

void launch_l1(hipStream_t st, int64_t P, const float* rgb, const float* target, const uint8_t* mask, float* dl,
               float* loss, float2* partial, float* scale, double weight) {
  const int64_t nb = l1_partial_count(P);
  if (nb > 0)
    hipLaunchKernelGGL(l1_partial_kernel, dim3((unsigned)nb), dim3(kLossBlock), 0, st, P, rgb, target, mask, partial);
  hipLaunchKernelGGL(l1_finalize_kernel, dim3(1), dim3(kLossBlock), 0, st, nb, (const float2*)partial, weight, loss,
                     scale);
  if (P > 0)
    hipLaunchKernelGGL(l1_grad_kernel, dim3((unsigned)((P + kLossBlock - 1) / kLossBlock)), dim3(kLossBlock), 0, st, P,
                       rgb, target, mask, (const float*)scale, dl);
}

}  // namespace geer
