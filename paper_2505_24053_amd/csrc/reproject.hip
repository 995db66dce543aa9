// Native camera-space output: resampling of a rendered BEAP image onto the
// native sensor of its camera (the inverse interpolation of App. E, used to
// evaluate in native pinhole / Kannala-Brandt image space).
//
// The sampling map is computed on the host in FP64 (tables.cpp) and cached
// per camera: for each native pixel its top-left BEAP neighbour and the two
// bilinear fractions, or a marker that no BEAP ray reaches it.  The kernel is
// a streaming gather: one lane per native pixel, the 16-byte map entry read
// coalesced, four neighbours per channel (mostly L2 hits: neighbouring native
// pixels share them), one coalesced write per channel.  It is bound by HBM:
// 16 B of map, C x 4 B written and about C x 4 B of image read per pixel.
#include <hip/hip_runtime.h>

#include <stdint.h>

namespace geer {

__global__ __launch_bounds__(256) void reproject_kernel(const int4* __restrict__ map, int64_t npix, int W, int H,
                                                        int C, const float* __restrict__ beap,
                                                        float* __restrict__ native, uint8_t* __restrict__ valid) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= npix) return;
  const int4 m = map[p];
  if (m.x < 0) {
    for (int c = 0; c < C; ++c) native[(int64_t)c * npix + p] = 0.0f;
    if (valid) valid[p] = 0;
    return;
  }
  const int i0 = m.x, j0 = m.y;
  const int i1 = min(i0 + 1, W - 1), j1 = min(j0 + 1, H - 1);
  const float fx = __int_as_float(m.z), fy = __int_as_float(m.w);
  const float w00 = (1.0f - fx) * (1.0f - fy), w10 = fx * (1.0f - fy);
  const float w01 = (1.0f - fx) * fy, w11 = fx * fy;
  const int64_t hw = (int64_t)W * H;
  const int64_t a00 = (int64_t)j0 * W + i0, a10 = (int64_t)j0 * W + i1;
  const int64_t a01 = (int64_t)j1 * W + i0, a11 = (int64_t)j1 * W + i1;
  for (int c = 0; c < C; ++c) {
    const float* b = beap + (int64_t)c * hw;
    const float v = fmaf(w11, b[a11], fmaf(w01, b[a01], fmaf(w10, b[a10], w00 * b[a00])));
    native[(int64_t)c * npix + p] = v;
  }
  if (valid) valid[p] = 1;
}

void launch_reproject(hipStream_t st, const int4* map, int64_t npix, int W, int H, int C, const float* beap,
                      float* native, uint8_t* valid) {
  if (npix <= 0) return;
  hipLaunchKernelGGL(reproject_kernel, dim3((unsigned)((npix + 255) / 256)), dim3(256), 0, st, map, npix, W, H, C,
                     beap, native, valid);
}

}  // namespace geer
