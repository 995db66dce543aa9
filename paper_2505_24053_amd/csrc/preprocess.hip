// Stage (a): per-Gaussian preprocessing and particle bounding frustum (PBF).
//
// One lane per Gaussian; the lane loops over the views of the batch so the
// scene is read from HBM once per batch.  For every (Gaussian, view) item it
// writes the half-tile rectangle, tile count and depth key (the association,
// bit-exact IEEE single arithmetic in a fixed order, no contraction) and the
// 64-byte render record (radiometric, free-form FP32).
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

namespace geer {

__device__ __forceinline__ float f_max(float a, float b) { return a > b ? a : b; }
__device__ __forceinline__ float f_min(float a, float b) { return a < b ? a : b; }

// first cell h in [0, n) whose closed interval [e[h], e[h+1]] can meet [a, ...]
__device__ __forceinline__ int first_cell(const float* __restrict__ e, int n, float a) {
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (e[mid + 1] >= a) hi = mid; else lo = mid + 1;
  }
  return lo;
}
// last cell h in [0, n) with e[h] <= b (-1 if none)
__device__ __forceinline__ int last_cell(const float* __restrict__ e, int n, float b) {
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (e[mid] <= b) lo = mid + 1; else hi = mid;
  }
  return lo - 1;
}

__device__ __forceinline__ float pad_of(float x) {
#pragma clang fp contract(off)
  float ax = fabsf(x);
  float s = 1.0f + ax;
  return s * 0x1p-14f;
}

__device__ __forceinline__ bool pieces_range(const float* __restrict__ e, int n, int np, const float* a,
                                             const float* b, int& c0, int& c1) {
  int lo = n, hi = -1;
  bool any = false;
  for (int p = 0; p < np; ++p) {
    int x0 = first_cell(e, n, a[p]);
    int x1 = last_cell(e, n, b[p]);
    if (x0 <= x1) {
      any = true;
      lo = min(lo, x0);
      hi = max(hi, x1);
    }
  }
  c0 = lo;
  c1 = hi;
  return any;
}

struct AssocOut {
  float A[9];   // Rc R
  float mc[3];  // camera-space mean
  float vou[3]; // S^-1 A^T mu_c = -o_u
  uint32_t key;
  int hx0, hx1, hy0, hy1;
  bool visible;
};

// The FP32 association.  Each statement is one IEEE single operation.
__device__ __noinline__ void associate(const float mu[3], const float s[3], const float q[4], float sigma,
                                       const ViewDev& V, const Opts& op, const float* __restrict__ lam_tab,
                                       const float* __restrict__ edges, AssocOut& o) {
#pragma clang fp contract(off)
  o.visible = false;
  o.hx0 = 1; o.hx1 = 0; o.hy0 = 1; o.hy1 = 0;

  float qq = q[0] * q[0];
  qq = qq + q[1] * q[1];
  qq = qq + q[2] * q[2];
  qq = qq + q[3] * q[3];
  float qn = __builtin_sqrtf(qq);
  float r = q[0] / qn, i = q[1] / qn, j = q[2] / qn, k = q[3] / qn;

  float xx = i * i, yy = j * j, zz = k * k, xy = i * j, xz = i * k, yz = j * k;
  float rx = r * i, ry = r * j, rz = r * k;
  float R[9];
  R[0] = 1.0f - 2.0f * (yy + zz); R[1] = 2.0f * (xy - rz);        R[2] = 2.0f * (xz + ry);
  R[3] = 2.0f * (xy + rz);        R[4] = 1.0f - 2.0f * (xx + zz); R[5] = 2.0f * (yz - rx);
  R[6] = 2.0f * (xz - ry);        R[7] = 2.0f * (yz + rx);        R[8] = 1.0f - 2.0f * (xx + yy);

  float M[9];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      float t0 = V.Rc[a * 3 + 0] * R[0 * 3 + b];
      float t1 = V.Rc[a * 3 + 1] * R[1 * 3 + b];
      float t2 = V.Rc[a * 3 + 2] * R[2 * 3 + b];
      float acc = t0 + t1;
      acc = acc + t2;
      o.A[a * 3 + b] = acc;
      M[a * 3 + b] = acc * s[b];
    }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float t0 = V.Rc[a * 3 + 0] * mu[0];
    float t1 = V.Rc[a * 3 + 1] * mu[1];
    float t2 = V.Rc[a * 3 + 2] * mu[2];
    float acc = t0 + t1;
    acc = acc + t2;
    o.mc[a] = acc + V.tc[a];
  }
  const float* mc = o.mc;
  {
    float d0 = mc[0] * mc[0], d1 = mc[1] * mc[1], d2 = mc[2] * mc[2];
    float dd = d0 + d1;
    dd = dd + d2;
    o.key = __float_as_uint(dd);
  }
  float ou2 = 0.0f;
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    float t0 = o.A[0 * 3 + b] * mc[0];
    float t1 = o.A[1 * 3 + b] * mc[1];
    float t2 = o.A[2 * 3 + b] * mc[2];
    float acc = t0 + t1;
    acc = acc + t2;
    float v = acc / s[b];
    o.vou[b] = v;
    float v2 = v * v;
    ou2 = b == 0 ? v2 : ou2 + v2;
  }
  if (ou2 < 9.0f) return;  // camera inside 3 sigma: culled
  if (!(qq > 0.0f)) return;
  if (!(sigma > op.alpha_min)) return;

  float L;
  if (op.lambda_mode == 1) {
    L = op.lam2_fixed;
  } else {
    int bkt = (int)(__float_as_uint(sigma) >> kLamShift) - op.lam_lo;
    bkt = bkt < 0 ? 0 : (bkt >= op.lam_n ? op.lam_n - 1 : bkt);
    L = lam_tab[bkt];
  }

#define DOT3(a, b) ((M[(a)*3 + 0] * M[(b)*3 + 0] + M[(a)*3 + 1] * M[(b)*3 + 1]) + M[(a)*3 + 2] * M[(b)*3 + 2])
  float S00 = DOT3(0, 0), S02 = DOT3(0, 2), S22 = DOT3(2, 2), S11 = DOT3(1, 1), S12 = DOT3(1, 2);
#undef DOT3
  float T00 = L * S00 - mc[0] * mc[0];
  float T02 = L * S02 - mc[0] * mc[2];
  float T22 = L * S22 - mc[2] * mc[2];
  float T11 = L * S11 - mc[1] * mc[1];
  float T12 = L * S12 - mc[1] * mc[2];

  const float* ex = edges + V.ex_off;
  const float* ey = edges + V.ey_off;

  int hx0, hx1;
  {
    float e0 = mc[0] * M[6] - mc[2] * M[0];
    float e1 = mc[0] * M[7] - mc[2] * M[1];
    float e2 = mc[0] * M[8] - mc[2] * M[2];
    float P = (e0 * e0 + e1 * e1) + e2 * e2;
    float c0 = M[1] * M[8] - M[2] * M[7];
    float c1 = M[2] * M[6] - M[0] * M[8];
    float c2 = M[0] * M[7] - M[1] * M[6];
    float Qd = (c0 * c0 + c1 * c1) + c2 * c2;
    float D = P - L * Qd;
    bool full = !(D > P * 0x1p-12f);
    if (full) {
      hx0 = 0;
      hx1 = V.nhx - 1;
    } else {
      float sd = __builtin_sqrtf(L * D);
      float qv = T02 >= 0.0f ? T02 + sd : T02 - sd;
      float rs[2] = {qv, T00}, rk[2] = {T22, qv};
      float cand[4];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        float ss = rs[t], kk = rk[t];
        if (kk < 0.0f) { ss = -ss; kk = -kk; }
        float rr = __builtin_sqrtf(ss * ss + kk * kk);
        float kr = kk + rr;
        cand[2 * t + 0] = ss / kr;
        cand[2 * t + 1] = -(kr / ss);
      }
      float rho = __builtin_sqrtf(mc[0] * mc[0] + mc[2] * mc[2]);
      float tmu = mc[2] >= 0.0f ? mc[0] / (mc[2] + rho) : (rho - mc[2]) / mc[0];
      bool has_lo = false, has_hi = false;
      float lo = 0.0f, hi = 0.0f, cmin = cand[0], cmax = cand[0];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        float c = cand[t];
        cmin = f_min(cmin, c);
        cmax = f_max(cmax, c);
        if (c < tmu) { lo = has_lo ? f_max(lo, c) : c; has_lo = true; }
        if (c > tmu) { hi = has_hi ? f_min(hi, c) : c; has_hi = true; }
      }
      float a[2], b[2];
      int np;
      if (has_lo && has_hi) {
        a[0] = lo - pad_of(lo); b[0] = hi + pad_of(hi); np = 1;
      } else {
        a[0] = -INFINITY; b[0] = cmin + pad_of(cmin);
        a[1] = cmax - pad_of(cmax); b[1] = INFINITY; np = 2;
      }
      if (!pieces_range(ex, V.nhx, np, a, b, hx0, hx1)) return;
    }
  }
  int hy0, hy1;
  {
    float e0 = mc[1] * M[6] - mc[2] * M[3];
    float e1 = mc[1] * M[7] - mc[2] * M[4];
    float e2 = mc[1] * M[8] - mc[2] * M[5];
    float P = (e0 * e0 + e1 * e1) + e2 * e2;
    float c0 = M[4] * M[8] - M[5] * M[7];
    float c1 = M[5] * M[6] - M[3] * M[8];
    float c2 = M[3] * M[7] - M[4] * M[6];
    float Qd = (c0 * c0 + c1 * c1) + c2 * c2;
    float D = P - L * Qd;
    float tz = (mc[2] * mc[2]) * 0x1p-12f;
    bool full = !(D > P * 0x1p-12f) || !(T22 < -tz || T22 > tz);
    if (full) {
      hy0 = 0;
      hy1 = V.nhy - 1;
    } else {
      float sd = __builtin_sqrtf(L * D);
      float qv = T12 >= 0.0f ? T12 + sd : T12 - sd;
      float r1 = qv / T22, r2 = T11 / qv;
      float cmin = f_min(r1, r2), cmax = f_max(r1, r2);
      float a[2], b[2];
      int np;
      if (T22 < 0.0f) {
        a[0] = cmin - pad_of(cmin); b[0] = cmax + pad_of(cmax); np = 1;
      } else {
        a[0] = -INFINITY; b[0] = cmin + pad_of(cmin);
        a[1] = cmax - pad_of(cmax); b[1] = INFINITY; np = 2;
      }
      if (!pieces_range(ey, V.nhy, np, a, b, hy0, hy1)) return;
    }
  }
  o.hx0 = hx0; o.hx1 = hx1; o.hy0 = hy0; o.hy1 = hy1;
  o.visible = true;
}

// Real SH (degree <= 3) at unit direction v, 3DGS sign convention; coef rows
// (k*3 + c) of an SoA array with stride n.
__device__ __forceinline__ void sh_color(int deg, const float v[3], const float* __restrict__ sh, int64_t n,
                                         int64_t g, float rgb[3]) {
  const float C0 = 0.28209479177387814f, C1 = 0.4886025119029199f;
  const float C2[5] = {1.0925484305920792f, -1.0925484305920792f, 0.31539156525252005f,
                       -1.0925484305920792f, 0.5462742152960396f};
  const float C3[7] = {-0.5900435899266435f, 2.890611442640554f, -0.4570457994644658f, 0.3731763325901154f,
                       -0.4570457994644658f, 1.445305721320277f, -0.5900435899266435f};
  float B[16];
  B[0] = C0;
  int K = 1;
  if (deg > 0) {
    float x = v[0], y = v[1], z = v[2];
    B[1] = -C1 * y; B[2] = C1 * z; B[3] = -C1 * x;
    K = 4;
    if (deg > 1) {
      float xx = x * x, yy = y * y, zz = z * z;
      B[4] = C2[0] * x * y;
      B[5] = C2[1] * y * z;
      B[6] = C2[2] * (2.0f * zz - xx - yy);
      B[7] = C2[3] * x * z;
      B[8] = C2[4] * (xx - yy);
      K = 9;
      if (deg > 2) {
        B[9] = C3[0] * y * (3.0f * xx - yy);
        B[10] = C3[1] * x * y * z;
        B[11] = C3[2] * y * (4.0f * zz - xx - yy);
        B[12] = C3[3] * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
        B[13] = C3[4] * x * (4.0f * zz - xx - yy);
        B[14] = C3[5] * z * (xx - yy);
        B[15] = C3[6] * x * (xx - 3.0f * yy);
        K = 16;
      }
    }
  }
  float acc[3] = {0.5f, 0.5f, 0.5f};
  for (int kk = 0; kk < K; ++kk)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[c] = fmaf(B[kk], sh[(int64_t)(kk * 3 + c) * n + g], acc[c]);
#pragma unroll
  for (int c = 0; c < 3; ++c) rgb[c] = fmaxf(acc[c], 0.0f);
}

// Orthonormal pair (e1, e2) completing n, built in the frame where n's
// largest component plays the role of z (Duff et al. 2017 branchless basis),
// so that every entry is accurate relative to n's small components.
__device__ __forceinline__ void ortho_basis(const float n[3], float e1[3], float e2[3]) {
  float ax = fabsf(n[0]), ay = fabsf(n[1]), az = fabsf(n[2]);
  int k = (ax > ay) ? (ax > az ? 0 : 2) : (ay > az ? 1 : 2);
  int a = k == 0 ? 1 : 0;
  int b = k == 2 ? 1 : 2;
  float x = n[a], y = n[b], z = n[k];
  float sg = copysignf(1.0f, z);
  float p = -1.0f / (sg + z);
  float q = x * y * p;
  float u[3] = {1.0f + sg * x * x * p, sg * q, -sg * x};
  float w[3] = {q, sg + y * y * p, -y};
  e1[a] = u[0]; e1[b] = u[1]; e1[k] = u[2];
  e2[a] = w[0]; e2[b] = w[1]; e2[k] = w[2];
}

__global__ __launch_bounds__(256) void preprocess_kernel(
    int64_t n, int32_t n_views, int32_t sh_degree, const float* __restrict__ mean, const float* __restrict__ scale,
    const float* __restrict__ quat, const float* __restrict__ opacity, const float* __restrict__ sh,
    const ViewDev* __restrict__ views, Opts op, const float* __restrict__ lam_tab,
    const float* __restrict__ edges, Record* __restrict__ recs, uint2* __restrict__ rects,
    uint32_t* __restrict__ keys, uint32_t* __restrict__ counts, unsigned long long* __restrict__ totals) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long my_entries = 0, my_visible = 0;
  if (g < n) {
    float mu[3] = {mean[g], mean[n + g], mean[2 * n + g]};
    float s[3] = {scale[g], scale[n + g], scale[2 * n + g]};
    float q[4] = {quat[g], quat[n + g], quat[2 * n + g], quat[3 * n + g]};
    float sigma = opacity[g];
    for (int v = 0; v < n_views; ++v) {
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
      float Wc[9];  // S^-1 A^T: Wc[k][i] = A[i][k] / s_k
#pragma unroll
      for (int kk = 0; kk < 3; ++kk)
#pragma unroll
        for (int ii = 0; ii < 3; ++ii) Wc[kk * 3 + ii] = A.A[ii * 3 + kk] / s[kk];
      float ou[3] = {-A.vou[0], -A.vou[1], -A.vou[2]};
      float r2 = ou[0] * ou[0] + ou[1] * ou[1] + ou[2] * ou[2];
      float rinv = rsqrtf(r2);
      float rr = r2 * rinv;
      float nn[3] = {ou[0] * rinv, ou[1] * rinv, ou[2] * rinv};
      float e1[3], e2[3];
      ortho_basis(nn, e1, e2);
      Record rec;
#pragma unroll
      for (int ii = 0; ii < 3; ++ii) {
        float a0 = e1[0] * Wc[0 * 3 + ii] + e1[1] * Wc[1 * 3 + ii] + e1[2] * Wc[2 * 3 + ii];
        float a1 = e2[0] * Wc[0 * 3 + ii] + e2[1] * Wc[1 * 3 + ii] + e2[2] * Wc[2 * 3 + ii];
        float a2 = ou[0] * Wc[0 * 3 + ii] + ou[1] * Wc[1 * 3 + ii] + ou[2] * Wc[2 * 3 + ii];
        rec.g[0 * 3 + ii] = rr * a0;
        rec.g[1 * 3 + ii] = rr * a1;
        rec.g[2 * 3 + ii] = -a2;
      }
      rec.c0 = -0.72134752044448170f * r2;  // -log2(e) / 2 * r^2
      rec.lsig = __log2f(sigma);
      rec.c1 = r2;
      rec.qmax = op.lambda_mode == 1 ? op.kmax_fixed / r2 : INFINITY;
      float dv[3] = {mu[0] - V.campos[0], mu[1] - V.campos[1], mu[2] - V.campos[2]};
      float dinv = rsqrtf(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
      float vdir[3] = {dv[0] * dinv, dv[1] * dinv, dv[2] * dinv};
      sh_color(sh_degree, vdir, sh, n, g, rec.rgb);
      float4* dst = reinterpret_cast<float4*>(recs + item);
      const float4* src = reinterpret_cast<const float4*>(&rec);
      dst[0] = src[0]; dst[1] = src[1]; dst[2] = src[2]; dst[3] = src[3];
    }
  }
  // block totals: association entries and visible items
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    my_entries += __shfl_xor(my_entries, off);
    my_visible += __shfl_xor(my_visible, off);
  }
  __shared__ unsigned long long red[2][4];
  int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) { red[0][wv] = my_entries; red[1][wv] = my_visible; }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long e = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    unsigned long long vv = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    if (e) atomicAdd(&totals[0], e);
    if (vv) atomicAdd(&totals[1], vv);
  }
}

void launch_preprocess(hipStream_t st, int64_t n, int32_t n_views, int32_t sh_degree, const float* mean,
                       const float* scale, const float* quat, const float* opacity, const float* sh,
                       const ViewDev* views, const Opts& op, const float* lam_tab, const float* edges,
                       Record* recs, uint2* rects, uint32_t* keys, uint32_t* counts,
                       unsigned long long* totals) {
  if (n == 0) return;
  int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(preprocess_kernel, dim3((unsigned)blocks), dim3(256), 0, st, n, n_views, sh_degree, mean,
                     scale, quat, opacity, sh, views, op, lam_tab, edges, recs, rects, keys, counts, totals);
}

}  // namespace geer
