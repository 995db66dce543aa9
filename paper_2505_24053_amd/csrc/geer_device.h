// Device functions shared by the forward and the backward kernels of libgeer:
// the bit-exact FP32 association, the render record, the SH basis and the
// per-pair evaluation.  The backward recomputes with these same functions so
// that every decision it replays is bit-identical to the forward's.
#pragma once
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

// Union of the cells met by np <= 2 intervals [a[p], b[p]] (the loop runs
// over the fixed maximum so that a and b stay in registers).
__device__ __forceinline__ bool pieces_range(const float* __restrict__ e, int n, int np, const float* a,
                                             const float* b, int& c0, int& c1) {
  int lo = n, hi = -1;
  bool any = false;
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    if (p >= np) break;
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

// Cells of the edge table e (n cells) met by the angle interval [lo, hi] of
// theta (e holds tan(theta / 2)) or of phi (e holds tan(phi)); an interval
// wider than a turn, or reaching past -pi / pi, wraps into two pieces.
__device__ __forceinline__ bool angle_cells(const float* __restrict__ e, int n, float lo, float hi, bool half,
                                            int& c0, int& c1) {
  const float PI = 3.14159265358979f;
  float a[2], b[2];
  int np = 1;
  if (half) {
    if (hi - lo >= 2.0f * PI) {
      c0 = 0;
      c1 = n - 1;
      return true;
    }
    a[0] = lo <= -PI ? -INFINITY : tanf(0.5f * lo);
    b[0] = hi >= PI ? INFINITY : tanf(0.5f * hi);
    if (lo < -PI) {  // the part beyond -pi comes back from +pi
      a[1] = tanf(0.5f * (lo + 2.0f * PI));
      b[1] = INFINITY;
      np = 2;
    } else if (hi > PI) {
      a[1] = -INFINITY;
      b[1] = tanf(0.5f * (hi - 2.0f * PI));
      np = 2;
    }
  } else {
    const float H = 0.5f * PI;
    a[0] = lo <= -H ? -INFINITY : tanf(lo);
    b[0] = hi >= H ? INFINITY : tanf(hi);
  }
  return pieces_range(e, n, np, a, b, c0, c1);
}

// BEAP angles of a camera-space point: theta = atan2(x, z), phi = atan(y / z).
__device__ __forceinline__ void beap_angles(float x, float y, float z, float& th, float& ph) {
  th = atan2f(x, z);
  ph = z != 0.0f ? atanf(y / z) : (y > 0.0f ? 1.57079632679f : (y < 0.0f ? -1.57079632679f : 0.0f));
}

// Half-tile rectangle of a projected-footprint association (kAssocEWA ..
// kAssocUTSnug): centre and 2x2 angular covariance C of the Gaussian
// (mean mc, camera-space factor M, Sigma_c = M M^T) in BEAP angles --
//   EWA: the angles of the mean and J Sigma_c J^T, J the Jacobian of the
//        angles at the mean (the local affine approximation);
//   UT:  the seven sigma points mc and mc +- sqrt(3) m_k (m_k the columns of
//        M) projected exactly, with the unscented weights of alpha = 1,
//        beta = 2, kappa = 0 (mean: 1/6 each off-centre point; covariance:
//        2 for the centre, 1/6 each other), theta unwrapped around the
//        centre point's;
// then the box centre +- sqrt(L) sqrt(lambda_max(C)) (square) or
// +- sqrt(L C_00), sqrt(L C_11) (snug), with L the same lambda^2 as the PBF.
__device__ __forceinline__ bool footprint_cells(int mode, const float mc[3], const float M[9], float L,
                                                const ViewDev& V, const float* __restrict__ edges, int& hx0,
                                                int& hx1, int& hy0, int& hy1) {
  const float PI = 3.14159265358979f;
  float tc, pc, c00, c01, c11;
  if (mode == kAssocEWA || mode == kAssocEWASnug) {
    beap_angles(mc[0], mc[1], mc[2], tc, pc);
    const float rxz = mc[0] * mc[0] + mc[2] * mc[2], ryz = mc[1] * mc[1] + mc[2] * mc[2];
    // d theta = (z dx - x dz) / (x^2 + z^2), d phi = (z dy - y dz) / (y^2 + z^2)
    const float jt[3] = {mc[2] / rxz, 0.0f, -mc[0] / rxz};
    const float jp[3] = {0.0f, mc[2] / ryz, -mc[1] / ryz};
    float vt[3], vp[3];  // J_t M and J_p M (rows of J M)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      vt[k] = jt[0] * M[0 * 3 + k] + jt[1] * M[1 * 3 + k] + jt[2] * M[2 * 3 + k];
      vp[k] = jp[0] * M[0 * 3 + k] + jp[1] * M[1 * 3 + k] + jp[2] * M[2 * 3 + k];
    }
    c00 = vt[0] * vt[0] + vt[1] * vt[1] + vt[2] * vt[2];
    c01 = vt[0] * vp[0] + vt[1] * vp[1] + vt[2] * vp[2];
    c11 = vp[0] * vp[0] + vp[1] * vp[1] + vp[2] * vp[2];
  } else {
    float t0, p0;
    beap_angles(mc[0], mc[1], mc[2], t0, p0);
    float ts[6], ps[6];
    const float sq3 = 1.7320508075688772f;
    float mt = 0.0f, mp = 0.0f;
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      const int k = i >> 1;
      const float sg = (i & 1) ? -sq3 : sq3;
      float t, p;
      beap_angles(mc[0] + sg * M[0 * 3 + k], mc[1] + sg * M[1 * 3 + k], mc[2] + sg * M[2 * 3 + k], t, p);
      float dt = t - t0;
      dt = dt > PI ? dt - 2.0f * PI : (dt < -PI ? dt + 2.0f * PI : dt);
      ts[i] = t0 + dt;
      ps[i] = p;
      mt += ts[i] * (1.0f / 6.0f);
      mp += p * (1.0f / 6.0f);
    }
    tc = mt;
    pc = mp;
    c00 = 2.0f * (t0 - mt) * (t0 - mt);
    c01 = 2.0f * (t0 - mt) * (p0 - mp);
    c11 = 2.0f * (p0 - mp) * (p0 - mp);
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      const float a = ts[i] - mt, b = ps[i] - mp;
      c00 += (1.0f / 6.0f) * a * a;
      c01 += (1.0f / 6.0f) * a * b;
      c11 += (1.0f / 6.0f) * b * b;
    }
  }
  float rt, rp;
  if (mode == kAssocEWASnug || mode == kAssocUTSnug) {
    rt = sqrtf(L * c00);
    rp = sqrtf(L * c11);
  } else {
    const float mid = 0.5f * (c00 + c11);
    const float dd = sqrtf(fmaxf(0.25f * (c00 - c11) * (c00 - c11) + c01 * c01, 0.0f));
    rt = rp = sqrtf(L * (mid + dd));
  }
  if (!(rt == rt) || !(rp == rp)) return false;  // degenerate projection (NaN)
  const bool okx = angle_cells(edges + V.ex_off, V.nhx, tc - rt, tc + rt, true, hx0, hx1);
  const bool oky = angle_cells(edges + V.ey_off, V.nhy, pc - rp, pc + rp, false, hy0, hy1);
  return okx && oky;
}

// EWA covariance of the BEAP angles at the camera-space mean mc for the
// camera-space axes A = Rc R and scales s (Sigma_c = A S S A^T): J Sigma_c J^T
// with J the Jacobian of (atan2(x, z), atan(y / z)) at mc.
__device__ __forceinline__ void splat_cov(const float mc[3], const float A[9], const float s[3], float& c00,
                                          float& c01, float& c11) {
  const float rxz = mc[0] * mc[0] + mc[2] * mc[2], ryz = mc[1] * mc[1] + mc[2] * mc[2];
  const float jt[3] = {mc[2] / rxz, 0.0f, -mc[0] / rxz};
  const float jp[3] = {0.0f, mc[2] / ryz, -mc[1] / ryz};
  float vt[3], vp[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    vt[k] = (jt[0] * A[0 * 3 + k] + jt[2] * A[2 * 3 + k]) * s[k];
    vp[k] = (jp[1] * A[1 * 3 + k] + jp[2] * A[2 * 3 + k]) * s[k];
  }
  c00 = vt[0] * vt[0] + vt[1] * vt[1] + vt[2] * vt[2];
  c01 = vt[0] * vp[0] + vt[1] * vp[1] + vt[2] * vp[2];
  c11 = vp[0] * vp[0] + vp[1] * vp[1] + vp[2] * vp[2];
}

struct AssocOut {
  float R[9];   // local-to-world rotation of the unit quaternion
  float qh[4];  // unit quaternion
  float qn;     // |q|
  float A[9];   // Rc R
  float mc[3];  // camera-space mean
  float vou[3]; // S^-1 A^T mu_c = -o_u
  uint32_t key;
  int hx0, hx1, hy0, hy1;
  bool visible;
};

// The FP32 association.  Each statement is one IEEE single operation.
__device__ __forceinline__ void associate(const float mu[3], const float s[3], const float q[4], float sigma,
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
  o.qn = qn;
  o.qh[0] = r; o.qh[1] = i; o.qh[2] = j; o.qh[3] = k;

  float xx = i * i, yy = j * j, zz = k * k, xy = i * j, xz = i * k, yz = j * k;
  float rx = r * i, ry = r * j, rz = r * k;
  float* R = o.R;
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
  if (op.assoc != kAssocPBF) {
    int hy0, hy1;
    if (!footprint_cells(op.assoc, mc, M, L, V, edges, hx0, hx1, hy0, hy1)) return;
    o.hx0 = hx0; o.hx1 = hx1; o.hy0 = hy0; o.hy1 = hy1;
    o.visible = true;
    return;
  }
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

// SH basis (degree <= 3) at the unit direction v with the 3DGS sign
// convention; optionally its gradient with respect to (x, y, z).  Returns K.
__device__ __forceinline__ int sh_basis(int deg, const float v[3], float B[16], float (*dB)[3]) {
  const float C0 = 0.28209479177387814f, C1 = 0.4886025119029199f;
  const float C2[5] = {1.0925484305920792f, -1.0925484305920792f, 0.31539156525252005f,
                       -1.0925484305920792f, 0.5462742152960396f};
  const float C3[7] = {-0.5900435899266435f, 2.890611442640554f, -0.4570457994644658f, 0.3731763325901154f,
                       -0.4570457994644658f, 1.445305721320277f, -0.5900435899266435f};
  const float x = v[0], y = v[1], z = v[2];
  B[0] = C0;
  if (dB) { dB[0][0] = 0; dB[0][1] = 0; dB[0][2] = 0; }
  if (deg < 1) return 1;
  B[1] = -C1 * y; B[2] = C1 * z; B[3] = -C1 * x;
  if (dB) {
    dB[1][0] = 0; dB[1][1] = -C1; dB[1][2] = 0;
    dB[2][0] = 0; dB[2][1] = 0; dB[2][2] = C1;
    dB[3][0] = -C1; dB[3][1] = 0; dB[3][2] = 0;
  }
  if (deg < 2) return 4;
  const float xx = x * x, yy = y * y, zz = z * z;
  B[4] = C2[0] * x * y;
  B[5] = C2[1] * y * z;
  B[6] = C2[2] * (2.0f * zz - xx - yy);
  B[7] = C2[3] * x * z;
  B[8] = C2[4] * (xx - yy);
  if (dB) {
    dB[4][0] = C2[0] * y; dB[4][1] = C2[0] * x; dB[4][2] = 0;
    dB[5][0] = 0; dB[5][1] = C2[1] * z; dB[5][2] = C2[1] * y;
    dB[6][0] = -2.0f * C2[2] * x; dB[6][1] = -2.0f * C2[2] * y; dB[6][2] = 4.0f * C2[2] * z;
    dB[7][0] = C2[3] * z; dB[7][1] = 0; dB[7][2] = C2[3] * x;
    dB[8][0] = 2.0f * C2[4] * x; dB[8][1] = -2.0f * C2[4] * y; dB[8][2] = 0;
  }
  if (deg < 3) return 9;
  B[9] = C3[0] * y * (3.0f * xx - yy);
  B[10] = C3[1] * x * y * z;
  B[11] = C3[2] * y * (4.0f * zz - xx - yy);
  B[12] = C3[3] * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
  B[13] = C3[4] * x * (4.0f * zz - xx - yy);
  B[14] = C3[5] * z * (xx - yy);
  B[15] = C3[6] * x * (xx - 3.0f * yy);
  if (dB) {
    dB[9][0] = C3[0] * 6.0f * x * y; dB[9][1] = C3[0] * (3.0f * xx - 3.0f * yy); dB[9][2] = 0;
    dB[10][0] = C3[1] * y * z; dB[10][1] = C3[1] * x * z; dB[10][2] = C3[1] * x * y;
    dB[11][0] = -2.0f * C3[2] * x * y; dB[11][1] = C3[2] * (4.0f * zz - xx - 3.0f * yy);
    dB[11][2] = 8.0f * C3[2] * y * z;
    dB[12][0] = -6.0f * C3[3] * x * z; dB[12][1] = -6.0f * C3[3] * y * z;
    dB[12][2] = C3[3] * (6.0f * zz - 3.0f * xx - 3.0f * yy);
    dB[13][0] = C3[4] * (4.0f * zz - 3.0f * xx - yy); dB[13][1] = -2.0f * C3[4] * x * y;
    dB[13][2] = 8.0f * C3[4] * x * z;
    dB[14][0] = 2.0f * C3[5] * x * z; dB[14][1] = -2.0f * C3[5] * y * z; dB[14][2] = C3[5] * (xx - yy);
    dB[15][0] = C3[6] * (3.0f * xx - 3.0f * yy); dB[15][1] = -6.0f * C3[6] * x * y; dB[15][2] = 0;
  }
  return 16;
}

// Orthonormal pair (e1, e2) completing n, built in the frame where n's
// largest component k plays the role of z (Duff et al. 2017 branchless
// basis), so that every entry is accurate relative to n's small components.
// The other two components, in order, play x and y.  Components are moved
// with selects rather than an index, which keeps them in registers.
__device__ __forceinline__ void ortho_basis(const float n[3], float e1[3], float e2[3]) {
  const float ax = fabsf(n[0]), ay = fabsf(n[1]), az = fabsf(n[2]);
  const bool k0 = ax > ay && ax > az;   // k = 0
  const bool k2 = !k0 && !(ay > az);    // k = 2 (else k = 1)
  const float x = k0 ? n[1] : n[0];
  const float y = k2 ? n[1] : n[2];
  const float z = k0 ? n[0] : (k2 ? n[2] : n[1]);
  const float sg = copysignf(1.0f, z);
  const float p = -__builtin_amdgcn_rcpf(sg + z);
  const float q = x * y * p;
  const float u0 = 1.0f + sg * x * x * p, u1 = sg * q, u2 = -sg * x;
  const float w0 = q, w1 = sg + y * y * p, w2 = -y;
  // component 0 is x unless k = 0; component 1 is x (k = 0), y (k = 2) or z;
  // component 2 is y unless k = 2
  e1[0] = k0 ? u2 : u0;
  e1[1] = k0 ? u0 : (k2 ? u1 : u2);
  e1[2] = k2 ? u2 : u1;
  e2[0] = k0 ? w2 : w0;
  e2[1] = k0 ? w0 : (k2 ? w1 : w2);
  e2[2] = k2 ? w2 : w1;
}

// Rotated canonical frame of one (Gaussian, view) item: Wc = S^-1 A^T maps a
// camera-space direction to canonical coordinates, o_u is the canonical
// camera centre, and Q = (e1; e2; n) rotates o_u onto the third axis.
struct Frame3 {
  float Wc[9];
  float ou[3];
  float r2, r;
  float e1[3], e2[3], nn[3];
};

__device__ __forceinline__ void canonical_frame(const AssocOut& A, const float s[3], Frame3& F) {
#pragma unroll
  for (int kk = 0; kk < 3; ++kk) {
    const float is = __builtin_amdgcn_rcpf(s[kk]);
#pragma unroll
    for (int ii = 0; ii < 3; ++ii) F.Wc[kk * 3 + ii] = A.A[ii * 3 + kk] * is;
  }
  F.ou[0] = -A.vou[0]; F.ou[1] = -A.vou[1]; F.ou[2] = -A.vou[2];
  F.r2 = F.ou[0] * F.ou[0] + F.ou[1] * F.ou[1] + F.ou[2] * F.ou[2];
  const float rinv = rsqrtf(F.r2);
  F.r = F.r2 * rinv;
  F.nn[0] = F.ou[0] * rinv; F.nn[1] = F.ou[1] * rinv; F.nn[2] = F.ou[2] * rinv;
  ortho_basis(F.nn, F.e1, F.e2);
}

// Adds a wave's evaluated-pair count to *total; every wave of the grid calls
// it exactly once (kWaves waves per workgroup).  The wave adds its count,
// with one wave in the top bits, to the counter of its workgroup's slot; the
// wave that completes a slot's tally adds the slot's sum to *total, so
// *total takes kEvalSlots atomics instead of one per wave (contended atomics
// on one word serialise).  The slots must start at zero.
template <int kWaves>
__device__ __forceinline__ void add_evals(unsigned long long* __restrict__ total,
                                          unsigned long long* __restrict__ slots, uint64_t evals) {
  if (!total || (threadIdx.x & 63) != 0) return;
  const unsigned s = blockIdx.x % kEvalSlots;
  const unsigned long long waves = (unsigned long long)((gridDim.x - 1 - s) / kEvalSlots + 1) * kWaves;
  const unsigned long long mine = (1ull << kEvalTallyShift) | evals;
  const unsigned long long old = atomicAdd(&slots[s * kEvalStride], mine);
  if ((old >> kEvalTallyShift) + 1 == waves) {
    const unsigned long long sum = (old + mine) & ((1ull << kEvalTallyShift) - 1);
    if (sum) atomicAdd(total, sum);
  }
}

// Workgroups are dealt round-robin to the 8 XCDs; give each XCD a contiguous
// band of tiles so that neighbouring tiles share its L2.
__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
  int q = nblocks >> 3, r = nblocks & 7, x = bid & 7;
  return x * q + min(x, r) + (bid >> 3);
}

// Unit camera-space direction of BEAP pixel (px, py) from the per-view
// (sin, cos) tables.
__device__ __forceinline__ void pixel_direction(const ViewDev& V, const float2* __restrict__ dtab, int px, int py,
                                                float& dx, float& dy, float& dz) {
  const float2 cth = dtab[V.dx_off + min(px, V.width - 1)];   // (sin, cos) theta
  const float2 cph = dtab[V.dy_off + min(py, V.height - 1)];  // (sin, cos) phi
  dx = cth.x * cph.y;
  dy = cth.y * cph.x;
  dz = cth.y * cph.y;
  const float dn = rsqrtf(dx * dx + dy * dy + dz * dz);
  dx *= dn;
  dy *= dn;
  dz *= dn;
}

// Work of one render wave: a block of rays of one tile.  Ordinary tiles are
// split into four 8x8 half-tiles (one lane per ray).  Tiles flagged heavy --
// list longer than 3x their view's mean (+64), which on wide BEAP grids
// happens where a tile fans over a wide range of directions and its rays see
// mostly different Gaussians -- are split into sixteen 4x4 blocks.  Their
// waves come first in the grid: kHeavySplit per heavy slot, and the waves of
// slot s render the listed tiles s, s + slots, s + 2 slots, ...  The rest of
// the grid addresses ordinary blocks (XCD-banded), skipping heavy tiles.
constexpr int kHeavySplit = 16;

struct WaveBlock {
  int tile, v;     // global tile, view
  int bx0, by0;    // first pixel of the block (view coordinates)
  int bs;          // block edge: 8, or 4 in heavy tiles
  bool live;       // false: nothing to do for this wave
};

// Wave index of wave w of workgroup j (K waves per workgroup, nwg
// workgroups, the first heavy_waves waves -- a multiple of K -- for heavy
// tiles).  Ordinary workgroups are banded by XCD as whole workgroups, so the
// K waves of a workgroup take K consecutive slots of its XCD's band.
__device__ __forceinline__ int wave_index(int j, int nwg, int K, int w, int heavy_waves) {
  const int jh = heavy_waves / K;
  if (j < jh) return j * K + w;
  return heavy_waves + K * xcd_remap(j - jh, nwg - jh) + w;
}

__device__ __forceinline__ WaveBlock block_of(int tile, int sub, int bs, const ViewDev* __restrict__ views,
                                              int nviews) {
  WaveBlock w;
  w.tile = tile;
  w.bs = bs;
  int v = 0;
  while (v + 1 < nviews && tile >= views[v + 1].tile_base) ++v;
  const ViewDev& V = views[v];
  w.v = v;
  const int lt = tile - V.tile_base;
  const int tx = lt % V.tiles_x, ty = lt / V.tiles_x;
  const int per = kTile / bs;  // blocks per tile edge
  w.bx0 = tx * kTile + (sub % per) * bs;
  w.by0 = ty * kTile + (sub / per) * bs;
  w.live = w.bx0 < V.width && w.by0 < V.height;
  return w;
}

// 4x4 block `sub` of a heavy tile.
__device__ __forceinline__ WaveBlock heavy_block(int tile, int sub, const ViewDev* __restrict__ views, int nviews) {
  return block_of(tile, sub, 4, views, nviews);
}

// Ordinary block of wave index wi (past the heavy waves); not live when its
// tile is heavy.
__device__ __forceinline__ WaveBlock ordinary_block(int wi, int heavy_waves, const ViewDev* __restrict__ views,
                                                    int nviews, const uint32_t* __restrict__ heavy_flag) {
  const int hidx = wi - heavy_waves;
  WaveBlock w = block_of(hidx >> 2, hidx & 3, 8, views, nviews);
  if (heavy_flag && heavy_flag[w.tile]) w.live = false;
  return w;
}

// Rays of a block of pixels.  Lines of constant theta and of constant phi
// on the BEAP grid are great circles (x cos(theta) = z sin(theta),
// y cos(phi) = z sin(phi)).  While cos(theta) keeps one sign over the block,
// theta = atan2(x, z) and sign(cos theta) (y cos(phi0) - z sin(phi0)) >= 0
// for phi >= phi0, so the block's directions are the intersection of four
// half-spaces: the convex cone spanned by its four corner rays, listed here
// in cyclic order.  A block whose theta range reaches +-90 degrees contains
// the pole where every phi line meets and is not that cone (valid = false).
struct QuadCone {
  float d[4][3];
  bool valid;
};

// Corner rays of the block of pixels [x0, x0 + size) x [y0, y0 + size) (clipped
// to the image).
__device__ __forceinline__ QuadCone block_cone(const ViewDev& V, const float2* __restrict__ dtab, int x0, int y0,
                                               int size) {
  const int x1 = min(x0 + size - 1, V.width - 1), y1 = min(y0 + size - 1, V.height - 1);
  QuadCone C;
  const float c0 = dtab[V.dx_off + x0].y, c1 = dtab[V.dx_off + x1].y;  // cos(theta) of the end columns
  C.valid = (c0 > 0.0f && c1 > 0.0f) || (c0 < 0.0f && c1 < 0.0f);
  pixel_direction(V, dtab, x0, y0, C.d[0][0], C.d[0][1], C.d[0][2]);
  pixel_direction(V, dtab, x1, y0, C.d[1][0], C.d[1][1], C.d[1][2]);
  pixel_direction(V, dtab, x1, y1, C.d[2][0], C.d[2][1], C.d[2][2]);
  pixel_direction(V, dtab, x0, y1, C.d[3][0], C.d[3][1], C.d[3][2]);
  return C;
}

__device__ __forceinline__ QuadCone half_tile_cone(const ViewDev& V, const float2* __restrict__ dtab, int hx, int hy) {
  return block_cone(V, dtab, hx * kHalf, hy * kHalf, kHalf);
}

// Conservative test of whether any ray of a block of pixels (a half-tile or
// a tile) can contribute through a record (false only when none can).  In
// the record's frame g = G d a ray contributes only if q = |g_xy|^2 / |g|^2
// <= Qc, the largest q that keeps sigma exp(-kappa/2) >= alpha_min (and,
// with a fixed lambda, q <= qmax), and g_z > 0: a circular cone
// |g_xy| <= tau g_z, tau^2 = Qc / (1 - Qc).  On the plane g_z = 1 that cone is
// the disc |p| <= tau.  When every corner is well in front (g_z > 0 and
// |g_x| + |g_y| <= 16 g_z) the block's cone meets that plane in the convex
// quad of the corners, and the test is the distance from the disc's centre
// to that quad (the common case, about half the arithmetic).  Otherwise the
// part of the block's cone (spanned by the
// corners g_k) in front, g_z > 0, is the intersection of the four half-planes
// n_k . (p, 1) >= 0 with n_k = g_k x g_(k+1) oriented inward (bounded or
// not, whatever the signs of the corners' g_z).  The test is whether the
// distance from the disc's centre to that region is at most tau: zero if
// every n_k,z >= 0, else the smallest of the distances to the face lines
// whose foot point lies in the region and to the corners in front.  The
// corner vectors are rescaled to unit max-norm first (the cone is unchanged);
// FP32 margins: Qc + 2^-8 Qc + 2^-20, tau^2 + 2^-8 tau^2 + 2^-18 (1 + d^2),
// and 2^-12 relative slack in the foot-point test.  Quotients and square
// roots use the hardware reciprocal and square root (about 1 ulp): the
// margins are orders of magnitude wider, and the rescale only needs a
// positive factor.
__device__ __forceinline__ bool cone_meets_quad(const float4& p0, const float4& p1, const float4& p2, const float4& p3,
                                                const QuadCone& C, float log2_amin, bool fixed) {
  if (!C.valid) return true;
  const float G[9] = {p0.x, p0.y, p0.z, p0.w, p1.x, p1.y, p1.z, p1.w, p2.x};
  const float c0 = p2.y, lsig = p2.z, qmax = p3.w;
  float Qc = (lsig - log2_amin) * __builtin_amdgcn_rcpf(-c0);
  if (fixed) Qc = fminf(Qc, qmax);
  Qc = fmaf(Qc, 0x1p-8f, Qc) + 0x1p-20f;
  if (!(Qc > 0.0f)) return false;
  if (Qc >= 1.0f) return true;
  const float tau2 = Qc * __builtin_amdgcn_rcpf(1.0f - Qc);
  float g[4][3];
  bool bounded = true;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float* d = C.d[k];
    g[k][0] = fmaf(G[2], d[2], fmaf(G[1], d[1], G[0] * d[0]));
    g[k][1] = fmaf(G[5], d[2], fmaf(G[4], d[1], G[3] * d[0]));
    g[k][2] = fmaf(G[8], d[2], fmaf(G[7], d[1], G[6] * d[0]));
    bounded &= g[k][2] > 0.0f && fabsf(g[k][0]) + fabsf(g[k][1]) <= 16.0f * g[k][2];
  }
  if (bounded) {
    // Every corner in front with |p| <= 16 sqrt 2 on the plane g_z = 1: the
    // region is the convex quad of the corners p_k, and its distance from
    // the disc's centre is zero when the centre is on the inner side of
    // every edge, else the least distance to the four edge segments.
    float vx[4], vy[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float iz = __builtin_amdgcn_rcpf(g[k][2]);
      vx[k] = g[k][0] * iz;
      vy[k] = g[k][1] * iz;
    }
    float best = INFINITY;
    bool pos = true, neg = true;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int k1 = (k + 1) & 3;
      const float ex = vx[k1] - vx[k], ey = vy[k1] - vy[k];
      const float cr = fmaf(vx[k], ey, -vy[k] * ex);  // side of the centre
      pos &= cr >= 0.0f;
      neg &= cr <= 0.0f;
      const float ee = fmaf(ex, ex, ey * ey);
      float t = ee > 0.0f ? -fmaf(vx[k], ex, vy[k] * ey) * __builtin_amdgcn_rcpf(ee) : 0.0f;
      t = fminf(fmaxf(t, 0.0f), 1.0f);
      const float px = fmaf(t, ex, vx[k]), py = fmaf(t, ey, vy[k]);
      best = fminf(best, fmaf(px, px, py * py));
    }
    return pos || neg || best <= fmaf(tau2, 0x1p-8f, tau2) + 0x1p-18f * (1.0f + best);
  }
  bool any_front = false;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float m = fmaxf(fmaxf(fabsf(g[k][0]), fabsf(g[k][1])), fabsf(g[k][2]));
    const float im = m > 0.0f ? __builtin_amdgcn_rcpf(m) : 0.0f;
    any_front |= g[k][2] > 0.0f;
    g[k][0] *= im;
    g[k][1] *= im;
    g[k][2] *= im;
  }
  if (!any_front) return false;  // every ray of the block has g_z <= 0
  float n[4][3];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float* a = g[k];
    const float* b = g[(k + 1) & 3];
    n[k][0] = a[1] * b[2] - a[2] * b[1];
    n[k][1] = a[2] * b[0] - a[0] * b[2];
    n[k][2] = a[0] * b[1] - a[1] * b[0];
  }
  // inward orientation: the corners' sum lies inside the cone
  const float ox = g[0][0] + g[1][0] + g[2][0] + g[3][0];
  const float oy = g[0][1] + g[1][1] + g[2][1] + g[3][1];
  const float oz = g[0][2] + g[1][2] + g[2][2] + g[3][2];
  const float orient = n[0][0] * ox + n[0][1] * oy + n[0][2] * oz;
  if (!(fabsf(orient) > 1e-12f)) return true;  // degenerate block cone
  const float sg = orient > 0.0f ? 1.0f : -1.0f;
  bool inside = true;
  float nxy2[4], nxy[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    n[k][0] *= sg;
    n[k][1] *= sg;
    n[k][2] *= sg;
    inside &= n[k][2] >= 0.0f;
    nxy2[k] = fmaf(n[k][0], n[k][0], n[k][1] * n[k][1]);
    nxy[k] = __builtin_amdgcn_sqrtf(nxy2[k]);
  }
  if (inside) return true;
  float best = INFINITY;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (!(nxy2[k] > 0.0f)) continue;
    const float inv = __builtin_amdgcn_rcpf(nxy2[k]);
    const float t = n[k][2] * inv;
    const float px = -t * n[k][0], py = -t * n[k][1];
    const float pn = __builtin_amdgcn_sqrtf(fmaf(px, px, py * py));
    bool on = true;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (j == k) continue;
      const float val = fmaf(n[j][0], px, fmaf(n[j][1], py, n[j][2]));
      on &= val >= -0x1p-12f * (fabsf(n[j][2]) + nxy[j] * pn);
    }
    if (on) best = fminf(best, (n[k][2] * n[k][2]) * inv);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (g[k][2] > 0.0f)
      best = fminf(best, fmaf(g[k][0], g[k][0], g[k][1] * g[k][1]) * __builtin_amdgcn_rcpf(g[k][2] * g[k][2]));
  return best <= fmaf(tau2, 0x1p-8f, tau2) + 0x1p-18f * (1.0f + best);
}

// One (ray, Gaussian) pair in the rotated canonical frame: g = G d,
// kappa = r^2 (gx^2 + gy^2) / |g|^2 = r^2 q, alpha_raw = sigma exp(-kappa/2).
struct PairEval {
  float gx, gy, gz, mm, ss, inv, q, a_raw;
};

__device__ __forceinline__ PairEval eval_pair(const Record& R, float dx, float dy, float dz) {
  PairEval E;
  E.gx = fmaf(R.g[2], dz, fmaf(R.g[1], dy, R.g[0] * dx));
  E.gy = fmaf(R.g[5], dz, fmaf(R.g[4], dy, R.g[3] * dx));
  E.gz = fmaf(R.g[8], dz, fmaf(R.g[7], dy, R.g[6] * dx));
  E.mm = fmaf(E.gy, E.gy, E.gx * E.gx);
  E.ss = fmaf(E.gz, E.gz, E.mm);
  E.inv = __builtin_amdgcn_rcpf(E.ss);
  E.q = E.mm * E.inv;
  E.a_raw = __builtin_amdgcn_exp2f(fmaf(R.c0, E.q, R.lsig));
  return E;
}

// The contribution rule: closest approach in front of the camera, alpha above
// alpha_min, and (fixed-lambda mode) kappa <= lambda^2.
template <bool kFixed>
__device__ __forceinline__ bool pair_contributes(const Record& R, const PairEval& E, const Opts& op) {
  bool ok = (E.gz > 0.0f) & (E.a_raw >= op.alpha_min);
  if (kFixed) ok = ok & (E.q <= R.qmax);
  return ok;
}

__device__ __forceinline__ float clamp_alpha(float a, const Opts& op) { return a < op.alpha_max ? a : op.alpha_max; }

}  // namespace geer
