/*
 * FP64 brute-force oracle for exact Gaussian ray rendering (3DGEER,
 * arXiv 2505.24053).  TEST INFRASTRUCTURE ONLY: nothing in the product path
 * may link, load or call this file; only the tests, the smoke check and the
 * CPU-baseline leg of the benchmark do.
 *
 * What it computes, with the passage each part follows:
 *   - per Gaussian: Sigma = R S S^T R^T with R from the unit quaternion, the
 *     whitening matrix W = S^-1 R^T written entry by entry as printed in the
 *     cookbook appendix (quaternion form of W_pca), canonical camera centre
 *     o_u = W (o - mu)                                   (App. B, C.1, C.5)
 *   - per ray: BEAP pixel centre (theta, phi) -> unit direction
 *                                                        (Sec. 3.3, App. E)
 *   - per (ray, Gaussian) pair, with NO culling structure: d_u = W d,
 *     m_u = o_u x d_u, kappa = |m_u|^2 / |d_u|^2 (cross-product form),
 *     alpha = sigma exp(-kappa / 2)          (Eq. trans:cano, mahdist_comp)
 *   - order: ascending depth key, then Gaussian index; front-to-back
 *     compositing C = sum c_i a_i prod_{j<i} (1 - a_j)       (Eq. color)
 *   - gradients by the two-stage chain of the cookbook appendix (Eq. b6, b9,
 *     scaling, rotation, mean), with the cross-product terms taken with the
 *     sign that follows from m_u = o_u x d_u (see the README-level notes in
 *     the repository design document: the printed cross terms correspond to
 *     m_u = d_u x o_u).
 *
 * Readings of the paper that this file fixes (each also listed in the design
 * document):
 *   - a pair contributes iff the Gaussian is not culled (camera at Mahalanobis
 *     distance >= 3, App. B), its closest approach lies in front of the
 *     camera (t* > 0), and kappa <= lambda_i^2 where lambda_i^2 =
 *     2 ln(sigma_i / alpha_min) (opacity-aware mode, the default) or
 *     kappa <= lambda^2 and alpha >= alpha_min (fixed-lambda mode, the
 *     paper's "typically 3");
 *   - alpha is clamped to alpha_max; compositing stops before the first
 *     Gaussian that would take the transmittance below T_min;
 *   - the depth key and the 3-sigma cull are integer decisions taken from
 *     floating point; they are computed in FP32 by the association
 *     reference below (same precision as the kernel), everything radiometric
 *     is FP64.
 *
 * The second half of the file is the FP32 association reference: the
 * particle-bounding-frustum bounds (Sec. 3.2, App. D.1 Eq. solve_tan,
 * pbf-cov3d), their mirror transform with xi = 1 (App. D.2 Eq. aabb) and the
 * camera-sub-frustum intersection, each IEEE single operation written out
 * in a fixed order with no fused multiply-add, so that its tile rectangles,
 * counts and depth keys are the bit-exact target of the GPU association.
 * Compile with -ffp-contract=off and without -ffast-math.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------- records -- */

typedef struct {
  int32_t model, width, height;
  int32_t grid; /* 0: BEAP grid over fov_x x fov_y; 1: native pinhole pixels */
  double fx, fy, cx, cy, k[4];
  double fov_x, fov_y;
  double R[9], t[3];
} orc_view;

typedef struct {
  double alpha_min, alpha_max, t_min, lambda_fixed;
  int32_t lambda_mode; /* 0 opacity-aware, 1 fixed lambda */
  int32_t splat;       /* 1: splat opacity (local affine footprint) instead of the exact one */
} orc_opts;

typedef struct {
  int64_t n;
  int32_t sh_degree, pad_;
  /* SoA arrays (layout of the synthetic-scene module); FP64 so that finite
   differences can perturb them below FP32 resolution.  The FP32 association
   reference rounds them to float first. */
  const double *mean, *scale, *quat, *opacity, *sh;
} orc_scene;

/* per-Gaussian FP32 association result */
typedef struct {
  int32_t hx0, hx1, hy0, hy1; /* half-tile (8 px) column / row ranges, inclusive */
  uint32_t count;             /* 16x16 tiles covered, 0 = not visible */
  uint32_t key;               /* bits of the FP32 squared camera distance */
  int32_t culled;             /* camera within 3 sigma (FP32 decision) */
  int32_t pad_;
} orc_assoc;

/* ---------------------------------------------------- FP32 reference ----- */
/* Every statement below is one IEEE single operation (or a comparison).      */

#define HALF 8 /* half-tile edge in pixels */

static float f_max(float a, float b) { return a > b ? a : b; }
static float f_min(float a, float b) { return a < b ? a : b; }

/* BEAP angles at pixel coordinate x (columns) / y (rows): uniform over the
 * field of view, or for a native pinhole grid the angle whose tangent is
 * the normalised image coordinate (x / z = tan(theta), y / z = tan(phi) of
 * the pinhole model, App. E). */
static double col_angle(const orc_view* v, double x) {
  if (v->grid == 1) return atan((x - v->cx) / v->fx);
  return -v->fov_x / 2 + x * v->fov_x / v->width;
}
static double row_angle(const orc_view* v, double y) {
  if (v->grid == 1) return atan((y - v->cy) / v->fy);
  return -v->fov_y / 2 + y * v->fov_y / v->height;
}

/* half-tile column edges: mirrored tan(theta / 2) at pixel boundaries 8h, w */
static void edges_theta(const orc_view* v, float* e, int* nh) {
  int w = v->width, n = (w + HALF - 1) / HALF;
  for (int h = 0; h <= n; ++h) {
    int b = h < n ? h * HALF : w;
    double th = col_angle(v, (double)b);
    e[h] = (float)tan(th / 2);
  }
  *nh = n;
}

/* half-tile row edges: tan(phi) at pixel boundaries 8h, h_img */
static void edges_phi(const orc_view* v, float* e, int* nh) {
  int hh = v->height, n = (hh + HALF - 1) / HALF;
  for (int h = 0; h <= n; ++h) {
    int b = h < n ? h * HALF : hh;
    double ph = row_angle(v, (double)b);
    e[h] = (float)tan(ph);
  }
  *nh = n;
}

static float round_up_f32(double x) {
  float f = (float)x;
  if ((double)f < x) f = nextafterf(f, INFINITY);
  return f;
}

/* Conservative lambda^2: buckets of 2^17 consecutive float bit patterns; the
 * bucket value is 2 ln(sigma_hi / alpha_min) at the bucket's upper end,
 * inflated by 2^-10 and rounded up. */
#define LAM_SHIFT 17
static uint32_t f2u(float f) { uint32_t u; memcpy(&u, &f, 4); return u; }
static float u2f(uint32_t u) { float f; memcpy(&f, &u, 4); return f; }

static float lambda2_hat(float sigma, float amin, int mode, double lam_fixed) {
  if (mode == 1) return round_up_f32(lam_fixed * lam_fixed * (1.0 + 1.0 / 1024.0));
  uint32_t lo = f2u(amin) >> LAM_SHIFT, hi = f2u(16.0f) >> LAM_SHIFT;
  uint32_t b = f2u(sigma) >> LAM_SHIFT;
  if (b < lo) b = lo;
  if (b > hi) b = hi;
  double top = (double)u2f((b + 1) << LAM_SHIFT);
  double l2 = 2.0 * log(top / (double)amin);
  if (l2 < 0) l2 = 0;
  return round_up_f32(l2 * (1.0 + 1.0 / 1024.0));
}

static float pad_of(float x) {
  float ax = fabsf(x);
  float one = 1.0f;
  float s = one + ax;
  return s * 0x1p-14f;
}

/* closed-interval overlap of [a, b] with cells [e[h], e[h+1]], h in [0, n) */
static int cell_range(const float* e, int n, float a, float b, int* c0, int* c1) {
  int lo = n, hi = -1;
  for (int h = 0; h < n; ++h) {
    if (e[h + 1] >= a && e[h] <= b) {
      if (h < lo) lo = h;
      if (h > hi) hi = h;
    }
  }
  *c0 = lo;
  *c1 = hi;
  return lo <= hi;
}

/* ranges of a 1-2 piece set given as [a0,b0] (and [a1,b1] if two) */
static int pieces_range(const float* e, int n, int npieces, const float* a, const float* b,
                        int* c0, int* c1) {
  int lo = n, hi = -1, any = 0;
  for (int p = 0; p < npieces; ++p) {
    int x0, x1;
    if (cell_range(e, n, a[p], b[p], &x0, &x1)) {
      any = 1;
      if (x0 < lo) lo = x0;
      if (x1 > hi) hi = x1;
    }
  }
  *c0 = lo;
  *c1 = hi;
  return any;
}

static void assoc_one(const float* mu, const float* s, const float* q, float sigma,
                      const float Rc[9], const float tc[3], float amin, int mode, double lam_fixed,
                      const float* ex, int nhx, const float* ey, int nhy, orc_assoc* out) {
  out->hx0 = 1; out->hx1 = 0; out->hy0 = 1; out->hy1 = 0;
  out->count = 0; out->key = 0; out->culled = 0; out->pad_ = 0;

  /* unit quaternion */
  float q0 = q[0], q1 = q[1], q2 = q[2], q3 = q[3];
  float qq = q0 * q0;
  qq = qq + q1 * q1;
  qq = qq + q2 * q2;
  qq = qq + q3 * q3;
  float qn = sqrtf(qq);
  float r = q0 / qn, i = q1 / qn, j = q2 / qn, k = q3 / qn;

  /* local-to-world rotation R */
  float xx = i * i, yy = j * j, zz = k * k, xy = i * j, xz = i * k, yz = j * k;
  float rx = r * i, ry = r * j, rz = r * k;
  float R[9];
  R[0] = 1.0f - 2.0f * (yy + zz); R[1] = 2.0f * (xy - rz);        R[2] = 2.0f * (xz + ry);
  R[3] = 2.0f * (xy + rz);        R[4] = 1.0f - 2.0f * (xx + zz); R[5] = 2.0f * (yz - rx);
  R[6] = 2.0f * (xz - ry);        R[7] = 2.0f * (yz + rx);        R[8] = 1.0f - 2.0f * (xx + yy);

  /* A = Rc R, M = A S (camera-space columns of the local frame, scaled) */
  float A[9], M[9];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      float t0 = Rc[a * 3 + 0] * R[0 * 3 + b];
      float t1 = Rc[a * 3 + 1] * R[1 * 3 + b];
      float t2 = Rc[a * 3 + 2] * R[2 * 3 + b];
      float acc = t0 + t1;
      acc = acc + t2;
      A[a * 3 + b] = acc;
      M[a * 3 + b] = acc * s[b];
    }

  /* camera-space mean */
  float mc[3];
  for (int a = 0; a < 3; ++a) {
    float t0 = Rc[a * 3 + 0] * mu[0];
    float t1 = Rc[a * 3 + 1] * mu[1];
    float t2 = Rc[a * 3 + 2] * mu[2];
    float acc = t0 + t1;
    acc = acc + t2;
    mc[a] = acc + tc[a];
  }

  /* depth key: squared camera distance */
  {
    float d0 = mc[0] * mc[0], d1 = mc[1] * mc[1], d2 = mc[2] * mc[2];
    float dd = d0 + d1;
    dd = dd + d2;
    out->key = f2u(dd);
  }

  /* 3-sigma cull: |S^-1 A^T mu_c|^2 < 9 */
  {
    float ou2 = 0.0f;
    for (int b = 0; b < 3; ++b) {
      float t0 = A[0 * 3 + b] * mc[0];
      float t1 = A[1 * 3 + b] * mc[1];
      float t2 = A[2 * 3 + b] * mc[2];
      float acc = t0 + t1;
      acc = acc + t2;
      float v = acc / s[b];
      float v2 = v * v;
      ou2 = b == 0 ? v2 : ou2 + v2;
    }
    if (ou2 < 9.0f) { out->culled = 1; return; }
  }
  if (!(qq > 0.0f)) return;
  if (!(sigma > amin)) return;

  float L = lambda2_hat(sigma, amin, mode, lam_fixed);

  /* view-space covariance entries Sigma_ab = m_a . m_b (m_a = row a of M) */
#define DOT3(a, b) ((M[(a)*3 + 0] * M[(b)*3 + 0] + M[(a)*3 + 1] * M[(b)*3 + 1]) + M[(a)*3 + 2] * M[(b)*3 + 2])
  float S00 = DOT3(0, 0), S02 = DOT3(0, 2), S22 = DOT3(2, 2), S11 = DOT3(1, 1), S12 = DOT3(1, 2);
#undef DOT3
  float T00 = L * S00 - mc[0] * mc[0];
  float T02 = L * S02 - mc[0] * mc[2];
  float T22 = L * S22 - mc[2] * mc[2];
  float T11 = L * S11 - mc[1] * mc[1];
  float T12 = L * S12 - mc[1] * mc[2];

  /* ---- theta bounds (planes through the camera y axis) ---- */
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
    int full = !(D > P * 0x1p-12f);
    if (full) {
      hx0 = 0; hx1 = nhx - 1;
    } else {
      float sd = sqrtf(L * D);
      float qv = T02 >= 0.0f ? T02 + sd : T02 - sd;
      float rs[2] = {qv, T00}, rk[2] = {T22, qv};
      float cand[4];
      for (int t = 0; t < 2; ++t) {
        float ss = rs[t], kk = rk[t];
        if (kk < 0.0f) { ss = -ss; kk = -kk; }
        float rr = sqrtf(ss * ss + kk * kk);
        float kr = kk + rr;
        cand[2 * t + 0] = ss / kr;
        cand[2 * t + 1] = -(kr / ss);
      }
      float rho = sqrtf(mc[0] * mc[0] + mc[2] * mc[2]);
      float tmu = mc[2] >= 0.0f ? mc[0] / (mc[2] + rho) : (rho - mc[2]) / mc[0];
      int has_lo = 0, has_hi = 0;
      float lo = 0.0f, hi = 0.0f, cmin = cand[0], cmax = cand[0];
      for (int t = 0; t < 4; ++t) {
        float c = cand[t];
        cmin = f_min(cmin, c);
        cmax = f_max(cmax, c);
        if (c < tmu) { lo = has_lo ? f_max(lo, c) : c; has_lo = 1; }
        if (c > tmu) { hi = has_hi ? f_min(hi, c) : c; has_hi = 1; }
      }
      float a[2], b[2];
      int np;
      if (has_lo && has_hi) {
        a[0] = lo - pad_of(lo); b[0] = hi + pad_of(hi); np = 1;
      } else {
        a[0] = -INFINITY; b[0] = cmin + pad_of(cmin);
        a[1] = cmax - pad_of(cmax); b[1] = INFINITY; np = 2;
      }
      if (!pieces_range(ex, nhx, np, a, b, &hx0, &hx1)) return;
    }
  }

  /* ---- phi bounds (planes through the camera x axis) ---- */
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
    int full = !(D > P * 0x1p-12f) || !(T22 < -tz || T22 > tz);
    if (full) {
      hy0 = 0; hy1 = nhy - 1;
    } else {
      float sd = sqrtf(L * D);
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
      if (!pieces_range(ey, nhy, np, a, b, &hy0, &hy1)) return;
    }
  }

  out->hx0 = hx0; out->hx1 = hx1; out->hy0 = hy0; out->hy1 = hy1;
  out->count = (uint32_t)((hx1 / 2 - hx0 / 2 + 1) * (hy1 / 2 - hy0 / 2 + 1));
}

static void view_f32(const orc_view* v, float Rc[9], float tc[3]) {
  for (int a = 0; a < 9; ++a) Rc[a] = (float)v->R[a];
  for (int a = 0; a < 3; ++a) tc[a] = (float)v->t[a];
}

/* FP32 association of every Gaussian against one view. */
int orc_assoc_fp32(const orc_scene* sc, const orc_view* v, const orc_opts* op, orc_assoc* out) {
  int nhx, nhy;
  float* ex = (float*)malloc(sizeof(float) * ((size_t)v->width / HALF + 2));
  float* ey = (float*)malloc(sizeof(float) * ((size_t)v->height / HALF + 2));
  if (!ex || !ey) { free(ex); free(ey); return -1; }
  edges_theta(v, ex, &nhx);
  edges_phi(v, ey, &nhy);
  float Rc[9], tc[3];
  view_f32(v, Rc, tc);
  int64_t n = sc->n;
  float amin = (float)op->alpha_min;
#pragma omp parallel for schedule(static)
  for (int64_t g = 0; g < n; ++g) {
    float mu[3] = {(float)sc->mean[g], (float)sc->mean[n + g], (float)sc->mean[2 * n + g]};
    float s[3] = {(float)sc->scale[g], (float)sc->scale[n + g], (float)sc->scale[2 * n + g]};
    float q[4] = {(float)sc->quat[g], (float)sc->quat[n + g], (float)sc->quat[2 * n + g], (float)sc->quat[3 * n + g]};
    assoc_one(mu, s, q, (float)sc->opacity[g], Rc, tc, amin, op->lambda_mode, op->lambda_fixed, ex, nhx,
              ey, nhy, &out[g]);
  }
  free(ex);
  free(ey);
  return 0;
}

/* Exposed for tests: the edge tables and the conservative lambda^2. */
int orc_edges(const orc_view* v, float* ex, float* ey, int* nhx, int* nhy) {
  edges_theta(v, ex, nhx);
  edges_phi(v, ey, nhy);
  return 0;
}

float orc_lambda2_hat(float sigma, float amin, int mode, double lam_fixed) {
  return lambda2_hat(sigma, amin, mode, lam_fixed);
}

/* --------------------------------------------------- spherical harmonics -- */
/* Real SH with the Condon-Shortley phase, index k = l^2 + l + m, l <= 3:
 *   m = 0 : K_l^0 P_l(z)
 *   m > 0 : sqrt(2) K_l^m (-1)^m P_l^(m)(z) Re((x + i y)^m)
 *   m < 0 : sqrt(2) K_l^|m| (-1)^|m| P_l^(|m|)(z) Im((x + i y)^|m|)
 * with K_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) and P_l^(m) the m-th
 * derivative of the Legendre polynomial; on the unit sphere this equals the
 * usual real SH basis.  Evaluated together with its gradient in R^3. */

static double fact(int n) { double f = 1; for (int i = 2; i <= n; ++i) f *= i; return f; }

static void legendre_coeffs(int l, double* c /* [4], c[p] z^p */) {
  double P[4][4] = {{0}};
  P[0][0] = 1;
  P[1][1] = 1;
  for (int n = 1; n < 3; ++n)
    for (int p = 0; p < 4; ++p) {
      double v = -(double)n * P[n - 1][p];
      if (p > 0) v += (2.0 * n + 1) * P[n][p - 1];
      P[n + 1][p] = v / (n + 1);
    }
  for (int p = 0; p < 4; ++p) c[p] = P[l][p];
}

static void sh_basis(int deg, const double v[3], double* Y, double (*dY)[3]) {
  const double x = v[0], y = v[1], z = v[2];
  for (int l = 0; l <= deg; ++l) {
    double c[4];
    legendre_coeffs(l, c);
    for (int m = -l; m <= l; ++m) {
      int am = m < 0 ? -m : m;
      /* m-th derivative of P_l */
      double dc[4] = {c[0], c[1], c[2], c[3]};
      for (int t = 0; t < am; ++t) {
        for (int p = 0; p < 3; ++p) dc[p] = dc[p + 1] * (p + 1);
        dc[3] = 0;
      }
      double D = ((dc[3] * z + dc[2]) * z + dc[1]) * z + dc[0];
      double Dz = (3 * dc[3] * z + 2 * dc[2]) * z + dc[1];
      /* w = (x + i y)^am and w' = am (x + i y)^(am-1) */
      double wr = 1, wi = 0, pr = 0, pi = 0;
      for (int t = 0; t < am; ++t) {
        if (t == am - 1) { pr = wr * am; pi = wi * am; }
        double nr = wr * x - wi * y, ni = wr * y + wi * x;
        wr = nr; wi = ni;
      }
      double K = sqrt((2.0 * l + 1) / (4.0 * M_PI) * fact(l - am) / fact(l + am));
      double N = (am == 0) ? K : sqrt(2.0) * K * ((am & 1) ? -1.0 : 1.0);
      double F, Fx, Fy;
      if (m == 0) { F = 1; Fx = 0; Fy = 0; }
      else if (m > 0) { F = wr; Fx = pr; Fy = -pi; }
      else { F = wi; Fx = pi; Fy = pr; }
      int k = l * l + l + m;
      Y[k] = N * D * F;
      if (dY) {
        dY[k][0] = N * D * Fx;
        dY[k][1] = N * D * Fy;
        dY[k][2] = N * Dz * F;
      }
    }
  }
}

int orc_sh_basis(int deg, int64_t nd, const double* dirs, double* Y, double* dY) {
  int K = (deg + 1) * (deg + 1);
  for (int64_t i = 0; i < nd; ++i)
    sh_basis(deg, dirs + 3 * i, Y + K * i, dY ? (double(*)[3])(dY + 3 * K * i) : NULL);
  return 0;
}

/* ------------------------------------------------------- FP64 renderer -- */

typedef struct {
  double W[9];     /* whitening matrix S^-1 R^T */
  double R[9];     /* local-to-world rotation from the unit quaternion */
  double ou[3];    /* canonical camera centre */
  double col[3];   /* view-dependent colour, clamped at 0 */
  double craw[3];  /* colour before the clamp */
  double sigma, lam2;
  double v[3], dist; /* unit direction centre - camera, and its length */
  double qh[4], qn, s[3];
  int active;      /* not culled and sigma > alpha_min */
  uint32_t key;
  int hx0, hx1, hy0, hy1, vis; /* FP32 association: half-tile rectangle, visible */
  /* splat opacity: BEAP angles of the mean, conic C^-1 = [ia ib; ib ic] of
     the local affine footprint, its largest eigenvalue, the condition
     c00 c11 / det(C), and the mean's camera distance */
  double tc, pc, ia, ib, ic, icmax, ccond, mdist;
} gprep;

static void prep_gaussians(const orc_scene* sc, const orc_view* vw, const orc_opts* op, gprep* P,
                           const orc_assoc* as) {
  int64_t n = sc->n;
  int deg = sc->sh_degree, K = (deg + 1) * (deg + 1);
  const double* Rc = vw->R;
  double o[3];
  for (int a = 0; a < 3; ++a) o[a] = -(Rc[0 * 3 + a] * vw->t[0] + Rc[1 * 3 + a] * vw->t[1] + Rc[2 * 3 + a] * vw->t[2]);
#pragma omp parallel for schedule(static)
  for (int64_t g = 0; g < n; ++g) {
    gprep* p = &P[g];
    double mu[3] = {sc->mean[g], sc->mean[n + g], sc->mean[2 * n + g]};
    double s[3] = {sc->scale[g], sc->scale[n + g], sc->scale[2 * n + g]};
    double q[4] = {sc->quat[g], sc->quat[n + g], sc->quat[2 * n + g], sc->quat[3 * n + g]};
    double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    double qr = q[0] / qn, qi = q[1] / qn, qj = q[2] / qn, qk = q[3] / qn;
    p->qh[0] = qr; p->qh[1] = qi; p->qh[2] = qj; p->qh[3] = qk; p->qn = qn;
    for (int a = 0; a < 3; ++a) p->s[a] = s[a];
    /* W_pca as printed (quaternion form), rows scaled by 1/s_k */
    double W[9] = {
        2 * (0.5 - qj * qj - qk * qk) / s[0], 2 * (qi * qj + qr * qk) / s[0], 2 * (qi * qk - qr * qj) / s[0],
        2 * (qi * qj - qr * qk) / s[1], 2 * (0.5 - qi * qi - qk * qk) / s[1], 2 * (qj * qk + qr * qi) / s[1],
        2 * (qi * qk + qr * qj) / s[2], 2 * (qj * qk - qr * qi) / s[2], 2 * (0.5 - qi * qi - qj * qj) / s[2]};
    memcpy(p->W, W, sizeof W);
    /* R = (S W)^T */
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) p->R[a * 3 + b] = W[b * 3 + a] * s[b];
    double om[3] = {o[0] - mu[0], o[1] - mu[1], o[2] - mu[2]};
    for (int a = 0; a < 3; ++a) p->ou[a] = W[a * 3 + 0] * om[0] + W[a * 3 + 1] * om[1] + W[a * 3 + 2] * om[2];
    p->sigma = sc->opacity[g];
    double amin = op->alpha_min;
    if (op->lambda_mode == 1) p->lam2 = op->lambda_fixed * op->lambda_fixed;
    else p->lam2 = p->sigma > amin ? 2.0 * log(p->sigma / amin) : -1.0;
    /* colour */
    double dv[3] = {mu[0] - o[0], mu[1] - o[1], mu[2] - o[2]};
    double dn = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
    p->dist = dn;
    for (int a = 0; a < 3; ++a) p->v[a] = dn > 0 ? dv[a] / dn : 0;
    double Y[16];
    sh_basis(deg, p->v, Y, NULL);
    for (int c = 0; c < 3; ++c) {
      double acc = 0.5;
      for (int k = 0; k < K; ++k) acc += Y[k] * (double)sc->sh[(size_t)(k * 3 + c) * n + g];
      p->craw[c] = acc;
      p->col[c] = acc > 0 ? acc : 0;
    }
    p->key = as[g].key;
    p->active = !as[g].culled && ((float)sc->opacity[g] > (float)op->alpha_min);
    p->hx0 = as[g].hx0; p->hx1 = as[g].hx1; p->hy0 = as[g].hy0; p->hy1 = as[g].hy1;
    p->vis = as[g].count > 0;
    if (op->splat) {
      /* camera-space mean and covariance Sigma_c = (Rc R S)(Rc R S)^T */
      double mc[3], A[9];
      for (int a = 0; a < 3; ++a) {
        mc[a] = Rc[a * 3 + 0] * mu[0] + Rc[a * 3 + 1] * mu[1] + Rc[a * 3 + 2] * mu[2] + vw->t[a];
        for (int b = 0; b < 3; ++b)
          A[a * 3 + b] = (Rc[a * 3 + 0] * p->R[0 * 3 + b] + Rc[a * 3 + 1] * p->R[1 * 3 + b] +
                          Rc[a * 3 + 2] * p->R[2 * 3 + b]) * s[b];
      }
      p->tc = atan2(mc[0], mc[2]);
      p->pc = mc[2] != 0 ? atan(mc[1] / mc[2]) : (mc[1] > 0 ? M_PI / 2 : (mc[1] < 0 ? -M_PI / 2 : 0));
      /* J: derivatives of (atan2(x, z), atan(y / z)) at the mean */
      double rxz = mc[0] * mc[0] + mc[2] * mc[2], ryz = mc[1] * mc[1] + mc[2] * mc[2];
      double jt[3] = {mc[2] / rxz, 0, -mc[0] / rxz}, jp[3] = {0, mc[2] / ryz, -mc[1] / ryz};
      double vt[3], vp[3];
      for (int k = 0; k < 3; ++k) {
        vt[k] = jt[0] * A[0 * 3 + k] + jt[1] * A[1 * 3 + k] + jt[2] * A[2 * 3 + k];
        vp[k] = jp[0] * A[0 * 3 + k] + jp[1] * A[1 * 3 + k] + jp[2] * A[2 * 3 + k];
      }
      double pt = vw->fov_x / vw->width, pp = vw->fov_y / vw->height;
      double c00 = vt[0] * vt[0] + vt[1] * vt[1] + vt[2] * vt[2] + 0.3 * pt * pt;
      double c01 = vt[0] * vp[0] + vt[1] * vp[1] + vt[2] * vp[2];
      double c11 = vp[0] * vp[0] + vp[1] * vp[1] + vp[2] * vp[2] + 0.3 * pp * pp;
      double det = c00 * c11 - c01 * c01;
      p->ia = c11 / det; p->ib = -c01 / det; p->ic = c00 / det;
      double mid = 0.5 * (p->ia + p->ic), dd = sqrt(0.25 * (p->ia - p->ic) * (p->ia - p->ic) + p->ib * p->ib);
      p->icmax = mid + dd;
      p->ccond = c00 * c11 / det;
      p->mdist = sqrt(mc[0] * mc[0] + mc[1] * mc[1] + mc[2] * mc[2]);
    }
  }
}

static void pixel_dir(const orc_view* v, int px, int py, double d[3]) {
  double th = col_angle(v, px + 0.5);
  double ph = row_angle(v, py + 0.5);
  double dc[3] = {sin(th) * cos(ph), cos(th) * sin(ph), cos(th) * cos(ph)};
  double nn = sqrt(dc[0] * dc[0] + dc[1] * dc[1] + dc[2] * dc[2]);
  for (int a = 0; a < 3; ++a) dc[a] /= nn;
  /* world direction R^T d_c */
  for (int a = 0; a < 3; ++a) d[a] = v->R[0 * 3 + a] * dc[0] + v->R[1 * 3 + a] * dc[1] + v->R[2 * 3 + a] * dc[2];
}

typedef struct {
  uint32_t key;
  int64_t g;
  double alpha, araw, kappa, tstar;
  double u[3], m[3], uu;
  double band; /* FP32 error bound of kappa for this pair */
  int clamped;
  int in64;    /* contributes in FP64 */
  int flag;    /* within the FP32 error band of a contribution decision */
} contrib;

static int contrib_cmp(const void* a, const void* b) {
  const contrib* x = (const contrib*)a;
  const contrib* y = (const contrib*)b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  return x->g < y->g ? -1 : (x->g > y->g ? 1 : 0);
}

/* Bound on how far FP32 evaluation can move kappa.  First order: the ray
 * direction carries a few units in the last place (|grad_d kappa| * 2^-21,
 * four ulps of a unit vector's components), the camera-space mean a few
 * ulps of |mu| + |o| (|grad_mu kappa| * 2^-21 of that), plus a relative
 * floor for the rounding of log2(sigma) and of the exponent.  Both
 * gradients come from the chain of the cookbook appendix (dkappa/dd_u,
 * dkappa/do_u) mapped through W^T.  Float32 evaluations of kappa near the
 * threshold, with inputs moved by up to 4 ulps, stay within half of it (the
 * band's own test). */
static double kappa_band(const gprep* p, const double u[3], const double m[3], double uu, double kappa,
                         const double o[3]) {
  const double* ou = p->ou;
  const double* W = p->W;
  double gm[3] = {2 * m[0] / uu, 2 * m[1] / uu, 2 * m[2] / uu};
  double dku[3] = {gm[1] * ou[2] - gm[2] * ou[1], gm[2] * ou[0] - gm[0] * ou[2], gm[0] * ou[1] - gm[1] * ou[0]};
  double kk = 2 * kappa / uu;
  for (int a = 0; a < 3; ++a) dku[a] -= kk * u[a];
  double dko[3] = {u[1] * gm[2] - u[2] * gm[1], u[2] * gm[0] - u[0] * gm[2], u[0] * gm[1] - u[1] * gm[0]};
  double gd2 = 0, gmu2 = 0;
  for (int q = 0; q < 3; ++q) {
    double a = W[0 * 3 + q] * dku[0] + W[1 * 3 + q] * dku[1] + W[2 * 3 + q] * dku[2];
    double b = W[0 * 3 + q] * dko[0] + W[1 * 3 + q] * dko[1] + W[2 * 3 + q] * dko[2];
    gd2 += a * a;
    gmu2 += b * b;
  }
  double mu_mag = p->dist + sqrt(o[0] * o[0] + o[1] * o[1] + o[2] * o[2]);
  /* second order: kappa = |P o_u|^2 with P = I - u u^T / |u|^2 the projection
   off d_u, so a move delta of o_u adds |P delta|^2 beyond the linear term,
   and a turn of d_u by the angle e = |P delta_u| / |d_u| adds at most
   |o_u|^2 e^2.  Both moves are W times a move of the mean or of the
   direction, so |P W| (Frobenius) bounds the amplification.  They matter
   only for needles, whose W amplifies input rounding by 1/s_min across every
   direction; for a disk P removes the amplified normal axis (nearly d_u). */
  double wf = 0, r2 = ou[0] * ou[0] + ou[1] * ou[1] + ou[2] * ou[2];
  for (int q = 0; q < 3; ++q) {
    const double ud = (u[0] * W[0 * 3 + q] + u[1] * W[1 * 3 + q] + u[2] * W[2 * 3 + q]) / uu;
    for (int a = 0; a < 3; ++a) {
      const double pw = W[a * 3 + q] - u[a] * ud;
      wf += pw * pw;
    }
  }
  wf = sqrt(wf) * 1.01;
  const double dou = 0x1p-21 * mu_mag * wf, dang = 0x1p-21 * wf / sqrt(uu);
  return 0x1p-21 * sqrt(gd2) + 0x1p-21 * mu_mag * sqrt(gmu2) + dou * dou + r2 * dang * dang +
         1e-6 * (p->lam2 > 1 ? p->lam2 : 1);
}

/* The contribution rule for one (ray, Gaussian) pair, FP64: not culled,
 * closest approach in front of the camera, kappa <= lambda_i^2, and (fixed
 * lambda) alpha_raw >= alpha_min. */
static int pair_contributes64(const gprep* p, const orc_opts* op, const double d[3]) {
  if (!p->active) return 0;
  const double* W = p->W;
  double u[3];
  for (int a = 0; a < 3; ++a) u[a] = W[a * 3 + 0] * d[0] + W[a * 3 + 1] * d[1] + W[a * 3 + 2] * d[2];
  const double* ou = p->ou;
  double m[3] = {ou[1] * u[2] - ou[2] * u[1], ou[2] * u[0] - ou[0] * u[2], ou[0] * u[1] - ou[1] * u[0]};
  double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  double kappa = (m[0] * m[0] + m[1] * m[1] + m[2] * m[2]) / uu;
  double od = ou[0] * u[0] + ou[1] * u[1] + ou[2] * u[2];
  double tstar = -od / uu;
  double araw = p->sigma * exp(-0.5 * kappa);
  return tstar > 0 && kappa <= p->lam2 && !(op->lambda_mode == 1 && !(araw >= op->alpha_min));
}

static int contrib_cmp(const void* a, const void* b);

/* The splat opacity's pairs of one ray (px, py) of a BEAP grid: Gaussians
 * whose FP32 association rectangle holds the ray's half-tile, with
 * alpha_raw = sigma exp(-m / 2), m = d^T C^-1 d the conic distance of the
 * ray's BEAP angles from the mean's (theta difference wrapped to (-pi, pi]).
 * A pair contributes iff alpha_raw >= alpha_min, i.e. m <= 2 ln(sigma /
 * alpha_min); it is flagged when m is within the FP32 band of that
 * threshold: angle differences good to 2e-6 rad (2 sqrt(m |C^-1|) 2e-6 +
 * |C^-1| 4e-12), the conic's rounding amplified by its condition
 * (1e-6 c00 c11 / det (1 + m)), and 1e-4 (1 + m) relative.  The depth is the
 * mean's camera distance.  In (key, index) order. */
static int64_t gather_splat(const gprep* P, int64_t n, const orc_opts* op, const orc_view* v, int px, int py,
                            contrib** buf, int64_t* cap) {
  const double th = col_angle(v, px + 0.5), ph = row_angle(v, py + 0.5);
  const int hx = px / HALF, hy = py / HALF;
  int64_t cnt = 0;
  for (int64_t g = 0; g < n; ++g) {
    const gprep* p = &P[g];
    if (!p->active || !p->vis || hx < p->hx0 || hx > p->hx1 || hy < p->hy0 || hy > p->hy1) continue;
    double dt = th - p->tc;
    if (dt > M_PI) dt -= 2 * M_PI;
    if (dt < -M_PI) dt += 2 * M_PI;
    const double dp = ph - p->pc;
    const double m = p->ia * dt * dt + 2 * p->ib * dt * dp + p->ic * dp * dp;
    const double araw = p->sigma * exp(-0.5 * m);
    const double thr = 2.0 * log(p->sigma / op->alpha_min);
    const double band = 2 * sqrt((m > 0 ? m : 0) * p->icmax) * 2e-6 + p->icmax * 4e-12 +
                        1e-6 * p->ccond * (1 + m) + 1e-4 * (1 + m);
    const int in64 = araw >= op->alpha_min;
    const int flag = fabs(m - thr) <= band;
    if (!in64 && !flag) continue;
    if (cnt == *cap) {
      *cap = *cap ? *cap * 2 : 256;
      *buf = (contrib*)realloc(*buf, sizeof(contrib) * (size_t)*cap);
    }
    contrib* c = &(*buf)[cnt++];
    memset(c, 0, sizeof *c);
    c->key = p->key;
    c->g = g;
    c->araw = araw;
    c->clamped = araw > op->alpha_max;
    c->alpha = c->clamped ? op->alpha_max : araw;
    c->kappa = m;
    c->tstar = p->mdist;
    c->band = band;
    c->in64 = in64;
    c->flag = flag;
  }
  qsort(*buf, (size_t)cnt, sizeof(contrib), contrib_cmp);
  return cnt;
}

/* Collects, in (key, index) order, every pair that contributes in FP64 and
 * every pair whose contribution decision lies within the FP32 error band of
 * its threshold (flag = 1: FP32 may decide either way). */
static int64_t gather(const gprep* P, int64_t n, const orc_opts* op, const double o[3], const double d[3],
                      contrib** buf, int64_t* cap) {
  int64_t cnt = 0;
  for (int64_t g = 0; g < n; ++g) {
    const gprep* p = &P[g];
    if (!p->active) continue;
    const double* W = p->W;
    double u[3];
    for (int a = 0; a < 3; ++a) u[a] = W[a * 3 + 0] * d[0] + W[a * 3 + 1] * d[1] + W[a * 3 + 2] * d[2];
    const double* ou = p->ou;
    double m[3] = {ou[1] * u[2] - ou[2] * u[1], ou[2] * u[0] - ou[0] * u[2], ou[0] * u[1] - ou[1] * u[0]};
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    double kappa = (m[0] * m[0] + m[1] * m[1] + m[2] * m[2]) / uu;
    double od = ou[0] * u[0] + ou[1] * u[1] + ou[2] * u[2];
    double tstar = -od / uu;
    double band = kappa_band(p, u, m, uu, kappa, o);
    int flag = 0;
    if (fabs(kappa - p->lam2) <= band && tstar > 0) flag = 1;
    if (fabs(od) <= 1e-4 * sqrt(uu) * sqrt(ou[0] * ou[0] + ou[1] * ou[1] + ou[2] * ou[2]) && kappa <= p->lam2 + band)
      flag = 1;
    double araw = p->sigma * exp(-0.5 * kappa);
    if (op->lambda_mode == 1 && fabs(araw - op->alpha_min) <= 1e-3 * op->alpha_min) flag = 1;
    const int in64 = tstar > 0 && kappa <= p->lam2 && !(op->lambda_mode == 1 && !(araw >= op->alpha_min));
    if (!in64 && !flag) continue;
    if (cnt == *cap) {
      *cap = *cap ? *cap * 2 : 256;
      *buf = (contrib*)realloc(*buf, sizeof(contrib) * (size_t)*cap);
    }
    contrib* c = &(*buf)[cnt++];
    c->key = p->key;
    c->g = g;
    c->araw = araw;
    c->clamped = araw > op->alpha_max;
    c->alpha = c->clamped ? op->alpha_max : araw;
    c->kappa = kappa;
    c->tstar = tstar;
    c->band = band;
    for (int a = 0; a < 3; ++a) { c->u[a] = u[a]; c->m[a] = m[a]; }
    c->uu = uu;
    c->in64 = in64;
    c->flag = flag;
  }
  qsort(*buf, (size_t)cnt, sizeof(contrib), contrib_cmp);
  return cnt;
}

/* Keeps only the pairs that contribute in FP64 (order preserved). */
static int64_t keep_contributors(contrib* buf, int64_t cnt) {
  int64_t k = 0;
  for (int64_t i = 0; i < cnt; ++i)
    if (buf[i].in64) buf[k++] = buf[i];
  return k;
}

static void camera_centre(const orc_view* v, double o[3]) {
  for (int a = 0; a < 3; ++a) o[a] = -(v->R[0 * 3 + a] * v->t[0] + v->R[1 * 3 + a] * v->t[1] + v->R[2 * 3 + a] * v->t[2]);
}

/* Relative FP32 error that one compositing step adds to the transmittance:
 * the step's alpha carries the kappa band (d alpha / alpha = -d kappa / 2),
 * amplified by 1 / (1 - alpha) in T (1 - alpha), plus rounding. */
static double step_trel(const contrib* c) {
  return (c->clamped ? 0.0 : c->alpha * 0.5 * c->band) / (1 - c->alpha) + 0x1p-22;
}

/* A termination decision T_next < T_min within the FP32 error band. */
static int term_ambiguous(double Tn, double trel, double t_min) {
  return fabs(Tn - t_min) <= (trel + 0x1p-20) * Tn;
}

/* Outcome (RGB, depth, T) of one sequence of decisions. */
typedef struct {
  double rgb[3], depth, trans;
} leaf_t;

/* Enumeration of the decision branches of one ray.  Every decision that lies
 * within the FP32 error band (a flagged contribution: pair in or out; a
 * termination step: stop or go on) is taken both ways; every other decision
 * is the FP64 one.  Each complete sequence is a leaf.  At most maxb leaves
 * are stored; n counts them all (n > maxb: the enumeration stopped). */
typedef struct {
  const contrib* buf;
  int64_t cnt;
  const gprep* P;
  const orc_opts* op;
  leaf_t* leaves;
  int64_t maxb, n;
} branch_walk;

static void emit_leaf(branch_walk* b, double c0, double c1, double c2, double D, double T) {
  if (b->leaves && b->n < b->maxb) {
    leaf_t* l = &b->leaves[b->n];
    l->rgb[0] = c0; l->rgb[1] = c1; l->rgb[2] = c2;
    l->depth = D;
    l->trans = T;
  }
  b->n++;
}

/* Front to back from contributor i with transmittance T, colour (c0, c1, c2),
 * depth D and accumulated relative error trel.  Recursion happens only at
 * branch points, so its depth is bounded by the number of leaves. */
static void walk_branches(branch_walk* b, int64_t i, double T, double c0, double c1, double c2, double D,
                          double trel) {
  const double t_min = b->op->t_min;
  for (; i < b->cnt; ++i) {
    if (b->n > b->maxb) return;
    const contrib* c = &b->buf[i];
    if (c->flag) walk_branches(b, i + 1, T, c0, c1, c2, D, trel);  /* the pair left out */
    else if (!c->in64) continue;
    const double Tn = T * (1 - c->alpha);
    const double tr = trel + step_trel(c);
    if (t_min > 0) {
      if (term_ambiguous(Tn, tr, t_min)) emit_leaf(b, c0, c1, c2, D, T);  /* stop here; also go on */
      else if (Tn < t_min) { emit_leaf(b, c0, c1, c2, D, T); return; }
    }
    const double w = c->alpha * T;
    const gprep* p = &b->P[c->g];
    c0 += w * p->col[0];
    c1 += w * p->col[1];
    c2 += w * p->col[2];
    D += w * c->tstar;
    T = Tn;
    trel = tr;
  }
  emit_leaf(b, c0, c1, c2, D, T);
}

/*
 * Render a list of BEAP pixels (linear index y * width + x) of one view.
 * Outputs per pixel: rgb[3], depth (sum of w_i t*_i), final transmittance and
 * the number of composited Gaussians, all from the FP64 decisions; amb = 1
 * when some decision on that path lies within the FP32 error band (a
 * contribution threshold, or the termination test), so that FP32 may take
 * another branch.  With leaves != NULL (maxb slots of 5 doubles per pixel:
 * rgb, depth, T) every branch's outcome is listed and nleaves[t] holds
 * their number (above maxb: too many to list).
 */
int orc_render(const orc_scene* sc, const orc_view* v, const orc_opts* op, int64_t npix,
               const int64_t* pix, double* rgb, double* depth, double* trans, int32_t* ncomp,
               int32_t* amb, int64_t maxb, double* leaves, int64_t* nleaves, int nthreads) {
  int64_t n = sc->n;
  orc_assoc* as = (orc_assoc*)malloc(sizeof(orc_assoc) * (size_t)(n > 0 ? n : 1));
  gprep* P = (gprep*)malloc(sizeof(gprep) * (size_t)(n > 0 ? n : 1));
  if (!as || !P) { free(as); free(P); return -1; }
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
  orc_assoc_fp32(sc, v, op, as);
  prep_gaussians(sc, v, op, P, as);
  double o[3];
  camera_centre(v, o);
#pragma omp parallel
  {
    contrib* buf = NULL;
    int64_t cap = 0;
#pragma omp for schedule(dynamic, 16)
    for (int64_t t = 0; t < npix; ++t) {
      int px = (int)(pix[t] % v->width), py = (int)(pix[t] / v->width);
      double d[3];
      pixel_dir(v, px, py, d);
      int64_t cnt = op->splat ? gather_splat(P, n, op, v, px, py, &buf, &cap) : gather(P, n, op, o, d, &buf, &cap);
      /* the FP64 path; a branch point on it means other outcomes exist */
      int a_flag = 0;
      double T = 1, C[3] = {0, 0, 0}, D = 0;
      double trel = 0;
      int32_t nc = 0;
      for (int64_t i = 0; i < cnt; ++i) {
        const contrib* c = &buf[i];
        if (c->flag) a_flag = 1;
        if (!c->in64) continue;
        double Tn = T * (1 - c->alpha);
        trel += step_trel(c);
        if (op->t_min > 0) {
          if (term_ambiguous(Tn, trel, op->t_min)) a_flag = 1;
          if (Tn < op->t_min) break;
        }
        double w = c->alpha * T;
        const gprep* p = &P[c->g];
        for (int ch = 0; ch < 3; ++ch) C[ch] += w * p->col[ch];
        D += w * c->tstar;
        T = Tn;
        ++nc;
      }
      for (int ch = 0; ch < 3; ++ch) rgb[3 * t + ch] = C[ch];
      depth[t] = D;
      trans[t] = T;
      ncomp[t] = nc;
      amb[t] = a_flag;
      if (leaves) {
        branch_walk bw = {buf, cnt, P, op, (leaf_t*)(leaves + (size_t)t * (size_t)maxb * 5), maxb, 0};
        if (a_flag) {
          walk_branches(&bw, 0, 1.0, 0.0, 0.0, 0.0, 0.0, 0.0);
        } else {
          emit_leaf(&bw, C[0], C[1], C[2], D, T);
        }
        nleaves[t] = bw.n;
      }
    }
    free(buf);
  }
  free(as);
  free(P);
  return 0;
}

/*
 * Gradients of L with respect to the raw parameters (mean, linear scale, raw
 * quaternion, raw opacity, SH coefficients), given dL/dRGB on the listed
 * pixels of one view.  Outputs are FP64 SoA arrays in the scene layout,
 * overwritten.
 */
int orc_render_backward(const orc_scene* sc, const orc_view* v, const orc_opts* op, int64_t npix,
                        const int64_t* pix, const double* dl_drgb, double* g_mean, double* g_scale,
                        double* g_quat, double* g_opac, double* g_sh, int nthreads) {
  int64_t n = sc->n;
  int deg = sc->sh_degree, K = (deg + 1) * (deg + 1);
  orc_assoc* as = (orc_assoc*)malloc(sizeof(orc_assoc) * (size_t)(n > 0 ? n : 1));
  gprep* P = (gprep*)malloc(sizeof(gprep) * (size_t)(n > 0 ? n : 1));
  if (!as || !P) { free(as); free(P); return -1; }
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
  orc_assoc_fp32(sc, v, op, as);
  prep_gaussians(sc, v, op, P, as);
  double o[3];
  camera_centre(v, o);
  enum { NA = 16 }; /* dsigma, dcol[3], dou[3], dW_rc[9] */
  int nt = 1;
#ifdef _OPENMP
  nt = omp_get_max_threads();
#endif
  double* acc = (double*)calloc((size_t)nt * (size_t)n * NA, sizeof(double));
  if (!acc) { free(as); free(P); return -1; }
#pragma omp parallel
  {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    double* A = acc + (size_t)tid * (size_t)n * NA;
    contrib* buf = NULL;
    int64_t cap = 0;
    double* Tb = NULL;
    int64_t tcap = 0;
#pragma omp for schedule(dynamic, 16)
    for (int64_t t = 0; t < npix; ++t) {
      int px = (int)(pix[t] % v->width), py = (int)(pix[t] / v->width);
      double d[3];
      pixel_dir(v, px, py, d);
      int64_t cnt = keep_contributors(buf, gather(P, n, op, o, d, &buf, &cap));
      if (cnt > tcap) { tcap = cnt; Tb = (double*)realloc(Tb, sizeof(double) * (size_t)tcap); }
      /* forward pass storing T before each composited Gaussian */
      double T = 1;
      int64_t nc = 0;
      for (int64_t i = 0; i < cnt; ++i) {
        double Tn = T * (1 - buf[i].alpha);
        if (op->t_min > 0 && Tn < op->t_min) break;
        Tb[i] = T;
        T = Tn;
        ++nc;
      }
      const double* G = dl_drgb + 3 * t;
      double Cb[3] = {0, 0, 0};
      for (int64_t i = nc - 1; i >= 0; --i) {
        const contrib* c = &buf[i];
        const gprep* p = &P[c->g];
        double* a = A + (size_t)c->g * NA;
        double Ti = Tb[i], al = c->alpha;
        double dl_da = 0;
        for (int ch = 0; ch < 3; ++ch) {
          a[1 + ch] += al * Ti * G[ch];
          dl_da += G[ch] * Ti * (p->col[ch] - Cb[ch]);
        }
        for (int ch = 0; ch < 3; ++ch) Cb[ch] = al * p->col[ch] + (1 - al) * Cb[ch];
        if (c->clamped) continue;
        double e = exp(-0.5 * c->kappa);
        a[0] += dl_da * e;                       /* d alpha / d sigma */
        double dk = dl_da * (-0.5 * c->araw);    /* dL / dkappa */
        const double* u = c->u;
        const double* ou = p->ou;
        double gm[3];
        for (int q = 0; q < 3; ++q) gm[q] = 2.0 * c->m[q] / c->uu;
        /* dkappa/do_u = d_u x g_m ; dkappa/dd_u = -(2 kappa/|d_u|^2) d_u + g_m x o_u */
        double gou[3] = {u[1] * gm[2] - u[2] * gm[1], u[2] * gm[0] - u[0] * gm[2], u[0] * gm[1] - u[1] * gm[0]};
        double gdu[3] = {gm[1] * ou[2] - gm[2] * ou[1], gm[2] * ou[0] - gm[0] * ou[2], gm[0] * ou[1] - gm[1] * ou[0]};
        double kk = 2.0 * c->kappa / c->uu;
        for (int q = 0; q < 3; ++q) gdu[q] -= kk * u[q];
        for (int q = 0; q < 3; ++q) a[4 + q] += dk * gou[q];
        for (int r = 0; r < 3; ++r)
          for (int q = 0; q < 3; ++q) a[7 + r * 3 + q] += dk * gdu[r] * d[q]; /* RC: g_du d^T */
      }
    }
    free(buf);
    free(Tb);
  }
  /* reduce thread accumulators into thread 0's slab */
  for (int tt = 1; tt < nt; ++tt) {
    double* B = acc + (size_t)tt * (size_t)n * NA;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n * NA; ++i) acc[i] += B[i];
  }
  /* Gaussian-wise stage */
#pragma omp parallel for schedule(static)
  for (int64_t g = 0; g < n; ++g) {
    const gprep* p = &P[g];
    const double* a = acc + (size_t)g * NA;
    double mu[3] = {sc->mean[g], sc->mean[n + g], sc->mean[2 * n + g]};
    double om[3] = {o[0] - mu[0], o[1] - mu[1], o[2] - mu[2]};
    double dW[9];
    for (int r = 0; r < 3; ++r)
      for (int q = 0; q < 3; ++q) dW[r * 3 + q] = a[7 + r * 3 + q] + a[4 + r] * om[q]; /* + PC: g_ou (o-mu)^T */
    double dmu[3];
    for (int q = 0; q < 3; ++q) dmu[q] = -(p->W[0 * 3 + q] * a[4] + p->W[1 * 3 + q] * a[5] + p->W[2 * 3 + q] * a[6]);
    /* colour: SH coefficients and the view direction */
    double Y[16], dY[16][3];
    sh_basis(deg, p->v, Y, dY);
    double dv[3] = {0, 0, 0};
    for (int ch = 0; ch < 3; ++ch) {
      double dc = p->craw[ch] > 0 ? a[1 + ch] : 0.0;
      for (int k = 0; k < K; ++k) {
        g_sh[(size_t)(k * 3 + ch) * n + g] = Y[k] * dc;
        double cf = (double)sc->sh[(size_t)(k * 3 + ch) * n + g];
        for (int q = 0; q < 3; ++q) dv[q] += cf * dY[k][q] * dc;
      }
    }
    if (p->dist > 0) {
      double vd = p->v[0] * dv[0] + p->v[1] * dv[1] + p->v[2] * dv[2];
      for (int q = 0; q < 3; ++q) dmu[q] += (dv[q] - p->v[q] * vd) / p->dist;
    }
    for (int q = 0; q < 3; ++q) g_mean[(size_t)q * n + g] = dmu[q];
    /* scale: dW_ij/ds_i = -R_ji / s_i^2 */
    for (int i = 0; i < 3; ++i) {
      double acc_s = 0;
      for (int j = 0; j < 3; ++j) acc_s += dW[i * 3 + j] * (-p->R[j * 3 + i] / (p->s[i] * p->s[i]));
      g_scale[(size_t)i * n + g] = acc_s;
    }
    /* rotation: the four dW/dq matrices of the unit quaternion */
    double qr = p->qh[0], qi = p->qh[1], qj = p->qh[2], qk = p->qh[3];
    const double* s = p->s;
    double Dr[9] = {0, qk / s[0], -qj / s[0], -qk / s[1], 0, qi / s[1], qj / s[2], -qi / s[2], 0};
    double Di[9] = {0, qj / s[0], qk / s[0], qj / s[1], -2 * qi / s[1], qr / s[1], qk / s[2], -qr / s[2], -2 * qi / s[2]};
    double Dj[9] = {-2 * qj / s[0], qi / s[0], -qr / s[0], qi / s[1], 0, qk / s[1], qr / s[2], qk / s[2], -2 * qj / s[2]};
    double Dk[9] = {-2 * qk / s[0], qr / s[0], qi / s[0], -qr / s[1], -2 * qk / s[1], qj / s[1], qi / s[2], qj / s[2], 0};
    double dqh[4] = {0, 0, 0, 0};
    for (int e = 0; e < 9; ++e) {
      dqh[0] += 2 * Dr[e] * dW[e];
      dqh[1] += 2 * Di[e] * dW[e];
      dqh[2] += 2 * Dj[e] * dW[e];
      dqh[3] += 2 * Dk[e] * dW[e];
    }
    double proj = dqh[0] * qr + dqh[1] * qi + dqh[2] * qj + dqh[3] * qk;
    g_quat[(size_t)0 * n + g] = (dqh[0] - qr * proj) / p->qn;
    g_quat[(size_t)1 * n + g] = (dqh[1] - qi * proj) / p->qn;
    g_quat[(size_t)2 * n + g] = (dqh[2] - qj * proj) / p->qn;
    g_quat[(size_t)3 * n + g] = (dqh[3] - qk * proj) / p->qn;
    g_opac[g] = a[0];
  }
  free(acc);
  free(as);
  free(P);
  return 0;
}

/* Ray-level query for tests: kappa, t*, sigma exp(-kappa/2), lambda_i^2 of
 * one (ray, Gaussian) pair in FP64 (cross-product form), given a world
 * direction d, and the FP32 error band of kappa used to flag decisions. */
int orc_pair(const orc_scene* sc, const orc_view* v, const orc_opts* op, int64_t g, const double d[3],
             double out[5]) {
  int64_t n = sc->n;
  int K = (sc->sh_degree + 1) * (sc->sh_degree + 1);
  double m1[3], s1v[3], q1[4], o1[1], sh1[48];
  for (int a = 0; a < 3; ++a) { m1[a] = sc->mean[(size_t)a * n + g]; s1v[a] = sc->scale[(size_t)a * n + g]; }
  for (int a = 0; a < 4; ++a) q1[a] = sc->quat[(size_t)a * n + g];
  o1[0] = sc->opacity[g];
  for (int k = 0; k < K * 3; ++k) sh1[k] = sc->sh[(size_t)k * n + g];
  orc_scene s1 = *sc;
  s1.n = 1; s1.mean = m1; s1.scale = s1v; s1.quat = q1; s1.opacity = o1; s1.sh = sh1;
  orc_assoc as;
  orc_assoc_fp32(&s1, v, op, &as);
  gprep p;
  prep_gaussians(&s1, v, op, &p, &as);
  const double* W = p.W;
  double u[3];
  for (int a = 0; a < 3; ++a) u[a] = W[a * 3 + 0] * d[0] + W[a * 3 + 1] * d[1] + W[a * 3 + 2] * d[2];
  const double* ou = p.ou;
  double m[3] = {ou[1] * u[2] - ou[2] * u[1], ou[2] * u[0] - ou[0] * u[2], ou[0] * u[1] - ou[1] * u[0]};
  double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  out[0] = (m[0] * m[0] + m[1] * m[1] + m[2] * m[2]) / uu;
  out[1] = -(ou[0] * u[0] + ou[1] * u[1] + ou[2] * u[2]) / uu;
  out[2] = p.sigma * exp(-0.5 * out[0]);
  out[3] = p.lam2;
  double o[3];
  camera_centre(v, o);
  out[4] = kappa_band(&p, u, m, uu, out[0], o);
  return 0;
}

/* Brute-force contribution mask for tiny inputs: mask[t * n + g] = 1 iff the
 * pair (pixel pix[t], Gaussian g) satisfies the contribution rule (culling,
 * t* > 0, kappa <= lambda_i^2, and alpha >= alpha_min in fixed-lambda mode),
 * independent of the compositing order and of early termination. */
int orc_contrib_mask(const orc_scene* sc, const orc_view* v, const orc_opts* op, int64_t npix,
                     const int64_t* pix, uint8_t* mask) {
  int64_t n = sc->n;
  orc_assoc* as = (orc_assoc*)malloc(sizeof(orc_assoc) * (size_t)(n > 0 ? n : 1));
  gprep* P = (gprep*)malloc(sizeof(gprep) * (size_t)(n > 0 ? n : 1));
  if (!as || !P) { free(as); free(P); return -1; }
  orc_assoc_fp32(sc, v, op, as);
  prep_gaussians(sc, v, op, P, as);
  double o[3];
  camera_centre(v, o);
#pragma omp parallel
  {
    contrib* buf = NULL;
    int64_t cap = 0;
#pragma omp for schedule(dynamic, 16)
    for (int64_t t = 0; t < npix; ++t) {
      int px = (int)(pix[t] % v->width), py = (int)(pix[t] / v->width);
      double d[3];
      pixel_dir(v, px, py, d);
      int64_t cnt = keep_contributors(buf, gather(P, n, op, o, d, &buf, &cap));
      memset(mask + (size_t)t * (size_t)n, 0, (size_t)n);
      for (int64_t i = 0; i < cnt; ++i) mask[(size_t)t * (size_t)n + (size_t)buf[i].g] = 1;
    }
    free(buf);
  }
  free(as);
  free(P);
  return 0;
}

/* For (tile, Gaussian) pairs of one view: 1 when some ray of the 16x16 tile
 * (clipped to the grid) meets the contribution rule with the Gaussian (FP64,
 * no early termination), else 0.  The tests use it to prove that pairs left
 * out of the GPU association list are ones no ray of their tile can see
 * (the list is the PBF list of Sec. 3.2 minus such pairs). */
int orc_tile_pairs_contribute(const orc_scene* sc, const orc_view* v, const orc_opts* op, int64_t npairs,
                              const int32_t* tiles, const int64_t* gids, uint8_t* out, int nthreads) {
  int64_t n = sc->n;
  orc_assoc* as = (orc_assoc*)malloc(sizeof(orc_assoc) * (size_t)(n > 0 ? n : 1));
  gprep* P = (gprep*)malloc(sizeof(gprep) * (size_t)(n > 0 ? n : 1));
  if (!as || !P) { free(as); free(P); return -1; }
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
  orc_assoc_fp32(sc, v, op, as);
  prep_gaussians(sc, v, op, P, as);
  const int tw = (v->width + 15) / 16;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < npairs; ++i) {
    const gprep* p = &P[gids[i]];
    const int tx = tiles[i] % tw, ty = tiles[i] / tw;
    int hit = 0;
    for (int py = ty * 16; py < ty * 16 + 16 && py < v->height && !hit; ++py)
      for (int px = tx * 16; px < tx * 16 + 16 && px < v->width && !hit; ++px) {
        double d[3];
        pixel_dir(v, px, py, d);
        hit = pair_contributes64(p, op, d);
      }
    out[i] = (uint8_t)hit;
  }
  free(as);
  free(P);
  return 0;
}
