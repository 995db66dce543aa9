// Host-side camera and camera-sub-frustum tables (computed in FP64, rounded to
// FP32 once), the conservative lambda^2 table and the valid-ray mask.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "geer.h"
#include "geer_common.h"
#include "tables.h"

namespace geer {

static float round_up_f32(double x) {
  float f = (float)x;
  if ((double)f < x) f = std::nextafter(f, INFINITY);
  return f;
}

static uint32_t f2u(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  return u;
}
static float u2f(uint32_t u) {
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

// Buckets of 2^17 consecutive FP32 bit patterns of sigma; each stores
// 2 ln(sigma_hi / alpha_min) at the bucket's upper end, inflated by 2^-10,
// rounded up: an upper bound of the opacity-aware lambda^2 over the bucket.
void lambda_table(float alpha_min, std::vector<float>& tab, int& lo, int& n) {
  lo = (int)(f2u(alpha_min) >> kLamShift);
  int hi = (int)(f2u(16.0f) >> kLamShift);
  n = hi - lo + 1;
  tab.resize(n);
  for (int b = 0; b < n; ++b) {
    double top = (double)u2f((uint32_t)(lo + b + 1) << kLamShift);
    double l2 = 2.0 * std::log(top / (double)alpha_min);
    if (l2 < 0) l2 = 0;
    tab[b] = round_up_f32(l2 * (1.0 + 1.0 / 1024.0));
  }
}

float lambda_fixed_hat(float lambda_fixed) {
  double l = (double)lambda_fixed;
  return round_up_f32(l * l * (1.0 + 1.0 / 1024.0));
}

// Half-tile edges: columns in the xi = 1 mirrored space tan(theta / 2), rows
// in tan(phi); entry h is the boundary at pixel 8h (the last at the image edge).
void edge_tables(const geer_view& v, std::vector<float>& ex, std::vector<float>& ey) {
  int w = v.width, h = v.height;
  int nx = (w + kHalf - 1) / kHalf, ny = (h + kHalf - 1) / kHalf;
  ex.resize(nx + 1);
  ey.resize(ny + 1);
  for (int i = 0; i <= nx; ++i) {
    int b = i < nx ? i * kHalf : w;
    double th = -v.fov_x / 2 + (double)b * v.fov_x / w;
    ex[i] = (float)std::tan(th / 2);
  }
  for (int j = 0; j <= ny; ++j) {
    int b = j < ny ? j * kHalf : h;
    double ph = -v.fov_y / 2 + (double)b * v.fov_y / h;
    ey[j] = (float)std::tan(ph);
  }
}

// Per-column (sin, cos) of theta and per-row (sin, cos) of phi at BEAP pixel
// centres (Sec. 3.3): the ray direction is (sin t cos p, cos t sin p, cos t cos p).
void direction_tables(const geer_view& v, std::vector<float>& dx, std::vector<float>& dy) {
  dx.resize(2 * (size_t)v.width);
  dy.resize(2 * (size_t)v.height);
  for (int i = 0; i < v.width; ++i) {
    double th = -v.fov_x / 2 + (i + 0.5) * v.fov_x / v.width;
    dx[2 * i] = (float)std::sin(th);
    dx[2 * i + 1] = (float)std::cos(th);
  }
  for (int j = 0; j < v.height; ++j) {
    double ph = -v.fov_y / 2 + (j + 0.5) * v.fov_y / v.height;
    dy[2 * j] = (float)std::sin(ph);
    dy[2 * j + 1] = (float)std::cos(ph);
  }
}

void view_constants(const geer_view& v, ViewDev& d) {
  std::memset(&d, 0, sizeof d);
  for (int a = 0; a < 9; ++a) d.Rc[a] = (float)v.R[a];
  for (int a = 0; a < 3; ++a) d.tc[a] = (float)v.t[a];
  for (int a = 0; a < 3; ++a)
    d.campos[a] = (float)(-(v.R[0 * 3 + a] * v.t[0] + v.R[1 * 3 + a] * v.t[1] + v.R[2 * 3 + a] * v.t[2]));
  d.width = v.width;
  d.height = v.height;
  d.tiles_x = (v.width + kTile - 1) / kTile;
  d.tiles_y = (v.height + kTile - 1) / kTile;
  d.nhx = (v.width + kHalf - 1) / kHalf;
  d.nhy = (v.height + kHalf - 1) / kHalf;
}

// Valid-ray mask through the native camera model (App. E); the incidence
// angle atan2(|xy|, z) keeps rays beyond 90 degrees well defined.
void valid_mask(const geer_view& v, uint8_t* mask) {
  for (int j = 0; j < v.height; ++j) {
    double ph = -v.fov_y / 2 + (j + 0.5) * v.fov_y / v.height;
    for (int i = 0; i < v.width; ++i) {
      double th = -v.fov_x / 2 + (i + 0.5) * v.fov_x / v.width;
      double x = std::sin(th) * std::cos(ph), y = std::cos(th) * std::sin(ph), z = std::cos(th) * std::cos(ph);
      double nn = std::sqrt(x * x + y * y + z * z);
      x /= nn; y /= nn; z /= nn;
      double u, w;
      bool ok;
      if (v.model == GEER_CAM_PINHOLE) {
        ok = z > 0;
        u = v.fx * x / z + v.cx;
        w = v.fy * y / z + v.cy;
      } else {
        double rxy = std::hypot(x, y);
        double inc = std::atan2(rxy, z);
        double i2 = inc * inc;
        double td = inc * (1 + v.k[0] * i2 + v.k[1] * i2 * i2 + v.k[2] * i2 * i2 * i2 + v.k[3] * i2 * i2 * i2 * i2);
        double cx = rxy > 0 ? x / rxy : 0.0, cy = rxy > 0 ? y / rxy : 0.0;
        u = v.fx * td * cx + v.cx;
        w = v.fy * td * cy + v.cy;
        ok = true;
      }
      ok = ok && u >= 0 && u < v.width && w >= 0 && w < v.height;
      mask[(size_t)j * v.width + i] = ok ? 1 : 0;
    }
  }
}

}  // namespace geer
