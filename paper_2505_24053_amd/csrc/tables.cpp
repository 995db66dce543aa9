// Host-side camera and camera-sub-frustum tables (computed in FP64, rounded to
// FP32 once), the conservative lambda^2 table and the valid-ray mask.
#include <algorithm>
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
// BEAP angles of a column / row boundary or centre at pixel coordinate x: the
// uniform BEAP grid, or (native pinhole grid) the angle whose tangent is the
// normalised image coordinate.
static double theta_at(const geer_view& v, double x) {
  return v.grid == GEER_GRID_NATIVE ? std::atan((x - v.cx) / v.fx) : -v.fov_x / 2 + x * v.fov_x / v.width;
}
static double phi_at(const geer_view& v, double y) {
  return v.grid == GEER_GRID_NATIVE ? std::atan((y - v.cy) / v.fy) : -v.fov_y / 2 + y * v.fov_y / v.height;
}

void edge_tables(const geer_view& v, std::vector<float>& ex, std::vector<float>& ey) {
  int w = v.width, h = v.height;
  int nx = (w + kHalf - 1) / kHalf, ny = (h + kHalf - 1) / kHalf;
  ex.resize(nx + 1);
  ey.resize(ny + 1);
  for (int i = 0; i <= nx; ++i) {
    int b = i < nx ? i * kHalf : w;
    double th = theta_at(v, (double)b);
    ex[i] = (float)std::tan(th / 2);
  }
  for (int j = 0; j <= ny; ++j) {
    int b = j < ny ? j * kHalf : h;
    double ph = phi_at(v, (double)b);
    ey[j] = (float)std::tan(ph);
  }
}

// Per-column (sin, cos) of theta and per-row (sin, cos) of phi at BEAP pixel
// centres (Sec. 3.3): the ray direction is (sin t cos p, cos t sin p, cos t cos p).
void direction_tables(const geer_view& v, std::vector<float>& dx, std::vector<float>& dy) {
  dx.resize(2 * (size_t)v.width);
  dy.resize(2 * (size_t)v.height);
  for (int i = 0; i < v.width; ++i) {
    double th = theta_at(v, i + 0.5);
    dx[2 * i] = (float)std::sin(th);
    dx[2 * i + 1] = (float)std::cos(th);
  }
  for (int j = 0; j < v.height; ++j) {
    double ph = phi_at(v, j + 0.5);
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
  // the splat opacity's low-pass filter: 0.3 squared pixels, in BEAP angles
  const double pt = v.fov_x / v.width, pp = v.fov_y / v.height;
  d.dil_t = (float)(0.3 * pt * pt);
  d.dil_p = (float)(0.3 * pp * pp);
}

// Valid-ray mask through the native camera model (App. E); the incidence
// angle atan2(|xy|, z) keeps rays beyond 90 degrees well defined.
void valid_mask(const geer_view& v, uint8_t* mask) {
  if (v.grid == GEER_GRID_NATIVE) {  // the sensor's own pixels
    std::memset(mask, 1, (size_t)v.width * v.height);
    return;
  }
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

// Incidence angle theta of a KB distorted radius td = theta (1 + k1 theta^2 +
// ... + k4 theta^8) (App. E), on the increasing branch from 0; false when td
// lies beyond that branch's maximum (no ray lands there).  Safeguarded
// Newton in FP64: the bracket [lo, hi] always holds the root.
static bool kb_incidence(double td, const double k[4], double& theta) {
  auto f = [&](double t) {
    const double t2 = t * t;
    return t * (1 + t2 * (k[0] + t2 * (k[1] + t2 * (k[2] + t2 * k[3])))) - td;
  };
  auto df = [&](double t) {
    const double t2 = t * t;
    return 1 + t2 * (3 * k[0] + t2 * (5 * k[1] + t2 * (7 * k[2] + t2 * 9 * k[3])));
  };
  // end of the increasing branch on [0, pi]
  double hi = M_PI;
  for (int i = 1; i <= 4096; ++i) {
    const double t = M_PI * i / 4096;
    if (df(t) <= 0) {
      hi = t;
      break;
    }
  }
  if (f(hi) < 0) return false;
  double lo = 0, t = std::min(td, hi);
  for (int it = 0; it < 100; ++it) {
    const double ft = f(t);
    if (ft == 0) break;
    if (ft < 0) lo = t; else hi = t;
    double nt = t - ft / df(t);
    if (!(nt > lo && nt < hi)) nt = 0.5 * (lo + hi);
    if (std::fabs(nt - t) <= 1e-16 * std::max(1.0, t)) {
      t = nt;
      break;
    }
    t = nt;
  }
  theta = t;
  return true;
}

// Sampling map of the native sensor (App. E models) in the BEAP grid of v:
// per native pixel (i, j), centre (i + 1/2, j + 1/2) in sensor coordinates,
// the ray through it (pinhole: ((u - cx) / fx, (v - cy) / fy, 1); KB and
// equidistant: incidence from the distorted radius, azimuth of the offset),
// its BEAP angles theta = atan2(x, z), phi = atan(y / z), and their
// continuous grid position x = (theta + fov_x / 2) w / fov_x - 1/2 (likewise
// y).  Positions within half a pixel outside the grid are clamped to it;
// beyond that, or where no ray lands, the entry is (-1, -1, 0, 0).  Entry:
// i0, j0 (top-left neighbour, i0 <= w - 2 unless w = 1) and the bilinear
// fractions as float bits.
void reproject_map(const geer_view& v, int nw, int nh, std::vector<int32_t>& map) {
  map.assign((size_t)4 * nw * nh, 0);
  const int W = v.width, H = v.height;
  for (int j = 0; j < nh; ++j)
    for (int i = 0; i < nw; ++i) {
      int32_t* e = &map[4 * ((size_t)j * nw + i)];
      e[0] = e[1] = -1;
      const double mx = (i + 0.5 - v.cx) / v.fx, my = (j + 0.5 - v.cy) / v.fy;
      double x, y, z;
      if (v.model == GEER_CAM_PINHOLE) {
        x = mx; y = my; z = 1.0;
      } else {
        const double td = std::hypot(mx, my);
        double th;
        if (!kb_incidence(td, v.k, th)) continue;
        if (td > 0) {
          x = std::sin(th) * mx / td;
          y = std::sin(th) * my / td;
        } else {
          x = y = 0.0;
        }
        z = std::cos(th);
      }
      const double tb = std::atan2(x, z);
      const double pb = z != 0 ? std::atan(y / z) : (y > 0 ? M_PI / 2 : (y < 0 ? -M_PI / 2 : 0.0));
      double gx = (tb + v.fov_x / 2) * W / v.fov_x - 0.5;
      double gy = (pb + v.fov_y / 2) * H / v.fov_y - 0.5;
      if (!(gx >= -0.5 && gx <= W - 0.5 && gy >= -0.5 && gy <= H - 0.5)) continue;
      gx = std::min(std::max(gx, 0.0), (double)(W - 1));
      gy = std::min(std::max(gy, 0.0), (double)(H - 1));
      const int i0 = std::min((int)std::floor(gx), std::max(W - 2, 0));
      const int j0 = std::min((int)std::floor(gy), std::max(H - 2, 0));
      const float fx = (float)(gx - i0), fy = (float)(gy - j0);
      e[0] = i0;
      e[1] = j0;
      std::memcpy(&e[2], &fx, 4);
      std::memcpy(&e[3], &fy, 4);
    }
}

}  // namespace geer
