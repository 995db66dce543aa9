// Internal layouts shared by the host code and the gfx950 kernels of libgeer.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace geer {

constexpr int kTile = 16;      // CSF tile edge (pixels)
constexpr int kHalf = 8;       // half-tile edge: one wave64 covers an 8x8 half-tile
constexpr int kLamShift = 17;  // lambda^2 table: buckets of 2^17 float bit patterns

// Per-view constants, uploaded once per render call.
struct ViewDev {
  float Rc[9];        // world-to-camera rotation (FP32)
  float tc[3];        // world-to-camera translation (FP32)
  float campos[3];    // camera centre in world space (SH view direction)
  int32_t width, height;
  int32_t tiles_x, tiles_y;
  int32_t nhx, nhy;   // half-tile columns / rows
  int32_t tile_base;  // first global tile id of this view
  int32_t pix_base;   // first pixel of this view in the concatenated outputs
  int32_t ex_off, ey_off;  // offsets of the edge tables in the edge buffer
  int32_t dx_off, dy_off;  // offsets of the direction tables (2 floats per entry)
  float dil_t, dil_p;      // splat low-pass dilation: 0.3 x the squared angular pixel pitch
  int32_t pad_[3];
};
static_assert(sizeof(ViewDev) % 16 == 0, "ViewDev alignment");

// Render record of one (Gaussian, view) item: 64 bytes, read wave-uniformly.
//   G rows (9): r e1^T Wc, r e2^T Wc, -o_u^T Wc   (rotated canonical frame)
//   c0 = -r^2 log2(e) / 2, lsig = log2(sigma), c1 = r^2
//   rgb (3), qmax (kappa / r^2 bound of the fixed-lambda mode, +inf otherwise)
struct alignas(16) Record {
  float g[9];
  float c0, lsig, c1;
  float rgb[3];
  float qmax;
};
static_assert(sizeof(Record) == 64, "Record is 64 bytes");

struct Opts {
  float alpha_min, alpha_max, t_min, lambda_fixed;
  int32_t lambda_mode;
  float lam2_fixed;   // conservative lambda_fixed^2 for the PBF
  float kmax_fixed;   // lambda_fixed^2 for the contribution test
  int32_t lam_lo;     // first bucket index of the lambda^2 table
  int32_t lam_n;      // number of buckets
  float log2_amin;    // log2(alpha_min), for the half-tile cone test
  int32_t cone_cull;  // 1: skip entries whose contribution cone misses the half-tile
  int32_t assoc;      // association: 0 PBF, else a projected-footprint box (kAssoc*)
  int32_t splat;      // 1: render-time splat opacity (2D conic in BEAP angles) instead of the exact one
  int32_t pad_[3];
};

// Associations compared against the PBF (the splatting baselines): the box of
// a projected 2D footprint in BEAP angles, from the local affine (EWA) or
// unscented (UT) projection of the Gaussian, either square (lambda times the
// largest standard deviation) or snug (the footprint ellipse's axis-aligned
// extents).
constexpr int kAssocPBF = 0, kAssocEWA = 1, kAssocEWASnug = 2, kAssocUT = 3, kAssocUTSnug = 4;

// One Adam step: learning rates of the mean, log-scale, quaternion, opacity
// logit and SH groups; moment decays, epsilon and the bias corrections
// 1 / (1 - b1^t), 1 / (1 - b2^t) of step t.
struct AdamParams {
  float lr[5];
  float b1, b2, eps, c1, c2;
  float omb1, omb2;  // 1 - b1 and 1 - b2 formed in double, rounded once (1 - 0.999f is 1.3e-5 off 1e-3)
};

// Refinement thresholds: mean-gradient norm averaged over the steps that saw
// a Gaussian; the largest log scale above which a Gaussian is split rather
// than cloned; the opacity logit below which it is pruned.
struct DensifyParams {
  float grad_threshold, split_log_scale, prune_logit;
};

// Heavy-tile work list of a frame (device buffers): up to hmax tile ids (a
// capacity no frame can exceed), a flag per tile, the device count of listed
// tiles, and the number of heavy wave slots that walk the list.
struct HeavyTiles {
  uint32_t* list;
  uint32_t* flag;
  unsigned long long* count;
  int hmax;
  int hslots;
  unsigned long long* evals;  // the render's evaluated-pair counters (kEvalSlots, kEvalStride apart)
};

// The render's evaluated-pair count is gathered through kEvalSlots counters
// on separate 128-byte lines (one atomic per wave on a single word was the
// render's bottleneck: such atomics serialise).
constexpr int kEvalSlots = 64;
constexpr int kEvalStride = 16;       // u64 words between counters
constexpr int kEvalTallyShift = 44;   // a counter's top 20 bits count the waves that added to it

__host__ __device__ inline uint32_t pack16(int lo, int hi) { return (uint32_t)lo | ((uint32_t)hi << 16); }

}  // namespace geer
