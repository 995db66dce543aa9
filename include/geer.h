/*
 * geer.h -- C ABI of the MI355X exact Gaussian ray renderer.
 *
 * The library implements the rendering hot path of 3DGEER (arXiv 2505.24053):
 *   (a) per-Gaussian particle bounding frustum (PBF) as a rectangle of BEAP
 *       tiles (Sec. 3.2 and App. D: Eq. planeTrans, ellipsoid_tangent,
 *       solve_tan, pbf-cov3d, tan_sol, and the xi = 1 mirror of Eq. aabb),
 *   (b) tile/Gaussian key generation and a per-tile depth sort
 *       (Alg. 1: DuplicateWithKeys, SortByKeys, IdentifyFrustumRanges),
 *   (c) per-pixel front-to-back compositing (Eq. color) with the closed-form
 *       ray opacity sigma exp(-kappa/2), kappa = |o_u x d_u|^2 / |d_u|^2
 *       (Eq. transmit / trans:cano / mahdist_comp),
 * over BEAP rays (Sec. 3.3, App. E), and its gradient (App. C).
 *
 * Conventions shared by every call:
 *   - All array pointers named "device" are HIP device pointers owned by the
 *     caller; the library never frees them and never keeps them after the
 *     call returns (a frame keeps its own copies of what the backward needs).
 *   - Scene arrays are FP32 structure-of-arrays, row-major, N = scene->n:
 *       mean [3][N], scale [3][N] (linear standard deviations),
 *       quat [4][N] as (r, i, j, k), any non-zero norm (normalised inside),
 *       opacity [N] in (0, 1], sh [(deg+1)^2 * 3][N] with row k*3 + channel.
 *   - Image outputs are planar FP32. For V views of sizes W_v x H_v they are
 *     concatenated view after view: rgb holds 3*W_v*H_v floats per view
 *     ([3][H][W]), depth and trans hold W_v*H_v floats per view ([H][W]).
 *   - Cameras: BEAP grid of width x height pixels spanning fov_x x fov_y
 *     radians; pixel (i, j) looks along theta_i = -fov_x/2 + (i+1/2) fov_x/w,
 *     phi_j = -fov_y/2 + (j+1/2) fov_y/h, direction (sin t cos p, cos t sin p,
 *     cos t cos p) normalised, in OpenCV camera axes; pose x_cam = R x + t.
 *     Requirements: 0 < fov_x <= 2 pi, 0 < fov_y <= pi (phi is the principal
 *     angle atan(y / z), so its grid spans at most the open half-turn).
 *   - Every call returns a geer_status and never aborts. Argument errors are
 *     detected on the host before any launch. Work is enqueued on `stream`
 *     (a hipStream_t, 0 for the default stream) unless a call says it
 *     synchronises.
 */
#ifndef GEER_H
#define GEER_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GEER_OK = 0,
  GEER_ERR_INVALID_ARG = 1, /* bad pointer, size, camera or option */
  GEER_ERR_OOM = 2,         /* device or host allocation failed */
  GEER_ERR_CAPACITY = 3,    /* more than 2^30 - 16 items (Gaussians x views) or list entries */
  GEER_ERR_HIP = 4,         /* a HIP runtime call failed; see geer_last_error */
  GEER_ERR_UNSUPPORTED = 5, /* feature not available in this build */
  GEER_ERR_STALLED = 6      /* a bounded device-side wait of the association sort gave
                               up (decoupled look-back spin limit): the outputs of that
                               forward are invalid and must be rendered again */
} geer_status;

typedef enum { GEER_CAM_PINHOLE = 0, GEER_CAM_EQUIDISTANT = 1, GEER_CAM_KB = 2 } geer_cam_model;

/* One view: camera model, native intrinsics (used for the valid-ray mask of
 * the loss), ray grid, pose.  The camera models are those of App. E
 * (pinhole; Kannala-Brandt with k1..k4; equidistant = KB with k = 0).
 * grid GEER_GRID_BEAP: the BEAP grid of width x height rays over
 * fov_x x fov_y (below).  grid GEER_GRID_NATIVE (pinhole only): the native
 * pixels of the pinhole sensor, width x height, pixel (i, j) looking along
 * ((i + 1/2 - cx) / fx, (j + 1/2 - cy) / fy, 1); fov_x / fov_y are then
 * ignored.  Since x / z = tan(theta) and y / z = tan(phi) for a pinhole ray
 * (App. E), its columns and rows are lines of constant BEAP angles, so each
 * 16 x 16 tile's sub-frustum is the angular box of its rays and the same
 * association and render apply unchanged; only the edge and direction tables
 * differ. */
#define GEER_GRID_BEAP 0
#define GEER_GRID_NATIVE 1
typedef struct {
  int32_t model;         /* geer_cam_model */
  int32_t width, height; /* grid in pixels, 1 .. 65536 */
  int32_t grid;          /* GEER_GRID_BEAP (0) or GEER_GRID_NATIVE (1) */
  double fx, fy, cx, cy; /* native pinhole / fisheye intrinsics */
  double k[4];           /* KB distortion k1..k4 (0 for pinhole, equidistant) */
  double fov_x, fov_y;   /* BEAP angular extents in radians */
  double R[9];           /* world-to-camera rotation, row-major */
  double t[3];           /* world-to-camera translation */
} geer_view;

/* A scene resident in device memory (not copied; layout in the header). */
typedef struct {
  int64_t n;         /* number of Gaussians, 0 .. 2^28 */
  int32_t sh_degree; /* 0 .. 3 */
  int32_t reserved;  /* must be 0 */
  const float* mean;    /* device [3][n] */
  const float* scale;   /* device [3][n], > 0 */
  const float* quat;    /* device [4][n] */
  const float* opacity; /* device [n] */
  const float* sh;      /* device [(deg+1)^2*3][n] */
} geer_scene;

/* Rendering options.  A pair (ray, Gaussian) contributes iff the camera is
 * outside the Gaussian's 3-sigma ellipsoid (culling, App. B), the closest
 * approach lies in front of the camera, and
 *   lambda_mode 0 (default): alpha_raw = sigma exp(-kappa/2) >= alpha_min,
 *     i.e. kappa <= 2 ln(sigma / alpha_min); the PBF uses that lambda;
 *   lambda_mode 1: kappa <= lambda_fixed^2 and alpha_raw >= alpha_min; the
 *     PBF uses lambda_fixed (the paper's "typically 3").
 * alpha = min(alpha_raw, alpha_max); compositing stops before the first
 * Gaussian that would take the transmittance below t_min (t_min = 0: never).
 * flags: GEER_OPT_NO_CONE_CULL keeps every (tile, Gaussian) pair of the PBF
 * rectangles in the association list and makes the render and its backward
 * evaluate every (ray, entry) pair whose half-tile rectangle test passes.
 * Without it, pairs whose contribution cone meets no ray of the tile (list)
 * or of the half-tile (render) are skipped; the outputs are the same bits
 * either way (the flag is for verification and measurement of the cull). */
#define GEER_OPT_NO_CONE_CULL 1
/* Association (bits 1-3 of flags): the PBF rectangle (0, default), or, for
 * comparison with the splatting pipelines (App. on EWA splatting; the
 * association-method tables), the box of a projected footprint in BEAP
 * angles: EWA -- angles of the mean and J Sigma_c J^T, J the Jacobian of
 * (atan2(x, z), atan(y / z)) at the mean (local affine approximation); UT --
 * the seven unscented sigma points mu_c, mu_c +- sqrt(3) m_k (m_k the columns
 * of the camera-space factor R_c R S) projected exactly, weights of alpha = 1,
 * beta = 2, kappa = 0.  Square box: centre +- lambda sqrt(largest eigenvalue);
 * snug box: the ellipse's axis-aligned extents lambda sqrt(C_00),
 * lambda sqrt(C_11); lambda is the PBF's.  These boxes are not supersets of
 * the contributing rays: pairs outside them are lost from the image. */
#define GEER_OPT_ASSOC_EWA (1 << 1)
#define GEER_OPT_ASSOC_EWA_SNUG (2 << 1)
#define GEER_OPT_ASSOC_UT (3 << 1)
#define GEER_OPT_ASSOC_UT_SNUG (4 << 1)
#define GEER_OPT_ASSOC_MASK (7 << 1)
/* Render-time splat opacity (the local-affine ablation): each pair's alpha is
 * sigma exp(-m / 2), m = d^T C^-1 d with d the ray's BEAP angles minus the
 * mean's (theta wrapped to (-pi, pi]) and C the EWA footprint covariance
 * J Sigma_c J^T plus a 0.3-squared-pixel low-pass term per axis; a pair
 * contributes when that alpha >= alpha_min and the ray's half-tile lies in the
 * (exact) association rectangle; depth accumulates the means' camera
 * distances.  Forward only on BEAP grids (no frame backward, no training
 * plans: GEER_ERR_UNSUPPORTED); the contribution-cone cull is off. */
#define GEER_OPT_SPLAT_ALPHA (1 << 4)
typedef struct {
  float alpha_min;    /* default 1/255, in (0, 1) */
  float alpha_max;    /* default 0.99, in [alpha_min, 1) */
  float t_min;        /* default 1e-4, in [0, 1) */
  float lambda_fixed; /* default 3, > 0 */
  int32_t lambda_mode;
  int32_t flags; /* GEER_OPT_* bits, default 0 */
} geer_opts;

typedef struct geer_ctx geer_ctx;     /* per-device library state */
typedef struct geer_frame geer_frame; /* forward state kept for the backward */
typedef struct geer_plan geer_plan;   /* captured forward or training step (below) */

/* Statistics of one forward, counted on the device. */
typedef struct {
  int64_t n_items;     /* Gaussians x views */
  int64_t n_visible;   /* items whose PBF meets at least one tile */
  int64_t n_entries;   /* (tile, Gaussian) pairs of the association list */
  int64_t n_tiles;     /* 16x16 tiles over all views */
  int64_t n_pixels;    /* rays over all views */
  int64_t n_evaluated; /* (ray, entry) pairs evaluated by the render kernel */
  int64_t n_candidates;/* (tile, Gaussian) pairs of the PBF rectangles, before the
                          contribution-cone cull removed those no ray of the tile
                          can see (equal to n_entries with GEER_OPT_NO_CONE_CULL) */
} geer_frame_stats;

/* Association buffers a frame can export (for parity checks). */
typedef enum {
  GEER_BUF_RECT = 0,   /* uint32 [items][2]: hx0 | hx1 << 16, hy0 | hy1 << 16 (8-px half-tiles) */
  GEER_BUF_COUNT = 1,  /* uint32 [items]: tiles covered, 0 = not visible */
  GEER_BUF_KEY = 2,    /* uint32 [items]: depth key (bits of FP32 squared camera distance) */
  GEER_BUF_LIST = 3,   /* uint32 [entries]: item id (view * n + gaussian), tile-major, depth order */
  GEER_BUF_RANGES = 4, /* uint32 [tiles + 1]: start of each tile's run in LIST */
  GEER_BUF_NLAST = 5   /* uint32 [pixels]: one past the last LIST index blended by each ray */
} geer_buffer;

/* Creates the library state on HIP device `device`.  *out is set on success. */
geer_status geer_create(int32_t device, geer_ctx** out);
/* Releases every device buffer of the context (frames must be released first). */
void geer_destroy(geer_ctx* ctx);
/* Last error message of the context (static storage, valid until the next call). */
const char* geer_last_error(const geer_ctx* ctx);
/* Fills the defaults listed with geer_opts. */
void geer_default_opts(geer_opts* opts);

/*
 * Forward render of n_views views of one scene (Alg. 1).  All views share one
 * association list (a global tile space), so a batch of views reads the scene
 * once.  rgb, depth, trans: device outputs laid out as in the header; any of
 * depth / trans may be NULL.  If `frame` is not NULL a frame is created and
 * returned that holds what geer_render_backward needs; the caller releases it.
 * The host waits once, mid-call, for the association's entry count, which
 * sizes the list; the depth sort is already enqueued behind it by then, so
 * the device keeps working.  Calls on one context must not overlap.
 */
geer_status geer_render(geer_ctx* ctx, const geer_scene* scene, int32_t n_views, const geer_view* views,
                        const geer_opts* opts, float* rgb, float* depth, float* trans, geer_frame** frame,
                        void* stream);

/*
 * Gradient of a scalar loss given dL/dRGB (device, same layout as rgb) with
 * respect to mean, scale (linear), raw quaternion, opacity and SH
 * coefficients (App. C, with m_u = o_u x d_u).  Gradient arrays are device
 * buffers in the scene layout; accumulate = 0 overwrites them, 1 adds.
 * The scene passed to geer_render must be unchanged.
 */
geer_status geer_render_backward(geer_ctx* ctx, const geer_frame* frame, const float* dl_drgb,
                                 float* g_mean, float* g_scale, float* g_quat, float* g_opacity,
                                 float* g_sh, int32_t accumulate, void* stream);

/*
 * Allocation-free forward, for callers that cannot allocate device memory
 * (serving loops and harnesses that forbid hipMalloc / hipFree).  Same
 * arguments, outputs and bits as geer_render without a frame, but every
 * buffer of the forward lives in one fixed device array of
 * GEER_STATIC_SCRATCH_BYTES inside the library (one per device, held from
 * geer_create until the process ends); the call allocates no device or
 * pinned memory.  The caller owns and passes the scene and the outputs.
 *
 * Sizes: the per-item buffers (about 100 B per Gaussian x view) and the view
 * tables must fit the array with room for at least one list entry, else the
 * call returns GEER_ERR_CAPACITY before any launch; the rest of the array
 * bounds the association list (16 B per PBF pair: a 100k-Gaussian scene in
 * a 1024 x 1024 fisheye view, 2.8M pairs, fits).  A list beyond that is
 * caught on the device: the outputs are background (rgb 0, depth 0, trans 1)
 * and the call returns GEER_ERR_CAPACITY.
 *
 * The call waits for its stream before returning (it reads the entry count
 * and the sort-stall flag back: GEER_ERR_CAPACITY, GEER_ERR_STALLED).  All
 * calls on one device share the array and leave their contents in it; every
 * call clears what must start at zero.  Calls that overlapped on one device
 * would race on the array, so the library serialises its calls per device
 * (a lock held until the call's work has finished).
 */
#define GEER_STATIC_SCRATCH_BYTES (64u * 1024u * 1024u)
geer_status geer_render_static(geer_ctx* ctx, const geer_scene* scene, int32_t n_views,
                               const geer_view* views, const geer_opts* opts, float* rgb, float* depth,
                               float* trans, void* stream);

/*
 * Sort stalls.  Each radix pass of the association waits on earlier blocks
 * with a bounded spin; if it gives up, the outputs of that forward are
 * invalid.  An eager forward (geer_render) records this in a sticky flag of
 * the context; it is reported as GEER_ERR_STALLED, and cleared, by the next
 * geer_render on the context (which then renders nothing), by
 * geer_frame_get_stats, and by geer_check.  Plans report their own launches'
 * stalls through geer_plan_entries.
 */
/* Waits for the work on `stream` and reports (and clears) a stall of any
 * earlier forward on the context: GEER_OK or GEER_ERR_STALLED. */
geer_status geer_check(geer_ctx* ctx, void* stream);
/* Test hook: marks, from the host, the context (plan = NULL) or the plan's
 * last launch (after waiting for it) as if a sort had stalled, so that the
 * reporting paths can be exercised without a device-side stall. */
geer_status geer_debug_mark_stalled(geer_ctx* ctx, geer_plan* plan);
/* Test hook: the number of polls after which the radix passes of later
 * eager forwards on the context give up waiting (limit < 0: the default,
 * about 2^22).  A small limit makes those passes give up for real, so that
 * the handling of a stalled sort can be exercised with every kernel ending
 * normally: such a forward's list is left unordered, its tile ranges are all
 * empty (the frame renders background), and the stall is reported as
 * described above.  Plans keep the limit they were captured with. */
geer_status geer_debug_set_spin_limit(geer_ctx* ctx, int64_t limit);

/* Frees the frame's device state (after any pending backward has completed). */
void geer_frame_release(geer_frame* frame);

/* Device-counted statistics of the frame's forward.  Synchronises. */
geer_status geer_frame_get_stats(const geer_frame* frame, geer_frame_stats* out);

/* Size in bytes of an exportable frame buffer. */
int64_t geer_frame_buffer_bytes(const geer_frame* frame, int32_t which);

/* Copies a frame buffer to host memory `dst` of `bytes` (>= the size above).
 * Synchronises. */
geer_status geer_frame_export(const geer_frame* frame, int32_t which, void* dst, int64_t bytes);

/*
 * Valid-ray mask of a view (host): mask[j * width + i] = 1 iff BEAP ray (i, j)
 * projects onto the native sensor [0, width) x [0, height) through the view's
 * camera model (App. E, with the incidence angle atan2(|xy|, z) so that rays
 * beyond 90 degrees are defined).  `mask` is host memory of width*height bytes.
 */
geer_status geer_valid_mask(const geer_view* view, uint8_t* mask);

/*
 * Native camera-space output (App. E inverse interpolation): resamples a
 * rendered BEAP image of `view` (device, `channels` planes [C][H][W] of the
 * view's grid, e.g. rgb then depth then trans) onto the native sensor of the
 * same camera model, native_width x native_height pixels (0: the view's grid
 * size), into `native` (device, [C][Hn][Wn]).  Native pixel (i, j) has its
 * centre at (i + 1/2, j + 1/2) in the sensor coordinates of fx, fy, cx, cy;
 * its ray is the pinhole back-projection, or for Kannala-Brandt (and
 * equidistant) the incidence angle solving theta (1 + k1 theta^2 + ... +
 * k4 theta^8) = |offset| on the polynomial's increasing branch, at the
 * offset's azimuth.  The ray's BEAP angles give a position in the grid; the
 * output is the bilinear interpolation of the four neighbouring BEAP pixels
 * (positions within half a pixel outside the grid are clamped to it).  Native
 * pixels no BEAP ray of the grid reaches get 0 and valid = 0 (valid: device
 * uint8 [Hn][Wn], may be NULL).  The sampling map is computed once per camera
 * (intrinsics, FoV and sizes; the pose does not enter) in FP64 on the host and
 * cached in the context (at most 16 maps of 16 B per native pixel).
 */
geer_status geer_reproject(geer_ctx* ctx, const geer_view* view, int32_t native_width, int32_t native_height,
                           int32_t channels, const float* beap, float* native, uint8_t* valid, void* stream);

/*
 * L1 loss over valid rays and its gradient (device):
 *   L = sum_{valid rays, channels} |rgb - target| / (3 * n_valid),
 *   dl_drgb = sign(rgb - target) / (3 * n_valid) on valid rays, 0 elsewhere.
 * rgb, target, dl_drgb: [3][pixels]; mask: uint8 [pixels] (device, 1 = valid);
 * loss: device float, written.  n_valid is counted on the device.
 */
geer_status geer_l1_loss(geer_ctx* ctx, int64_t pixels, const float* rgb, const float* target,
                         const uint8_t* mask, float* dl_drgb, float* loss, void* stream);

/*
 * Training step (Alg. "3DGEER Initialization and Training Framework": Adam
 * on the loss gradient, and the periodic refinement of the Gaussian set,
 * driven by view-space mean gradients).  The optimiser holds the raw
 * parameters in one device block of (11 + 3K) rows of n floats -- mean 3, log
 * scale 3, quaternion 4 (any non-zero norm), opacity logit 1, SH 3K (K = (deg
 * + 1)^2, row k*3 + channel) -- and writes the activated scale = exp(log s)
 * [3][n] and opacity = sigmoid(logit) [n] the renderer reads, so a scene of
 * (raw, scale, raw + 6n, opacity, raw + 11n) renders what the optimiser holds.
 * m, v: Adam moments, same shape as raw; accum, count: per-Gaussian
 * densification statistics [n] (sum of mean-gradient norms, steps that saw
 * the Gaussian).  All pointers are device memory owned by the caller.
 */
typedef struct {
  int64_t n;
  int32_t sh_degree;
  int32_t reserved; /* must be 0 */
  float* raw;
  float* scale;
  float* opacity;
  float* m;
  float* v;
  float* accum;
  float* count;
} geer_train_state;

typedef struct {
  double beta1, beta2, eps;                            /* e.g. 0.9, 0.999, 1e-15; 1 - beta and the bias
                                                          corrections are formed in double, then rounded
                                                          once to FP32 */
  float lr_mean, lr_scale, lr_quat, lr_opacity, lr_sh; /* per parameter group */
  int32_t step;                                        /* 1, 2, ...: bias correction of step t */
  int32_t reserved;                                    /* must be 0 */
} geer_adam_opts;

typedef struct {
  float grad_threshold; /* mean-gradient norm averaged over the steps that saw a Gaussian */
  float split_scale;    /* largest linear scale above which a Gaussian is split, not cloned */
  float min_opacity;    /* opacity below which a Gaussian is pruned */
  float split_shrink;   /* scale divisor of split children, e.g. 1.6 */
} geer_densify_opts;

/* Writes state->scale and state->opacity from the raw rows (initialisation). */
geer_status geer_activate(geer_ctx* ctx, const geer_train_state* state, void* stream);

/*
 * One fused Adam step.  g_*: the gradients geer_render_backward (or a
 * training plan) gives for the scene (raw, scale, raw + 6n, opacity, raw +
 * 11n), i.e. with respect to the linear scale and the opacity; they are
 * chained through the activations (d/dlog s = s d/ds, d/dlogit = sigma (1 -
 * sigma) d/dsigma), then m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
 * raw -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps), and the
 * activated scale and opacity are rewritten.  The norm of each Gaussian's
 * mean gradient, when non-zero, is added to accum and 1 to count.  One
 * kernel; accum / count may be NULL (no statistics).
 */
geer_status geer_adam_step(geer_ctx* ctx, const geer_train_state* state, const geer_adam_opts* opts,
                           const float* g_mean, const float* g_scale, const float* g_quat, const float* g_opacity,
                           const float* g_sh, void* stream);

/*
 * Refinement of the Gaussian set (3DGS-style clone / split / prune).  Per
 * Gaussian of `in`: pruned if its opacity is below min_opacity; else, if
 * accum / count >= grad_threshold, cloned (kept plus a copy with zero
 * moments) when its largest scale is at most split_scale, split otherwise
 * into two Gaussians at mean + R S xi_c (xi_c the caller's standard normal
 * draws: noise is device [6][n], rows c*3 + axis for child c) with log scale
 * reduced by log(split_shrink), other parameters copied and zero moments.
 * The decisions compare raw rows with thresholds mapped to raw space
 * (logit(min_opacity), log(split_scale)), in FP32.  Outputs keep the input
 * order (a Gaussian's outputs at its place), statistics reset to zero.
 * `out` holds caller buffers for up to out->n Gaussians (its n on entry is
 * that capacity; 2 * in->n always suffices); on return out->n is the new
 * count n', and every array holds its rows back to back with n' floats each
 * (the layout of a state of n' Gaussians), or GEER_ERR_CAPACITY with nothing
 * written if n' exceeds the capacity.  Synchronises once for the count.
 */
geer_status geer_densify(geer_ctx* ctx, const geer_train_state* in, const geer_densify_opts* opts, const float* noise,
                         geer_train_state* out, void* stream);

/*
 * Stage timing.  While enabled, every geer_render records HIP events on its
 * stream around its stages (the preprocess / PBF kernel; the sort, expansion
 * and ranges; the render kernel) and copies its device counters, and every
 * geer_render_backward records events around its ray-wise replay kernel and
 * its Gaussian-wise kernel and copies the replay's pair count; up to 64
 * records are kept, oldest overwritten.  The forward stages are the Prep /
 * Dup+Sort / Render stages of the paper's timing tables.
 */
typedef struct {
  float ms_preprocess; /* forward: stage (a) kernel; backward: Gaussian-wise kernel */
  float ms_sort;       /* forward: stage (b): depth sort, count scan, expansion, tile sort, ranges */
  float ms_render;     /* forward: stage (c) render kernel; backward: ray-wise replay kernel */
  float ms_total;      /* first event to last (forward: including the host read-back of the list size) */
  int64_t n_entries;   /* forward: association list length */
  int64_t n_evaluated; /* (ray, entry) pairs evaluated by the render (replayed by the backward) kernel */
  int32_t kind;        /* 0: geer_render, 1: geer_render_backward */
  int32_t reserved;
} geer_profile_record;

/* Turns stage timing on (1) or off (0) for the context. */
geer_status geer_set_profiling(geer_ctx* ctx, int32_t enable);
/* Copies the most recent min(max, available) records to `out`, oldest
 * first, and returns how many were copied (negative on error).  Waits for
 * the recorded work to finish.  Clears the records. */
int32_t geer_profile_read(geer_ctx* ctx, geer_profile_record* out, int32_t max);

/*
 * Render plans (batched serving).  A plan fixes a batch shape -- the number
 * of views and each view's BEAP grid size -- the scene, the options, the
 * output buffers and a capacity for the association list.  Its forward is
 * enqueued with capacity-sized launches that read the live counts on the
 * device (no host read-back), captured once into a hipGraph, and replayed by
 * geer_plan_launch with new cameras (model, intrinsics, FoV, pose; the grid
 * sizes must match the plan's).  Results are identical to geer_render of the
 * same views.  A launch waits for the plan's previous launch; concurrent
 * batches use separate plans on separate streams.  A plan's radix passes
 * take their chunks by atomic ticket as blocks start, so plans replayed on
 * several streams at once never wait on each other's blocks.  (Eager forwards
 * and training plans number chunks by block index: their sorts assume no
 * other look-back pass runs beside them; if one does and a pass gives up, the
 * stall is contained and reported as above.)  The scene arrays and the
 * outputs must stay allocated while the plan lives (the scene's values are
 * read by each launch).
 * When a batch's association list exceeds the capacity, that launch renders
 * background and geer_plan_entries reports the overflow.
 */

/* Device workspace a plan of this shape needs, in bytes (same checks as
 * geer_plan_create). */
geer_status geer_plan_workspace_bytes(geer_ctx* ctx, const geer_scene* scene, int32_t n_views,
                                      const geer_view* views, const geer_opts* opts, int64_t entry_capacity,
                                      int64_t* bytes);
/* Captures the plan's graph.  `views` give the shapes (the cameras are taken
 * from each launch); rgb / depth / trans are device outputs as for
 * geer_render, written by every launch (depth, trans may be NULL).
 * entry_capacity bounds the association list.  workspace: caller-owned device
 * memory of at least geer_plan_workspace_bytes, 256-byte aligned, or NULL for
 * a plan-owned allocation.  Plans may share one workspace only if all their
 * launches go to one stream.  Nothing runs on the device until a launch. */
geer_status geer_plan_create(geer_ctx* ctx, const geer_scene* scene, int32_t n_views, const geer_view* views,
                             const geer_opts* opts, int64_t entry_capacity, void* workspace, int64_t workspace_bytes,
                             float* rgb, float* depth, float* trans, geer_plan** out);
/* Training plans (batched training step).  One graph runs, for each view in
 * turn (the next view's association overlapping the current view's render
 * and backward, one association at a time), the forward (keeping only each
 * ray's final transmittance and last
 * blended entry), the L1 loss of that view against its target over the valid
 * rays (mask, or every ray when NULL), and the backward (App. C), so that the
 * gradient arrays receive the gradient of
 *   loss = (1 / n_views) sum_v L1_v,   L1_v = sum |rgb - target| / (3 n_valid_v),
 * and *loss its value.  target / mask / rgb use the concatenated per-view
 * layout of geer_render; the gradient arrays use the scene layout and are
 * overwritten by every launch.  entry_capacity bounds the PBF pairs of each
 * view.  Launched, checked and destroyed with geer_plan_launch,
 * geer_plan_entries (largest view) and geer_plan_destroy.  The scene arrays
 * must stay allocated while the plan lives; their values are read by each
 * launch, so an optimiser may update them in place between launches. */
geer_status geer_train_plan_workspace_bytes(geer_ctx* ctx, const geer_scene* scene, int32_t n_views,
                                            const geer_view* views, const geer_opts* opts, int64_t entry_capacity,
                                            int64_t* bytes);
geer_status geer_train_plan_create(geer_ctx* ctx, const geer_scene* scene, int32_t n_views, const geer_view* views,
                                   const geer_opts* opts, int64_t entry_capacity, void* workspace,
                                   int64_t workspace_bytes, const float* target, const uint8_t* mask, float* rgb,
                                   float* loss, float* g_mean, float* g_scale, float* g_quat, float* g_opacity,
                                   float* g_sh, geer_plan** out);
/* Uploads the cameras of the next batch and replays the graph on `stream`. */
geer_status geer_plan_launch(geer_plan* plan, const geer_view* views, void* stream);
/* Waits for the last launch; reports its count of PBF (tile, Gaussian) pairs
 * -- what entry_capacity bounds, before the contribution-cone cull shortens
 * the list -- and the capacity, and returns GEER_ERR_CAPACITY if they did not
 * fit (the outputs of that launch are then background and must be
 * re-rendered). */
geer_status geer_plan_entries(geer_plan* plan, int64_t* entries, int64_t* capacity);
/* Waits for the last launch and fills the device-counted statistics of its
 * forward (summed over a training plan's views): visible items, PBF pairs
 * (n_candidates), list entries after the cone cull, evaluated (ray, entry)
 * pairs of the render kernel.  Before any launch only the sizes are set. */
geer_status geer_plan_get_stats(geer_plan* plan, geer_frame_stats* out);
/* Device memory the plan allocated itself (0 with a caller workspace). */
int64_t geer_plan_device_bytes(const geer_plan* plan);
/* Waits for the plan's last launch and releases it (before geer_destroy). */
void geer_plan_destroy(geer_plan* plan);

#ifdef __cplusplus
}
#endif

#endif /* GEER_H */
