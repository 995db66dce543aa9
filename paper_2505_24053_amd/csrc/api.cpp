// C ABI of libgeer: argument checks, device memory, and the order of the
// kernels of one forward (Alg. 1):
//   preprocess + PBF  ->  depth sort of visible items  ->  count scan  ->
//   expansion to (tile, item) entries  ->  tile sort  ->  ranges  ->  render.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "geer.h"
#include "geer_common.h"
#include "tables.h"

using namespace geer;

namespace {

struct Block {
  void* p = nullptr;
  size_t bytes = 0;
  hipStream_t stream = nullptr;
};

}  // namespace

struct ProfSlot {
  hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  uint64_t* host_stats = nullptr;  // pinned copy of the frame's device counters
  int kind = 0;                    // 0: forward, 1: backward
};

// Conservative lambda^2 table for one alpha_min (device copy).
struct LamTab {
  float amin = 0.0f;
  float* dev = nullptr;
  int lo = 0, n = 0;
};

// Cached native-sensor sampling map of one camera (intrinsics and grids;
// the pose does not enter).
struct ReprojMap {
  geer_view key{};
  int nw = 0, nh = 0;
  void* dev = nullptr;
};

struct geer_ctx {
  int device = 0;
  std::vector<ReprojMap> maps;  // most recent last
  bool profiling = false;
  std::vector<ProfSlot> prof;  // ring of stage-timing records
  int prof_next = 0, prof_count = 0;
  std::mutex mu;
  std::vector<Block> cache;  // released device blocks, reusable on the same stream
  std::string err;
  std::vector<LamTab> lams;  // lambda^2 tables by alpha_min, kept until destroy
  void* pinned = nullptr;  // host staging for table uploads and read-backs
  size_t pinned_bytes = 0;
  hipEvent_t totals_ready = nullptr;  // an eager forward's count read-back has landed
  int64_t live_frames = 0;
  // Sticky flag (device) of the eager forwards' sorts: set when a look-back
  // gave up; reported (and cleared) by the next forward, geer_check or the
  // statistics of a frame.
  unsigned long long* dev_err = nullptr;
  // look-back polls of the eager forwards' radix passes (a test hook lowers it)
  uint32_t spin_limit = kDefaultSpinLimit;
  // Look-up of the allocation-free forward's fixed device array on this
  // device (geer_create).
  hipError_t static_init = hipErrorNotInitialized;
};

// Largest key count of one sort (status words hold 30-bit counts).
constexpr int64_t kMaxKeys = ((int64_t)1 << 30) - 16;

struct geer_plan {
  geer_ctx* ctx = nullptr;
  geer_scene scene{};
  Opts op{};
  int32_t nviews = 0;
  std::vector<geer_view> shapes;
  int64_t n = 0, items = 0, ntiles = 0, npix = 0, ecap = 0, bytes = 0;
  size_t meta_bytes = 0;
  void* ws = nullptr;     // workspace (device)
  bool owns_ws = false;   // allocated by the plan
  void* meta = nullptr;   // view tables inside the workspace
  uint64_t* stats = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void* staging[2] = {nullptr, nullptr};
  hipEvent_t staged[2] = {nullptr, nullptr};
  bool staged_used[2] = {false, false};
  int next = 0;
  hipEvent_t done = nullptr;
  bool launched = false;
  uint64_t* host_stats = nullptr;
  // training plans: one segment (forward, loss, backward) per view
  int nseg = 0;                 // 0 for a forward plan
  std::vector<size_t> seg_off;  // offset of each view's tables in meta
  int nstat = 1;                // statistics blocks (8 words each), one per segment
};

struct geer_frame {
  geer_ctx* ctx = nullptr;
  hipStream_t stream = nullptr;
  geer_scene scene{};
  Opts op{};
  const float* lam = nullptr;  // lambda^2 table of the forward's alpha_min
  int32_t nviews = 0;
  int64_t n = 0, items = 0, ntiles = 0, npix = 0, entries = 0, visible = 0;
  mutable int64_t kept = -1;  // list length after the cone cull (read from the device on first use)
  size_t edges_off = 0, dtab_off = 0;  // sub-buffers of meta
  std::vector<geer_view> views;
  std::vector<ViewDev> hviews;
  Block meta, recs, rects, keys, counts, list, ranges, nlast, tfinal, stats, heavy_list, heavy_flag;
  int hmax = 0;
};

namespace {

geer_status fail(geer_ctx* c, geer_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return s;
}

#define HIP_TRY(ctx, call)                                                                      \
  do {                                                                                          \
    hipError_t e_ = (call);                                                                     \
    if (e_ != hipSuccess) return fail(ctx, GEER_ERR_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Device memory: a per-context cache of released blocks, reused only on the
// stream that released them (stream order makes the reuse safe).
geer_status acquire(geer_ctx* c, size_t bytes, hipStream_t st, Block& out) {
  bytes = round_up(std::max<size_t>(bytes, 256), 256);
  {
    std::lock_guard<std::mutex> lk(c->mu);
    int best = -1;
    for (int i = 0; i < (int)c->cache.size(); ++i) {
      const Block& b = c->cache[i];
      if (b.stream == st && b.bytes >= bytes && b.bytes <= 2 * bytes + (4u << 20) &&
          (best < 0 || b.bytes < c->cache[best].bytes))
        best = i;
    }
    if (best >= 0) {
      out = c->cache[best];
      c->cache.erase(c->cache.begin() + best);
      return GEER_OK;
    }
  }
  size_t alloc = round_up(bytes, (size_t)2 << 20);
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, alloc);
  if (e != hipSuccess) {
    // free the cache and try once more
    std::vector<Block> drop;
    {
      std::lock_guard<std::mutex> lk(c->mu);
      drop.swap(c->cache);
    }
    (void)hipDeviceSynchronize();
    for (auto& b : drop) (void)hipFree(b.p);
    (void)hipGetLastError();
    e = hipMalloc(&p, alloc);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(c, GEER_ERR_OOM, "device allocation of %zu bytes failed", alloc);
    }
  }
  out.p = p;
  out.bytes = alloc;
  out.stream = st;
  return GEER_OK;
}

void release(geer_ctx* c, Block& b) {
  if (!b.p) return;
  std::lock_guard<std::mutex> lk(c->mu);
  c->cache.push_back(b);
  b = Block{};
}

geer_status ensure_pinned(geer_ctx* c, size_t bytes) {
  if (c->pinned_bytes >= bytes) return GEER_OK;
  if (c->pinned) (void)hipHostFree(c->pinned);
  c->pinned = nullptr;
  c->pinned_bytes = 0;
  size_t alloc = round_up(std::max<size_t>(bytes, 1 << 16), 1 << 16);
  HIP_TRY(c, hipHostMalloc(&c->pinned, alloc, hipHostMallocDefault));
  c->pinned_bytes = alloc;
  return GEER_OK;
}

bool finite_all(const double* p, int n) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

geer_status check_view(geer_ctx* c, const geer_view& v, int i) {
  if (v.model < GEER_CAM_PINHOLE || v.model > GEER_CAM_KB)
    return fail(c, GEER_ERR_INVALID_ARG, "view %d: unknown camera model %d", i, v.model);
  if (v.width < 1 || v.height < 1 || v.width > 65536 || v.height > 65536)
    return fail(c, GEER_ERR_INVALID_ARG, "view %d: grid %dx%d out of range", i, v.width, v.height);
  if (v.grid != GEER_GRID_BEAP && v.grid != GEER_GRID_NATIVE)
    return fail(c, GEER_ERR_INVALID_ARG, "view %d: unknown grid %d", i, v.grid);
  if (v.grid == GEER_GRID_NATIVE) {
    if (v.model != GEER_CAM_PINHOLE)
      return fail(c, GEER_ERR_INVALID_ARG, "view %d: native pixel grids are for pinhole cameras", i);
    if (!(v.fx > 0 && v.fy > 0)) return fail(c, GEER_ERR_INVALID_ARG, "view %d: focal lengths must be positive", i);
  } else if (!(v.fov_x > 0 && v.fov_x <= 2 * M_PI) || !(v.fov_y > 0 && v.fov_y <= M_PI)) {
    return fail(c, GEER_ERR_INVALID_ARG, "view %d: fov (%g, %g) outside (0, 2pi] x (0, pi]", i, v.fov_x, v.fov_y);
  }
  if (!finite_all(v.R, 9) || !finite_all(v.t, 3) || !finite_all(v.k, 4) || !std::isfinite(v.fx) ||
      !std::isfinite(v.fy) || !std::isfinite(v.cx) || !std::isfinite(v.cy))
    return fail(c, GEER_ERR_INVALID_ARG, "view %d: non-finite camera parameter", i);
  return GEER_OK;
}

geer_status check_opts(geer_ctx* c, const geer_opts& o) {
  if (!(o.alpha_min > 0 && o.alpha_min < 1)) return fail(c, GEER_ERR_INVALID_ARG, "alpha_min must be in (0, 1)");
  if (!(o.alpha_max >= o.alpha_min && o.alpha_max < 1))
    return fail(c, GEER_ERR_INVALID_ARG, "alpha_max must be in [alpha_min, 1)");
  if (!(o.t_min >= 0 && o.t_min < 1)) return fail(c, GEER_ERR_INVALID_ARG, "t_min must be in [0, 1)");
  if (o.lambda_mode != 0 && o.lambda_mode != 1) return fail(c, GEER_ERR_INVALID_ARG, "lambda_mode must be 0 or 1");
  if (o.lambda_mode == 1 && !(o.lambda_fixed > 0 && o.lambda_fixed < 100))
    return fail(c, GEER_ERR_INVALID_ARG, "lambda_fixed must be in (0, 100)");
  if ((o.flags & ~(GEER_OPT_NO_CONE_CULL | GEER_OPT_ASSOC_MASK | GEER_OPT_SPLAT_ALPHA)) != 0 ||
      (o.flags & GEER_OPT_ASSOC_MASK) > GEER_OPT_ASSOC_UT_SNUG)
    return fail(c, GEER_ERR_INVALID_ARG, "unknown opts.flags bits");
  return GEER_OK;
}

// The device table for alpha_min, built on first use.  Tables are never freed
// before the context, so frames and plans keep plain pointers to them.
geer_status lambda_dev(geer_ctx* c, float amin, LamTab* out) {
  std::lock_guard<std::mutex> lk(c->mu);
  for (const LamTab& t : c->lams)
    if (t.amin == amin) {
      *out = t;
      return GEER_OK;
    }
  if (c->lams.size() >= 256) return fail(c, GEER_ERR_CAPACITY, "more than 256 distinct alpha_min values");
  std::vector<float> tab;
  LamTab t;
  t.amin = amin;
  lambda_table(amin, tab, t.lo, t.n);
  HIP_TRY(c, hipMalloc(&t.dev, tab.size() * sizeof(float)));
  hipError_t e = hipMemcpy(t.dev, tab.data(), tab.size() * sizeof(float), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(t.dev);
    return fail(c, GEER_ERR_HIP, "lambda table upload: %s", hipGetErrorString(e));
  }
  c->lams.push_back(t);
  *out = t;
  return GEER_OK;
}

void free_frame_buffers(geer_frame* f) {
  geer_ctx* c = f->ctx;
  for (Block* b : {&f->meta, &f->recs, &f->rects, &f->keys, &f->counts, &f->list, &f->ranges, &f->nlast,
                   &f->tfinal, &f->stats, &f->heavy_list, &f->heavy_flag})
    release(c, *b);
}

ProfSlot* prof_slot(geer_ctx* c) {
  if (!c->profiling || c->prof.empty()) return nullptr;
  ProfSlot* s = &c->prof[c->prof_next];
  c->prof_next = (c->prof_next + 1) % (int)c->prof.size();
  c->prof_count = std::min<int>(c->prof_count + 1, (int)c->prof.size());
  return s;
}

void prof_mark(ProfSlot* s, int i, hipStream_t st) {
  if (s) (void)hipEventRecord(s->ev[i], st);
}

// Digits of the tile sort: tile ids 0..ntiles-1 take `bits` significant
// bits, sorted in ceil(bits / 8) passes of equal width (e.g. 13 bits as
// 7 + 7 rather than 8 + 5), so no pass scatters over more buckets than
// needed.
struct TileDigits {
  int passes, bits;
};
TileDigits tile_digits(int64_t ntiles) {
  int tbits = 1;
  while (tbits < 32 && ((int64_t)1 << tbits) < ntiles) ++tbits;
  const int passes = (tbits + 7) / 8;
  return TileDigits{passes, (tbits + passes - 1) / passes};
}

// Tile-sort passes whose digit histograms the expansion counts (0: an upsweep
// counts them).
int hist_passes(int64_t ntiles) {
  const int p = tile_digits(ntiles).passes;
  return p <= 2 ? p : 0;
}


// Device pointers of one forward.
struct FwdBufs {
  const ViewDev* views = nullptr;
  const float* edges = nullptr;
  const float2* dtab = nullptr;
  Record* recs = nullptr;
  uint2* rects = nullptr;
  uint32_t *keys = nullptr, *counts = nullptr;
  uint64_t* stats = nullptr;  // [0] rectangle entries, [1] visible, [2] evaluated pairs, [3] entries before
                              // the guard, [4] sort stall flag, [5] list length after the cone cull,
                              // [6] heavy tiles, [7] stall flag of earlier eager forwards
  unsigned long long* err = nullptr;  // where the sorts flag a stall (null: stats[4])
  unsigned long long* sort_err() const { return err ? err : (unsigned long long*)(stats + 4); }
  // radix passes take their chunks by atomic tickets: set where the forward
  // may run beside look-back passes of other streams (render plans)
  bool tickets = false;
  uint32_t spin_limit = kDefaultSpinLimit;
  // owners of the expansion's blocks, written by the depth order
  uint32_t* owners = nullptr;
  int64_t owners_n = 0;
  uint32_t *ka = nullptr, *va = nullptr, *kb = nullptr, *vb = nullptr;
  uint32_t* hist = nullptr;   // the depth order's work (depth_work_words)
  uint32_t* twork = nullptr;  // the expansion's and tile sort's work (tile_work_words)
  uint32_t *cnt_sorted = nullptr, *tiles_a = nullptr, *tiles_b = nullptr, *items_b = nullptr;
  uint32_t *list = nullptr, *ranges = nullptr, *nlast = nullptr;
  bool depth_work_zeroed = false;  // the preprocess launch clears the depth sort's work area
  float* tfinal = nullptr;
  uint32_t *heavy_list = nullptr, *heavy_flag = nullptr;  // heavy-tile work list
  int hmax = 0;
  float4* tcones = nullptr;  // per-tile cones of the expansion's cull (tile_cone_bytes)
  HeavyTiles heavy() const {
    return HeavyTiles{heavy_list, heavy_flag, (unsigned long long*)(stats + 6), hmax, heavy_slots(hmax),
                      (unsigned long long*)(heavy_list + heavy_evals_offset(hmax))};
  }
};

// Stage (a): zero the counters, then preprocess + PBF of every item.
// With per_view_stats the counters of view v are the 8 words at b.stats + 8v.
void enqueue_preprocess(hipStream_t st, const geer_scene& sc, int32_t nviews, const Opts& op, const float* lam,
                        const FwdBufs& b, bool per_view_stats = false, const unsigned long long* err_in = nullptr,
                        bool defer_colour = false) {
  const int64_t nst = per_view_stats ? 16 * nviews : 16;
  if (b.depth_work_zeroed)
    launch_zero2_u32(st, (uint32_t*)b.stats, nst, b.hist, depth_zero_words(sc.n * nviews));
  else
    launch_fill_u32(st, (uint32_t*)b.stats, nst, 0u);
  launch_preprocess(st, sc.n, nviews, sc.sh_degree, sc.mean, sc.scale, sc.quat, sc.opacity, sc.sh, b.views, op, lam,
                    b.edges, b.recs, b.rects, b.keys, b.counts, (unsigned long long*)b.stats, per_view_stats ? 8 : 0,
                    err_in, defer_colour);
}

// Stage (b): association list; the tile-sorted list ends in b.list.
// First half: the depth order of the visible items and their entry offsets;
// none of it depends on the entry count.  dV: the live visible count on the
// device, or null when nvis_cap is exact.
void enqueue_depth_order(hipStream_t st, int64_t items, int64_t nvis_cap, const unsigned long long* dV,
                         const FwdBufs& b) {
  if (nvis_cap <= 0) return;
  // items in depth order to b.vb, their entry offsets to b.cnt_sorted
  depth_order(st, b.keys, b.counts, items, nvis_cap, dV, b.hist, b.depth_work_zeroed, b.ka, b.va, b.kb, b.vb,
              b.cnt_sorted, b.owners, b.owners_n, b.sort_err(), b.tickets, b.spin_limit);
}

// Second half: per-tile cones, expansion, tile sort and ranges.  dV / dE:
// live counts on the device, or null when nvis_cap / ecap are exact.
void enqueue_tile_lists(hipStream_t st, const Opts& op, int64_t n, int64_t items, int64_t nvis_cap,
                        const unsigned long long* dV, int64_t ecap, const unsigned long long* dE, int64_t ntiles,
                        const FwdBufs& b) {
  unsigned long long* kept = (unsigned long long*)(b.stats + 5);  // list length after the cone cull
  unsigned long long* err = b.sort_err();
  if (nvis_cap > 0 && ecap > 0) {
    // The tile cones' launch also clears the expansion's and the sort's work.
    // Expansion in depth order (entries no ray of their tile can see marked
    // for dropping), then the stable tile-id passes -- the first drops them
    // and counts the kept ones into stats[5] --, arranged so that the sorted
    // items end in b.list: pair P = (tiles_b, list), Q = (tiles_a, items_b);
    // odd pass counts run Q -> P -> Q ..., even ones P -> Q -> P ...
    const TileDigits td = tile_digits(ntiles);
    const int passes = td.passes;
    uint32_t *pt = b.tiles_b, *pi = b.list, *qt = b.tiles_a, *qi = b.items_b;
    uint32_t* tin = (passes % 2 == 1) ? qt : pt;
    uint32_t* iin = (passes % 2 == 1) ? qi : pi;
    uint32_t* at = (passes % 2 == 1) ? pt : qt;
    uint32_t* ai = (passes % 2 == 1) ? pi : qi;
    if (op.cone_cull)
      launch_tile_cones(st, b.views, n > 0 ? (int)(items / n) : 1, b.dtab, ntiles, b.tcones, b.twork,
                        tile_zero_words(ecap));
    else
      launch_fill_u32(st, b.twork, tile_zero_words(ecap), 0u);
    // the expansion also counts the tile digits of the kept entries (one or
    // two passes), which replaces the sort's histogram pass over the list
    const int hpass = hist_passes(ntiles);
    launch_expand(st, b.vb, b.cnt_sorted, nvis_cap, dV, ecap, dE, b.rects, b.views, n, b.tcones, b.recs, op, tin,
                  iin, b.twork, hpass, td.bits, items, ntiles, b.owners);
    tile_sort(st, tin, iin, ecap, dE, kept, passes, td.bits, at, ai, tin, iin, b.twork, hpass, err, b.tickets,
              b.spin_limit);
    uint32_t* tfinal = (passes % 2 == 1) ? at : tin;
    launch_ranges(st, tfinal, ecap, kept, ntiles, b.ranges, b.list, err);
  } else {
    launch_fill_u32(st, b.list, 8, 0u);
    launch_ranges(st, nullptr, 0, nullptr, ntiles, b.ranges);
  }
}

// Stage (b) in one go.  With exact sizes (dyn == false) nvis_cap and ecap are
// the counts read back from the device; otherwise they are capacities and
// every kernel reads the live counts from b.stats.
void enqueue_association(hipStream_t st, const Opts& op, int64_t n, int64_t items, int64_t nvis_cap, int64_t ecap,
                         int64_t ntiles, bool dyn, const FwdBufs& b) {
  const unsigned long long* dE = dyn ? (const unsigned long long*)b.stats : nullptr;
  const unsigned long long* dV = dyn ? (const unsigned long long*)(b.stats + 1) : nullptr;
  if (dyn) launch_capacity_guard(st, (unsigned long long*)b.stats, ecap);
  enqueue_depth_order(st, items, nvis_cap, dV, b);
  enqueue_tile_lists(st, op, n, items, nvis_cap, dV, ecap, dE, ntiles, b);
}

// Stage (c): the render kernel.
void enqueue_render(hipStream_t st, const Opts& op, int64_t ntiles, int32_t nviews, const FwdBufs& b, float* rgb,
                    float* depth, float* trans) {
  if (op.splat) {
    launch_render_splat(st, ntiles, b.views, nviews, b.dtab, b.ranges, b.list, b.rects, b.recs, op, rgb, depth, trans);
    return;
  }
  launch_mark_heavy(st, b.ranges, ntiles, b.views, nviews, b.heavy());
  launch_render(st, op.lambda_mode == 1, ntiles, b.views, nviews, b.dtab, b.ranges, b.list, b.rects, b.recs, op,
                b.heavy(), rgb, depth, trans, b.nlast, b.tfinal, (unsigned long long*)(b.stats + 2));
}

// Host-side per-view tables of a batch, packed as [ViewDev...][edges][dtab].
struct ViewTables {
  std::vector<ViewDev> hv;
  std::vector<float> edges, dtab;
  int64_t ntiles = 0, npix = 0;
  size_t views_bytes = 0, edges_off = 0, dtab_off = 0, bytes = 0;
};

geer_status build_tables(geer_ctx* c, int32_t n_views, const geer_view* views, ViewTables& t) {
  t.hv.assign(n_views, ViewDev{});
  t.edges.clear();
  t.dtab.clear();
  t.ntiles = t.npix = 0;
  for (int i = 0; i < n_views; ++i) {
    view_constants(views[i], t.hv[i]);
    std::vector<float> ex, ey, dx, dy;
    edge_tables(views[i], ex, ey);
    direction_tables(views[i], dx, dy);
    t.hv[i].tile_base = (int32_t)t.ntiles;
    t.hv[i].pix_base = (int32_t)t.npix;
    t.hv[i].ex_off = (int32_t)t.edges.size();
    t.edges.insert(t.edges.end(), ex.begin(), ex.end());
    t.hv[i].ey_off = (int32_t)t.edges.size();
    t.edges.insert(t.edges.end(), ey.begin(), ey.end());
    t.hv[i].dx_off = (int32_t)(t.dtab.size() / 2);
    t.dtab.insert(t.dtab.end(), dx.begin(), dx.end());
    t.hv[i].dy_off = (int32_t)(t.dtab.size() / 2);
    t.dtab.insert(t.dtab.end(), dy.begin(), dy.end());
    t.ntiles += (int64_t)t.hv[i].tiles_x * t.hv[i].tiles_y;
    t.npix += (int64_t)views[i].width * views[i].height;
    if (t.ntiles >= ((int64_t)1 << 31) || t.npix >= ((int64_t)1 << 31))
      return fail(c, GEER_ERR_CAPACITY, "batch exceeds 2^31 tiles or pixels");
  }
  t.views_bytes = sizeof(ViewDev) * t.hv.size();
  t.edges_off = round_up(t.views_bytes, 256);
  t.dtab_off = round_up(t.edges_off + t.edges.size() * sizeof(float), 256);
  t.bytes = t.dtab_off + t.dtab.size() * sizeof(float);
  return GEER_OK;
}

void pack_tables(const ViewTables& t, void* dst) {
  std::memcpy(dst, t.hv.data(), t.views_bytes);
  std::memcpy((char*)dst + t.edges_off, t.edges.data(), t.edges.size() * sizeof(float));
  std::memcpy((char*)dst + t.dtab_off, t.dtab.data(), t.dtab.size() * sizeof(float));
}

Opts make_opts(const LamTab& lt, const geer_opts& o) {
  Opts op{};
  op.alpha_min = o.alpha_min;
  op.alpha_max = o.alpha_max;
  op.t_min = o.t_min;
  op.lambda_fixed = o.lambda_fixed;
  op.lambda_mode = o.lambda_mode;
  op.lam2_fixed = lambda_fixed_hat(o.lambda_fixed);
  op.kmax_fixed = o.lambda_fixed * o.lambda_fixed;
  op.lam_lo = lt.lo;
  op.lam_n = lt.n;
  op.log2_amin = (float)std::log2((double)o.alpha_min);
  op.cone_cull = (o.flags & GEER_OPT_NO_CONE_CULL) ? 0 : 1;
  op.assoc = (o.flags & GEER_OPT_ASSOC_MASK) >> 1;
  op.splat = (o.flags & GEER_OPT_SPLAT_ALPHA) ? 1 : 0;
  if (op.splat) op.cone_cull = 0;  // the cull's cone is the exact opacity's
  return op;
}

geer_status check_scene(geer_ctx* c, const geer_scene* scene) {
  const int64_t n = scene->n;
  if (n < 0 || n > ((int64_t)1 << 28)) return fail(c, GEER_ERR_INVALID_ARG, "scene size %lld", (long long)n);
  if (scene->sh_degree < 0 || scene->sh_degree > 3) return fail(c, GEER_ERR_INVALID_ARG, "sh_degree must be 0..3");
  if (scene->reserved != 0) return fail(c, GEER_ERR_INVALID_ARG, "scene.reserved must be 0");
  if (n > 0 && (!scene->mean || !scene->scale || !scene->quat || !scene->opacity || !scene->sh))
    return fail(c, GEER_ERR_INVALID_ARG, "null scene array");
  return GEER_OK;
}

// Argument checks of a forward (geer_render, geer_render_static).
geer_status check_render_args(geer_ctx* c, const geer_scene* scene, int32_t n_views, const geer_view* views,
                              const geer_opts* opts, const float* rgb) {
  if (!scene || !views || !opts || !rgb) return fail(c, GEER_ERR_INVALID_ARG, "null argument");
  if (n_views < 1 || n_views > 4096) return fail(c, GEER_ERR_INVALID_ARG, "n_views %d out of range", n_views);
  geer_status s;
  if ((s = check_scene(c, scene)) != GEER_OK) return s;
  if ((s = check_opts(c, *opts)) != GEER_OK) return s;
  if (scene->n * n_views >= kMaxKeys) return fail(c, GEER_ERR_CAPACITY, "Gaussians x views exceeds 2^30");
  for (int i = 0; i < n_views; ++i) {
    if ((s = check_view(c, views[i], i)) != GEER_OK) return s;
    if ((opts->flags & GEER_OPT_SPLAT_ALPHA) && views[i].grid != GEER_GRID_BEAP)
      return fail(c, GEER_ERR_UNSUPPORTED, "the splat opacity is defined on BEAP grids");
  }
  return GEER_OK;
}

}  // namespace

extern "C" {

void geer_default_opts(geer_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->alpha_min = 1.0f / 255.0f;
  o->alpha_max = 0.99f;
  o->t_min = 1e-4f;
  o->lambda_fixed = 3.0f;
  o->lambda_mode = 0;
}

geer_status geer_create(int32_t device, geer_ctx** out) {
  if (!out) return GEER_ERR_INVALID_ARG;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
    (void)hipGetLastError();
    return GEER_ERR_INVALID_ARG;
  }
  if (hipSetDevice(device) != hipSuccess) return GEER_ERR_HIP;
  geer_ctx* c = new (std::nothrow) geer_ctx();
  if (!c) return GEER_ERR_OOM;
  c->device = device;
  c->static_init = static_scratch_init(device);
  if (c->static_init != hipSuccess) (void)hipGetLastError();
  if (hipMalloc(&c->dev_err, 256) != hipSuccess || hipMemset(c->dev_err, 0, 256) != hipSuccess) {
    (void)hipGetLastError();
    if (c->dev_err) (void)hipFree(c->dev_err);
    delete c;
    return GEER_ERR_OOM;
  }
  *out = c;
  return GEER_OK;
}

void geer_destroy(geer_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  for (auto& b : c->cache) (void)hipFree(b.p);
  for (auto& ps : c->prof) {
    for (auto& e : ps.ev)
      if (e) (void)hipEventDestroy(e);
    if (ps.host_stats) (void)hipHostFree(ps.host_stats);
  }
  for (LamTab& t : c->lams) (void)hipFree(t.dev);
  if (c->pinned) (void)hipHostFree(c->pinned);
  if (c->totals_ready) (void)hipEventDestroy(c->totals_ready);
  if (c->dev_err) (void)hipFree(c->dev_err);
  for (ReprojMap& m : c->maps) (void)hipFree(m.dev);
  delete c;
}

const char* geer_last_error(const geer_ctx* c) { return c ? c->err.c_str() : "null context"; }

geer_status geer_render(geer_ctx* c, const geer_scene* scene, int32_t n_views, const geer_view* views,
                        const geer_opts* opts, float* rgb, float* depth, float* trans, geer_frame** frame_out,
                        void* stream) {
  if (!c) return GEER_ERR_INVALID_ARG;
  if (frame_out) *frame_out = nullptr;
  geer_status s;
  if ((s = check_render_args(c, scene, n_views, views, opts, rgb)) != GEER_OK) return s;
  const int64_t n = scene->n;
  const int64_t items = n * n_views;
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(c, hipSetDevice(c->device));
  ViewTables tab;
  if ((s = build_tables(c, n_views, views, tab)) != GEER_OK) return s;
  LamTab lt;
  if ((s = lambda_dev(c, opts->alpha_min, &lt)) != GEER_OK) return s;
  const Opts op = make_opts(lt, *opts);
  const int64_t ntiles = tab.ntiles, npix = tab.npix;

  geer_frame* f = new (std::nothrow) geer_frame();
  if (!f) return fail(c, GEER_ERR_OOM, "frame allocation");
  f->ctx = c;
  f->stream = st;
  f->scene = *scene;
  f->op = op;
  f->lam = lt.dev;
  f->nviews = n_views;
  f->n = n;
  f->items = items;
  f->ntiles = ntiles;
  f->npix = npix;
  f->views.assign(views, views + n_views);
  f->hviews = tab.hv;
  f->edges_off = tab.edges_off;
  f->dtab_off = tab.dtab_off;

  // Temporaries of the sort; released at the end of the call.
  Block ka, va, kb, vb, hist, twork, tiles_a, tiles_b, items_b, cnt_sorted, tcones, owners;
  auto cleanup = [&](geer_status st_) {
    for (Block* b : {&ka, &va, &kb, &vb, &hist, &twork, &tiles_a, &tiles_b, &items_b, &cnt_sorted, &tcones, &owners})
      release(c, *b);
    if (st_ != GEER_OK) {
      free_frame_buffers(f);
      delete f;
    }
    return st_;
  };
#define TRY(x)                               \
  do {                                       \
    geer_status s_ = (x);                    \
    if (s_ != GEER_OK) return cleanup(s_);   \
  } while (0)
#define HTRY(call)                                                                                          \
  do {                                                                                                      \
    hipError_t e_ = (call);                                                                                 \
    if (e_ != hipSuccess) return cleanup(fail(c, GEER_ERR_HIP, "%s: %s", #call, hipGetErrorString(e_)));   \
  } while (0)

  TRY(acquire(c, tab.bytes, st, f->meta));
  TRY(ensure_pinned(c, std::max<size_t>(tab.bytes, 64)));
  // The previous call waited for its count read-back, which follows its
  // table upload on the stream, so the staging buffer is free again.
  pack_tables(tab, c->pinned);
  HTRY(hipMemcpyAsync(f->meta.p, c->pinned, tab.bytes, hipMemcpyHostToDevice, st));
  FwdBufs b;
  b.views = (const ViewDev*)f->meta.p;
  b.edges = (const float*)((char*)f->meta.p + tab.edges_off);
  b.dtab = (const float2*)((char*)f->meta.p + tab.dtab_off);

  // ---- stage (a): preprocess + PBF ----
  const int64_t it1 = std::max<int64_t>(items, 1);
  TRY(acquire(c, sizeof(Record) * it1, st, f->recs));
  TRY(acquire(c, sizeof(uint2) * it1, st, f->rects));
  TRY(acquire(c, 4 * it1, st, f->keys));
  TRY(acquire(c, 4 * it1, st, f->counts));
  TRY(acquire(c, 64, st, f->stats));
  b.recs = (Record*)f->recs.p;
  b.rects = (uint2*)f->rects.p;
  b.keys = (uint32_t*)f->keys.p;
  b.counts = (uint32_t*)f->counts.p;
  b.stats = (uint64_t*)f->stats.p;
  // depth-sort buffers, sized for all items (the visible count is read on
  // the device); the preprocess launch also clears the sort's work area
  TRY(acquire(c, 4 * it1, st, ka));
  TRY(acquire(c, 4 * it1, st, va));
  TRY(acquire(c, 4 * it1, st, kb));
  TRY(acquire(c, 4 * it1, st, vb));
  TRY(acquire(c, 4 * (size_t)depth_work_words(it1), st, hist));
  TRY(acquire(c, 4 * it1, st, cnt_sorted));
  TRY(acquire(c, tile_cone_bytes(ntiles), st, tcones));
  // owners of the expansion's blocks: the list is not sized yet, so the table
  // is, for the most entries the items can make (each at most every tile)
  const int64_t ebound = std::min<int64_t>(kMaxKeys, (int64_t)std::min<double>(1e18, (double)it1 * (double)ntiles));
  TRY(acquire(c, 4 * (size_t)owner_words(ebound), st, owners));
  b.owners = (uint32_t*)owners.p;
  b.owners_n = owner_words(ebound);
  b.tcones = (float4*)tcones.p;
  b.ka = (uint32_t*)ka.p; b.va = (uint32_t*)va.p; b.kb = (uint32_t*)kb.p; b.vb = (uint32_t*)vb.p;
  b.hist = (uint32_t*)hist.p; b.cnt_sorted = (uint32_t*)cnt_sorted.p;
  b.depth_work_zeroed = true;
  b.err = c->dev_err;
  b.spin_limit = c->spin_limit;
  ProfSlot* ps = prof_slot(c);
  if (ps) ps->kind = 0;
  prof_mark(ps, 0, st);
  enqueue_preprocess(st, *scene, n_views, op, lt.dev, b, false, c->dev_err);
  HTRY(hipGetLastError());
  prof_mark(ps, 1, st);
  // The entry count sizes the list, so it is read back; the depth order of
  // the visible items does not need it and is enqueued first (sized for all
  // items, with the live count read on the device), so the device has work
  // while the host waits for the count.
  if (!c->totals_ready) HTRY(hipEventCreateWithFlags(&c->totals_ready, hipEventDisableTiming));
  HTRY(hipMemcpyAsync(c->pinned, b.stats, 64, hipMemcpyDeviceToHost, st));
  HTRY(hipEventRecord(c->totals_ready, st));

  // ---- stage (b): depth sort, expansion, tile sort, ranges ----
  prof_mark(ps, 2, st);
  enqueue_depth_order(st, items, items, (const unsigned long long*)(b.stats + 1), b);
  HTRY(hipGetLastError());

  HTRY(hipEventSynchronize(c->totals_ready));
  uint64_t totals[8];
  std::memcpy(totals, c->pinned, 64);
  if (totals[7] != 0) {
    // an earlier forward on this context stalled: its outputs were invalid
    launch_fill_u32(st, (uint32_t*)c->dev_err, 2, 0u);
    return cleanup(fail(c, GEER_ERR_STALLED,
                        "the association sort of an earlier forward on this context stalled (look-back spin limit); "
                        "its outputs are invalid"));
  }
  const int64_t E = (int64_t)totals[0], nvis = (int64_t)totals[1];
  if (totals[0] >= (uint64_t)kMaxKeys)
    return cleanup(fail(c, GEER_ERR_CAPACITY, "association list of %llu entries exceeds 2^30",
                        (unsigned long long)totals[0]));
  f->entries = E;
  f->visible = nvis;

  const int64_t e1 = std::max<int64_t>(E, 1);
  TRY(acquire(c, 4 * (size_t)tile_work_words(e1), st, twork));
  b.twork = (uint32_t*)twork.p;
  TRY(acquire(c, 4 * (e1 + 8), st, tiles_a));
  TRY(acquire(c, 4 * (e1 + 8), st, tiles_b));
  TRY(acquire(c, 4 * (e1 + 8), st, f->list));
  TRY(acquire(c, 4 * (e1 + 8), st, items_b));
  TRY(acquire(c, 4 * (ntiles + 1), st, f->ranges));
  b.tiles_a = (uint32_t*)tiles_a.p; b.tiles_b = (uint32_t*)tiles_b.p; b.items_b = (uint32_t*)items_b.p;
  b.list = (uint32_t*)f->list.p; b.ranges = (uint32_t*)f->ranges.p;
  enqueue_tile_lists(st, op, n, items, nvis, nullptr, E, nullptr, ntiles, b);
  HTRY(hipGetLastError());

  // ---- stage (c): render ----
  f->hmax = heavy_capacity(ntiles);
  TRY(acquire(c, 4 * (size_t)heavy_list_words(ntiles), st, f->heavy_list));
  TRY(acquire(c, 4 * (size_t)ntiles, st, f->heavy_flag));
  b.heavy_list = (uint32_t*)f->heavy_list.p;
  b.heavy_flag = (uint32_t*)f->heavy_flag.p;
  b.hmax = f->hmax;
  const bool keep = frame_out != nullptr;
  if (keep) {
    TRY(acquire(c, 4 * npix, st, f->nlast));
    TRY(acquire(c, 4 * npix, st, f->tfinal));
    b.nlast = (uint32_t*)f->nlast.p;
    b.tfinal = (float*)f->tfinal.p;
  }
  prof_mark(ps, 3, st);
  enqueue_render(st, op, ntiles, n_views, b, rgb, depth, trans);
  HTRY(hipGetLastError());
  prof_mark(ps, 4, st);
  if (ps) HTRY(hipMemcpyAsync(ps->host_stats, b.stats, 48, hipMemcpyDeviceToHost, st));
  cleanup(GEER_OK);
  if (keep) {
    std::lock_guard<std::mutex> lk(c->mu);
    ++c->live_frames;
    *frame_out = f;
  } else {
    free_frame_buffers(f);
    delete f;
  }
  return GEER_OK;
#undef TRY
#undef HTRY
}

geer_status geer_render_backward(geer_ctx* c, const geer_frame* f, const float* dl_drgb, float* g_mean,
                                 float* g_scale, float* g_quat, float* g_opacity, float* g_sh, int32_t accumulate,
                                 void* stream) {
  if (!c) return GEER_ERR_INVALID_ARG;
  if (!f || f->ctx != c) return fail(c, GEER_ERR_INVALID_ARG, "frame missing or from another context");
  if (!dl_drgb) return fail(c, GEER_ERR_INVALID_ARG, "null dL/dRGB");
  if (f->n > 0 && (!g_mean || !g_scale || !g_quat || !g_opacity || !g_sh))
    return fail(c, GEER_ERR_INVALID_ARG, "null gradient array");
  if (f->op.splat) return fail(c, GEER_ERR_UNSUPPORTED, "the splat-opacity render has no backward");
  if (!f->nlast.p || !f->tfinal.p) return fail(c, GEER_ERR_INVALID_ARG, "frame holds no forward state");
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(c, hipSetDevice(c->device));
  // per-item accumulators, then the replay's pair counters and their total
  Block acc;
  const size_t acc_bytes = round_up(sizeof(float) * 16 * (size_t)std::max<int64_t>(f->items, 1), 256);
  geer_status s = acquire(c, acc_bytes + 8 * (size_t)(kEvalSlots + 1) * kEvalStride, st, acc);
  if (s != GEER_OK) return s;
  unsigned long long* counters = (unsigned long long*)((char*)acc.p + acc_bytes);
  const char* meta = (const char*)f->meta.p;
  const ViewDev* d_views = (const ViewDev*)meta;
  const float* d_edges = (const float*)(meta + f->edges_off);
  const float2* d_dtab = (const float2*)(meta + f->dtab_off);
  const geer_scene& sc = f->scene;
  const HeavyTiles heavy{(uint32_t*)f->heavy_list.p, (uint32_t*)f->heavy_flag.p,
                         (unsigned long long*)((uint64_t*)f->stats.p + 6), f->hmax, heavy_slots(f->hmax)};
  ProfSlot* ps = prof_slot(c);
  if (ps) ps->kind = 1;
  launch_zero_acc(st, (float*)acc.p, (const uint32_t*)f->counts.p, f->items, counters);
  prof_mark(ps, 0, st);
  launch_render_backward(st, f->op.lambda_mode == 1, f->ntiles, f->nviews, d_views, d_dtab, f->op, heavy,
                         (const uint32_t*)f->ranges.p, (const uint32_t*)f->list.p, (const uint2*)f->rects.p,
                         (const Record*)f->recs.p, (const uint32_t*)f->nlast.p, (const float*)f->tfinal.p, dl_drgb,
                         (float*)acc.p, counters);
  prof_mark(ps, 1, st);
  launch_preprocess_backward(st, f->n, f->nviews, sc.sh_degree, sc.mean, sc.scale, sc.quat, sc.opacity, sc.sh,
                             d_views, d_edges, f->lam, f->op, (const uint32_t*)f->counts.p, (const float*)acc.p,
                             (const Record*)f->recs.p, accumulate != 0, g_mean, g_scale, g_quat, g_opacity, g_sh);
  prof_mark(ps, 2, st);
  if (ps) {
    prof_mark(ps, 3, st);
    prof_mark(ps, 4, st);
    (void)hipMemcpyAsync(ps->host_stats, counters + kEvalSlots * kEvalStride, 8, hipMemcpyDeviceToHost, st);
  }
  hipError_t e = hipGetLastError();
  release(c, acc);
  if (e != hipSuccess) return fail(c, GEER_ERR_HIP, "backward launch: %s", hipGetErrorString(e));
  return GEER_OK;
}

void geer_frame_release(geer_frame* f) {
  if (!f) return;
  geer_ctx* c = f->ctx;
  free_frame_buffers(f);
  {
    std::lock_guard<std::mutex> lk(c->mu);
    --c->live_frames;
  }
  delete f;
}

// Reads and clears the context's sticky stall flag (after `stream` drains).
geer_status take_stall(geer_ctx* c, hipStream_t stream) {
  uint64_t e = 0;
  HIP_TRY(c, hipStreamSynchronize(stream));
  HIP_TRY(c, hipMemcpy(&e, c->dev_err, 8, hipMemcpyDeviceToHost));
  if (e == 0) return GEER_OK;
  HIP_TRY(c, hipMemset(c->dev_err, 0, 8));
  return fail(c, GEER_ERR_STALLED, "an association sort on this context stalled (look-back spin limit); the outputs "
                                   "of that forward are invalid");
}

geer_status read_frame_stats(const geer_frame* f, uint64_t st[6]) {
  geer_ctx* c = f->ctx;
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipMemcpyAsync(st, f->stats.p, 6 * sizeof(uint64_t), hipMemcpyDeviceToHost, f->stream));
  geer_status s = take_stall(c, f->stream);
  if (s != GEER_OK) return s;
  f->kept = f->entries > 0 ? (int64_t)st[5] : 0;
  return GEER_OK;
}

geer_status geer_frame_get_stats(const geer_frame* f, geer_frame_stats* out) {
  if (!f || !out) return GEER_ERR_INVALID_ARG;
  uint64_t st[6];
  geer_status s = read_frame_stats(f, st);
  if (s != GEER_OK) return s;
  out->n_items = f->items;
  out->n_visible = (int64_t)st[1];
  out->n_entries = f->kept;
  out->n_tiles = f->ntiles;
  out->n_pixels = f->npix;
  out->n_evaluated = (int64_t)st[2];
  out->n_candidates = (int64_t)st[0];
  return GEER_OK;
}

int64_t geer_frame_buffer_bytes(const geer_frame* f, int32_t which) {
  if (!f) return -1;
  switch (which) {
    case GEER_BUF_RECT: return 8 * f->items;
    case GEER_BUF_COUNT: return 4 * f->items;
    case GEER_BUF_KEY: return 4 * f->items;
    case GEER_BUF_LIST: {
      if (f->kept < 0) {
        uint64_t st[6];
        if (read_frame_stats(f, st) != GEER_OK) return -1;
      }
      return 4 * f->kept;
    }
    case GEER_BUF_RANGES: return 4 * (f->ntiles + 1);
    case GEER_BUF_NLAST: return 4 * f->npix;
    default: return -1;
  }
}

geer_status geer_frame_export(const geer_frame* f, int32_t which, void* dst, int64_t bytes) {
  if (!f || !dst) return GEER_ERR_INVALID_ARG;
  geer_ctx* c = f->ctx;
  int64_t need = geer_frame_buffer_bytes(f, which);
  if (need < 0) return fail(c, GEER_ERR_INVALID_ARG, "unknown buffer %d", which);
  if (bytes < need) return fail(c, GEER_ERR_INVALID_ARG, "destination too small (%lld < %lld)", (long long)bytes,
                                (long long)need);
  const Block* b = nullptr;
  switch (which) {
    case GEER_BUF_RECT: b = &f->rects; break;
    case GEER_BUF_COUNT: b = &f->counts; break;
    case GEER_BUF_KEY: b = &f->keys; break;
    case GEER_BUF_LIST: b = &f->list; break;
    case GEER_BUF_RANGES: b = &f->ranges; break;
    case GEER_BUF_NLAST: b = &f->nlast; break;
  }
  if (need == 0) return GEER_OK;
  if (!b || !b->p) return fail(c, GEER_ERR_INVALID_ARG, "buffer %d not kept by this frame", which);
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipMemcpyAsync(dst, b->p, (size_t)need, hipMemcpyDeviceToHost, f->stream));
  HIP_TRY(c, hipStreamSynchronize(f->stream));
  return GEER_OK;
}

geer_status geer_set_profiling(geer_ctx* c, int32_t enable) {
  if (!c) return GEER_ERR_INVALID_ARG;
  HIP_TRY(c, hipSetDevice(c->device));
  if (enable && c->prof.empty()) {
    c->prof.resize(64);
    for (auto& ps : c->prof) {
      for (auto& e : ps.ev) HIP_TRY(c, hipEventCreate(&e));
      HIP_TRY(c, hipHostMalloc((void**)&ps.host_stats, 64, hipHostMallocDefault));
    }
  }
  c->profiling = enable != 0;
  c->prof_next = 0;
  c->prof_count = 0;
  return GEER_OK;
}

int32_t geer_profile_read(geer_ctx* c, geer_profile_record* out, int32_t max) {
  if (!c || !out || max < 0) return -GEER_ERR_INVALID_ARG;
  if (hipSetDevice(c->device) != hipSuccess) return -GEER_ERR_HIP;
  int n = std::min<int>(max, c->prof_count);
  int size = (int)c->prof.size();
  for (int i = 0; i < n; ++i) {
    // oldest of the last n records first
    int idx = ((c->prof_next - n + i) % size + size) % size;
    ProfSlot& ps = c->prof[idx];
    if (hipEventSynchronize(ps.ev[4]) != hipSuccess) return -GEER_ERR_HIP;
    float t01 = 0, t12 = 0, t23 = 0, t34 = 0, t04 = 0;
    (void)hipEventElapsedTime(&t01, ps.ev[0], ps.ev[1]);
    (void)hipEventElapsedTime(&t12, ps.ev[1], ps.ev[2]);
    (void)hipEventElapsedTime(&t23, ps.ev[2], ps.ev[3]);
    (void)hipEventElapsedTime(&t34, ps.ev[3], ps.ev[4]);
    (void)hipEventElapsedTime(&t04, ps.ev[0], ps.ev[4]);
    out[i].kind = ps.kind;
    out[i].reserved = 0;
    if (ps.kind == 1) {  // backward: ray-wise replay, Gaussian-wise stage
      out[i].ms_render = t01;
      out[i].ms_preprocess = t12;
      out[i].ms_sort = 0.0f;
      out[i].ms_total = t04;
      out[i].n_entries = 0;
      out[i].n_evaluated = (int64_t)ps.host_stats[0];
    } else {
      out[i].ms_preprocess = t01;
      out[i].ms_sort = t23;
      out[i].ms_render = t34;
      out[i].ms_total = t04;
      out[i].n_entries = (int64_t)ps.host_stats[5];
      out[i].n_evaluated = (int64_t)ps.host_stats[2];
    }
  }
  c->prof_count = 0;
  return n;
}

geer_status geer_valid_mask(const geer_view* v, uint8_t* mask) {
  if (!v || !mask) return GEER_ERR_INVALID_ARG;
  geer_status s = check_view(nullptr, *v, 0);
  if (s != GEER_OK) return s;
  valid_mask(*v, mask);
  return GEER_OK;
}

geer_status geer_l1_loss(geer_ctx* c, int64_t pixels, const float* rgb, const float* target, const uint8_t* mask,
                         float* dl_drgb, float* loss, void* stream) {
  if (!c) return GEER_ERR_INVALID_ARG;
  if (pixels < 0 || (pixels > 0 && (!rgb || !target || !mask || !dl_drgb)) || !loss)
    return fail(c, GEER_ERR_INVALID_ARG, "bad loss arguments");
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(c, hipSetDevice(c->device));
  Block scratch;
  const int64_t nb = l1_partial_count(pixels);
  geer_status s = acquire(c, sizeof(float2) * (size_t)(nb + 1) + 16, st, scratch);
  if (s != GEER_OK) return s;
  float2* partial = (float2*)scratch.p;
  float* scale = (float*)(partial + nb + 1);
  launch_l1(st, pixels, rgb, target, mask, dl_drgb, loss, partial, scale, 1.0);
  hipError_t e = hipGetLastError();
  release(c, scratch);
  if (e != hipSuccess) return fail(c, GEER_ERR_HIP, "loss launch: %s", hipGetErrorString(e));
  return GEER_OK;
}

// Workspace layout of a plan: every buffer of the capacity-sized forward,
// 256-byte aligned, carved from one block.
struct PlanLayout {
  size_t meta = 0, recs = 0, rects = 0, keys = 0, counts = 0, stats = 0, ka = 0, va = 0, kb = 0, vb = 0, hist = 0,
         twork = 0, cnt_sorted = 0, tiles_a = 0, tiles_b = 0, items_b = 0, list = 0, ranges = 0, heavy_list = 0,
         heavy_flag = 0, tcones = 0, owners = 0, total = 0;
};

// pre_items (default: items) sizes the per-item outputs of the preprocess.
PlanLayout plan_layout(size_t meta_bytes, int64_t items, int64_t ecap, int64_t ntiles, int64_t pre_items = -1) {
  PlanLayout L;
  size_t off = 0;
  auto put = [&](size_t bytes) {
    const size_t at = off;
    off += round_up(std::max<size_t>(bytes, 256), 256);
    return at;
  };
  const int64_t it1 = std::max<int64_t>(items, 1);
  L.meta = put(meta_bytes);
  const int64_t pre1 = pre_items < 0 ? it1 : std::max<int64_t>(pre_items, 1);
  L.recs = put(sizeof(Record) * pre1);
  L.rects = put(sizeof(uint2) * pre1);
  L.keys = put(4 * pre1);
  L.counts = put(4 * pre1);
  L.stats = put(64);
  L.ka = put(4 * it1);
  L.va = put(4 * it1);
  L.kb = put(4 * it1);
  L.vb = put(4 * it1);
  L.hist = put(4 * (size_t)depth_work_words(it1));
  L.twork = put(4 * (size_t)tile_work_words(ecap));
  L.cnt_sorted = put(4 * it1);
  L.tiles_a = put(4 * (ecap + 8));
  L.tiles_b = put(4 * (ecap + 8));
  L.items_b = put(4 * (ecap + 8));
  L.list = put(4 * (ecap + 8));
  L.ranges = put(4 * (ntiles + 1));
  L.heavy_list = put(4 * (size_t)heavy_list_words(ntiles));
  L.heavy_flag = put(4 * (size_t)ntiles);
  L.tcones = put(tile_cone_bytes(ntiles));
  L.owners = put(4 * (size_t)owner_words(ecap));
  L.total = off;
  return L;
}

// Device pointers of a capacity-sized forward carved from the block at w.
FwdBufs carve_plan(char* w, const PlanLayout& lay, const ViewTables& tab, int64_t ntiles, int64_t ecap) {
  FwdBufs b;
  b.views = (const ViewDev*)(w + lay.meta);
  b.edges = (const float*)(w + lay.meta + tab.edges_off);
  b.dtab = (const float2*)(w + lay.meta + tab.dtab_off);
  b.recs = (Record*)(w + lay.recs);
  b.rects = (uint2*)(w + lay.rects);
  b.keys = (uint32_t*)(w + lay.keys);
  b.counts = (uint32_t*)(w + lay.counts);
  b.stats = (uint64_t*)(w + lay.stats);
  b.ka = (uint32_t*)(w + lay.ka);
  b.va = (uint32_t*)(w + lay.va);
  b.kb = (uint32_t*)(w + lay.kb);
  b.vb = (uint32_t*)(w + lay.vb);
  b.hist = (uint32_t*)(w + lay.hist);
  b.twork = (uint32_t*)(w + lay.twork);
  b.cnt_sorted = (uint32_t*)(w + lay.cnt_sorted);
  b.tiles_a = (uint32_t*)(w + lay.tiles_a);
  b.tiles_b = (uint32_t*)(w + lay.tiles_b);
  b.items_b = (uint32_t*)(w + lay.items_b);
  b.list = (uint32_t*)(w + lay.list);
  b.ranges = (uint32_t*)(w + lay.ranges);
  b.heavy_list = (uint32_t*)(w + lay.heavy_list);
  b.heavy_flag = (uint32_t*)(w + lay.heavy_flag);
  b.tcones = (float4*)(w + lay.tcones);
  b.owners = (uint32_t*)(w + lay.owners);
  b.owners_n = owner_words(ecap);
  b.hmax = heavy_capacity(ntiles);
  return b;
}

// Shared argument checks of geer_plan_workspace_bytes and geer_plan_create.
geer_status plan_check(geer_ctx* c, const geer_scene* scene, int32_t n_views, const geer_view* views,
                       const geer_opts* opts, int64_t entry_capacity, ViewTables& tab) {
  if (!scene || !views || !opts) return fail(c, GEER_ERR_INVALID_ARG, "null argument");
  if (n_views < 1 || n_views > 4096) return fail(c, GEER_ERR_INVALID_ARG, "n_views %d out of range", n_views);
  if (entry_capacity < 1 || entry_capacity >= kMaxKeys)
    return fail(c, GEER_ERR_INVALID_ARG, "entry capacity %lld out of range", (long long)entry_capacity);
  geer_status s;
  if ((s = check_scene(c, scene)) != GEER_OK) return s;
  if ((s = check_opts(c, *opts)) != GEER_OK) return s;
  for (int i = 0; i < n_views; ++i)
    if ((s = check_view(c, views[i], i)) != GEER_OK) return s;
  if (scene->n < 1) return fail(c, GEER_ERR_INVALID_ARG, "a plan needs a non-empty scene");
  if (scene->n * n_views >= kMaxKeys) return fail(c, GEER_ERR_CAPACITY, "Gaussians x views exceeds 2^30");
  return build_tables(c, n_views, views, tab);
}

geer_status geer_plan_workspace_bytes(geer_ctx* c, const geer_scene* scene, int32_t n_views, const geer_view* views,
                                      const geer_opts* opts, int64_t entry_capacity, int64_t* bytes) {
  if (!c || !bytes) return GEER_ERR_INVALID_ARG;
  ViewTables tab;
  geer_status s = plan_check(c, scene, n_views, views, opts, entry_capacity, tab);
  if (s != GEER_OK) return s;
  *bytes = (int64_t)plan_layout(tab.bytes, scene->n * n_views, entry_capacity, tab.ntiles).total;
  return GEER_OK;
}

geer_status geer_plan_create(geer_ctx* c, const geer_scene* scene, int32_t n_views, const geer_view* views,
                             const geer_opts* opts, int64_t entry_capacity, void* workspace,
                             int64_t workspace_bytes, float* rgb, float* depth, float* trans, geer_plan** out) {
  if (!c || !out) return GEER_ERR_INVALID_ARG;
  *out = nullptr;
  if (!rgb) return fail(c, GEER_ERR_INVALID_ARG, "null rgb");
  ViewTables tab;
  geer_status s = plan_check(c, scene, n_views, views, opts, entry_capacity, tab);
  if (s != GEER_OK) return s;
  const int64_t items = scene->n * n_views;
  const PlanLayout lay = plan_layout(tab.bytes, items, entry_capacity, tab.ntiles);
  if (workspace && ((uintptr_t)workspace % 256 != 0 || workspace_bytes < (int64_t)lay.total))
    return fail(c, GEER_ERR_INVALID_ARG, "workspace must be 256-byte aligned and hold %zu bytes", lay.total);
  HIP_TRY(c, hipSetDevice(c->device));
  LamTab lt;
  if ((s = lambda_dev(c, opts->alpha_min, &lt)) != GEER_OK) return s;

  geer_plan* P = new (std::nothrow) geer_plan();
  if (!P) return fail(c, GEER_ERR_OOM, "plan allocation");
  P->ctx = c;
  P->scene = *scene;
  P->op = make_opts(lt, *opts);
  P->nviews = n_views;
  P->shapes.assign(views, views + n_views);
  P->n = scene->n;
  P->items = items;
  P->ntiles = tab.ntiles;
  P->npix = tab.npix;
  P->ecap = entry_capacity;
  P->meta_bytes = tab.bytes;
  auto bail = [&](geer_status st_) {
    geer_plan_destroy(P);
    return st_;
  };
#define PHIP(call)                                                                                       \
  do {                                                                                                   \
    hipError_t e_ = (call);                                                                              \
    if (e_ != hipSuccess) return bail(fail(c, GEER_ERR_HIP, "%s: %s", #call, hipGetErrorString(e_)));    \
  } while (0)
  if (workspace) {
    P->ws = workspace;
  } else {
    if (hipMalloc(&P->ws, lay.total) != hipSuccess) {
      (void)hipGetLastError();
      P->ws = nullptr;
      return bail(fail(c, GEER_ERR_OOM, "plan workspace of %zu bytes", lay.total));
    }
    P->owns_ws = true;
    P->bytes = (int64_t)lay.total;
  }
  char* w = (char*)P->ws;
  FwdBufs b = carve_plan(w, lay, tab, P->ntiles, entry_capacity);
  P->meta = w + lay.meta;
  P->stats = b.stats;
  for (int k = 0; k < 2; ++k) {
    PHIP(hipHostMalloc(&P->staging[k], std::max<size_t>(tab.bytes, 64), hipHostMallocDefault));
    PHIP(hipEventCreateWithFlags(&P->staged[k], hipEventDisableTiming));
  }
  PHIP(hipEventCreateWithFlags(&P->done, hipEventDisableTiming));
  PHIP(hipHostMalloc((void**)&P->host_stats, 64 * (size_t)P->nstat, hipHostMallocDefault));

  // Capture the forward once.  Nothing runs at capture time; the tables are
  // uploaded by every launch before the graph.
  hipStream_t cs = nullptr;
  PHIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    b.depth_work_zeroed = true;
    b.tickets = true;  // slots of a server replay plans on several streams at once
    enqueue_preprocess(cs, P->scene, n_views, P->op, lt.dev, b);
    enqueue_association(cs, P->op, P->n, items, std::max<int64_t>(items, 1), entry_capacity, P->ntiles, true, b);
    enqueue_render(cs, P->op, P->ntiles, n_views, b, rgb, depth, trans);
    hipError_t e2 = hipStreamEndCapture(cs, &P->graph);
    e = e2 != hipSuccess ? e2 : hipGetLastError();
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0);
  (void)hipStreamDestroy(cs);
  if (e != hipSuccess) return bail(fail(c, GEER_ERR_HIP, "graph capture: %s", hipGetErrorString(e)));
  *out = P;
  return GEER_OK;
#undef PHIP
}

// ------------------------------------------------ allocation-free forward

geer_status geer_render_static(geer_ctx* c, const geer_scene* scene, int32_t n_views, const geer_view* views,
                               const geer_opts* opts, float* rgb, float* depth, float* trans, void* stream) {
  if (!c) return GEER_ERR_INVALID_ARG;
  geer_status s;
  if ((s = check_render_args(c, scene, n_views, views, opts, rgb)) != GEER_OK) return s;
  HIP_TRY(c, hipSetDevice(c->device));
  char* base = (char*)static_scratch_addr(c->device);
  if (c->static_init != hipSuccess || !base)
    return fail(c, GEER_ERR_HIP, "fixed scratch array of device %d unavailable: %s", c->device,
                hipGetErrorString(c->static_init));
  ViewTables tab;
  if ((s = build_tables(c, n_views, views, tab)) != GEER_OK) return s;
  // the lambda^2 table travels with the view tables (no device table is created)
  LamTab lt;
  std::vector<float> lam;
  lt.amin = opts->alpha_min;
  lambda_table(opts->alpha_min, lam, lt.lo, lt.n);
  const Opts op = make_opts(lt, *opts);
  const size_t lam_off = round_up(tab.bytes, 256);
  const size_t meta_bytes = lam_off + sizeof(float) * lam.size();
  const int64_t n = scene->n, items = n * n_views, ntiles = tab.ntiles, npix = tab.npix;
  const size_t limit = GEER_STATIC_SCRATCH_BYTES;
  // the largest association list that fits beside the per-item buffers
  if (plan_layout(meta_bytes, items, 1, ntiles).total > limit)
    return fail(c, GEER_ERR_CAPACITY,
                "%lld Gaussians x views over %lld tiles need %zu bytes before any list entry; the fixed scratch "
                "array holds %zu",
                (long long)items, (long long)ntiles, plan_layout(meta_bytes, items, 1, ntiles).total, limit);
  int64_t lo = 1, hi = kMaxKeys - 1;
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo + 1) / 2;
    if (plan_layout(meta_bytes, items, mid, ntiles).total <= limit) lo = mid;
    else hi = mid - 1;
  }
  const int64_t ecap = lo;
  const PlanLayout lay = plan_layout(meta_bytes, items, ecap, ntiles);
  std::vector<char> host(meta_bytes);
  pack_tables(tab, host.data());
  std::memcpy(host.data() + lam_off, lam.data(), sizeof(float) * lam.size());

  hipStream_t st = (hipStream_t)stream;
  std::lock_guard<std::mutex> lk(static_scratch_lock(c->device));
  if (n == 0) {  // nothing to associate: background
    launch_fill_u32(st, (uint32_t*)rgb, 3 * npix, 0u);
    if (depth) launch_fill_u32(st, (uint32_t*)depth, npix, 0u);
    if (trans) launch_fill_u32(st, (uint32_t*)trans, npix, 0x3f800000u);
    HIP_TRY(c, hipGetLastError());
    HIP_TRY(c, hipStreamSynchronize(st));
    return GEER_OK;
  }
  FwdBufs b = carve_plan(base, lay, tab, ntiles, ecap);
  b.depth_work_zeroed = true;
  HIP_TRY(c, hipMemcpyAsync(base + lay.meta, host.data(), meta_bytes, hipMemcpyHostToDevice, st));
  enqueue_preprocess(st, *scene, n_views, op, (const float*)(base + lay.meta + lam_off), b);
  enqueue_association(st, op, n, items, items, ecap, ntiles, true, b);
  enqueue_render(st, op, ntiles, n_views, b, rgb, depth, trans);
  HIP_TRY(c, hipGetLastError());
  uint64_t h[8];
  HIP_TRY(c, hipMemcpyAsync(h, b.stats, sizeof h, hipMemcpyDeviceToHost, st));
  HIP_TRY(c, hipStreamSynchronize(st));
  if (h[4] != 0)
    return fail(c, GEER_ERR_STALLED, "association sort stalled (look-back spin limit); the outputs are invalid");
  if ((int64_t)h[3] > ecap)
    return fail(c, GEER_ERR_CAPACITY,
                "association list of %lld entries exceeds the %lld that fit in the fixed scratch array; the outputs "
                "are background",
                (long long)h[3], (long long)ecap);
  return GEER_OK;
}

// ---------------------------------------------------------- training plans

// Workspace of a training plan: the forward plan's buffers sized for the
// largest view (one view at a time), then the state kept between a view's
// forward and backward, the loss and the per-view statistics.
struct TrainLayout {
  PlanLayout fwd;
  size_t nlast = 0, tfinal = 0, dl = 0, acc = 0, partial = 0, loss_views = 0, stats = 0, mask = 0, list2 = 0,
         ranges2 = 0, total = 0;
};

struct TrainShape {
  std::vector<ViewTables> tabs;
  std::vector<size_t> seg_off;
  std::vector<int64_t> pix_off;
  size_t meta_bytes = 0;
  size_t all_off = 0;  // ViewDev of every view, edge offsets relative to the meta base (Gaussian-wise backward)
  int64_t ntiles_max = 0, npix_max = 0, npix_total = 0;
};

geer_status train_shape(geer_ctx* c, int32_t n_views, const geer_view* views, TrainShape& S) {
  S.tabs.assign(n_views, ViewTables{});
  S.seg_off.assign(n_views, 0);
  S.pix_off.assign(n_views, 0);
  size_t off = 0;
  for (int v = 0; v < n_views; ++v) {
    geer_status s = build_tables(c, 1, views + v, S.tabs[v]);
    if (s != GEER_OK) return s;
    S.seg_off[v] = off;
    off += round_up(std::max<size_t>(S.tabs[v].bytes, 256), 256);
    S.pix_off[v] = S.npix_total;
    S.npix_total += S.tabs[v].npix;
    S.ntiles_max = std::max(S.ntiles_max, S.tabs[v].ntiles);
    S.npix_max = std::max(S.npix_max, S.tabs[v].npix);
  }
  S.all_off = off;
  off += round_up(sizeof(ViewDev) * (size_t)n_views, 256);
  S.meta_bytes = off;
  return GEER_OK;
}

// Packs the per-view table blocks and the all-views ViewDev array.
void pack_train_tables(const TrainShape& S, void* dst) {
  const int nv = (int)S.tabs.size();
  std::vector<ViewDev> all(nv);
  for (int v = 0; v < nv; ++v) {
    pack_tables(S.tabs[v], (char*)dst + S.seg_off[v]);
    all[v] = S.tabs[v].hv[0];
    const int32_t base = (int32_t)((S.seg_off[v] + S.tabs[v].edges_off) / sizeof(float));
    all[v].ex_off += base;
    all[v].ey_off += base;
  }
  std::memcpy((char*)dst + S.all_off, all.data(), sizeof(ViewDev) * (size_t)nv);
}

TrainLayout train_layout(const TrainShape& S, int64_t n, int64_t ecap, int32_t n_views) {
  TrainLayout L;
  L.fwd = plan_layout(S.meta_bytes, n, ecap, S.ntiles_max, n * n_views);
  size_t off = L.fwd.total;
  auto put = [&](size_t bytes) {
    const size_t at = off;
    off += round_up(std::max<size_t>(bytes, 256), 256);
    return at;
  };
  L.nlast = put(4 * (size_t)S.npix_max);
  L.tfinal = put(4 * (size_t)S.npix_max);
  L.dl = put(12 * (size_t)S.npix_max);
  L.acc = put(64 * (size_t)std::max<int64_t>(n, 1) * (size_t)n_views);
  L.partial = put(sizeof(float2) * (size_t)(l1_partial_count(S.npix_max) + 1) + 16);
  L.loss_views = put(4 * (size_t)n_views);
  L.stats = put(64 * (size_t)n_views);
  L.mask = put((size_t)S.npix_max);
  // the second list and ranges: odd views' (the next view's association runs
  // while the previous view's render and backward read the first)
  L.list2 = put(4 * (size_t)(std::max<int64_t>(ecap, 1) + 8));
  L.ranges2 = put(4 * (size_t)(S.ntiles_max + 1));
  L.total = off;
  return L;
}

geer_status train_check(geer_ctx* c, const geer_scene* scene, int32_t n_views, const geer_view* views,
                        const geer_opts* opts, int64_t entry_capacity, TrainShape& S) {
  if (!scene || !views || !opts) return fail(c, GEER_ERR_INVALID_ARG, "null argument");
  if (n_views < 1 || n_views > 4096) return fail(c, GEER_ERR_INVALID_ARG, "n_views %d out of range", n_views);
  if (entry_capacity < 1 || entry_capacity >= kMaxKeys)
    return fail(c, GEER_ERR_INVALID_ARG, "entry capacity %lld out of range", (long long)entry_capacity);
  geer_status s;
  if ((s = check_scene(c, scene)) != GEER_OK) return s;
  if ((s = check_opts(c, *opts)) != GEER_OK) return s;
  if (opts->flags & GEER_OPT_SPLAT_ALPHA) return fail(c, GEER_ERR_UNSUPPORTED, "no training with the splat opacity");
  for (int i = 0; i < n_views; ++i)
    if ((s = check_view(c, views[i], i)) != GEER_OK) return s;
  if (scene->n < 1) return fail(c, GEER_ERR_INVALID_ARG, "a plan needs a non-empty scene");
  return train_shape(c, n_views, views, S);
}

geer_status geer_train_plan_workspace_bytes(geer_ctx* c, const geer_scene* scene, int32_t n_views,
                                            const geer_view* views, const geer_opts* opts, int64_t entry_capacity,
                                            int64_t* bytes) {
  if (!c || !bytes) return GEER_ERR_INVALID_ARG;
  TrainShape S;
  geer_status s = train_check(c, scene, n_views, views, opts, entry_capacity, S);
  if (s != GEER_OK) return s;
  *bytes = (int64_t)train_layout(S, scene->n, entry_capacity, n_views).total;
  return GEER_OK;
}

geer_status geer_train_plan_create(geer_ctx* c, const geer_scene* scene, int32_t n_views, const geer_view* views,
                                   const geer_opts* opts, int64_t entry_capacity, void* workspace,
                                   int64_t workspace_bytes, const float* target, const uint8_t* mask, float* rgb,
                                   float* loss, float* g_mean, float* g_scale, float* g_quat, float* g_opacity,
                                   float* g_sh, geer_plan** out) {
  if (!c || !out) return GEER_ERR_INVALID_ARG;
  *out = nullptr;
  if (!target || !rgb || !loss || !g_mean || !g_scale || !g_quat || !g_opacity || !g_sh)
    return fail(c, GEER_ERR_INVALID_ARG, "null output or target");
  TrainShape S;
  geer_status s = train_check(c, scene, n_views, views, opts, entry_capacity, S);
  if (s != GEER_OK) return s;
  const int64_t n = scene->n;
  const TrainLayout lay = train_layout(S, n, entry_capacity, n_views);
  if (workspace && ((uintptr_t)workspace % 256 != 0 || workspace_bytes < (int64_t)lay.total))
    return fail(c, GEER_ERR_INVALID_ARG, "workspace must be 256-byte aligned and hold %zu bytes", lay.total);
  HIP_TRY(c, hipSetDevice(c->device));
  LamTab lt;
  if ((s = lambda_dev(c, opts->alpha_min, &lt)) != GEER_OK) return s;

  geer_plan* P = new (std::nothrow) geer_plan();
  if (!P) return fail(c, GEER_ERR_OOM, "plan allocation");
  P->ctx = c;
  P->scene = *scene;
  P->op = make_opts(lt, *opts);
  P->nviews = n_views;
  P->shapes.assign(views, views + n_views);
  P->n = n;
  P->items = n;
  P->ntiles = S.ntiles_max;
  P->npix = S.npix_total;
  P->ecap = entry_capacity;
  P->meta_bytes = S.meta_bytes;
  P->nseg = n_views;
  P->seg_off = S.seg_off;
  P->nstat = n_views;
  auto bail = [&](geer_status st_) {
    geer_plan_destroy(P);
    return st_;
  };
#define PHIP(call)                                                                                       \
  do {                                                                                                   \
    hipError_t e_ = (call);                                                                              \
    if (e_ != hipSuccess) return bail(fail(c, GEER_ERR_HIP, "%s: %s", #call, hipGetErrorString(e_)));    \
  } while (0)
  if (workspace) {
    P->ws = workspace;
  } else {
    if (hipMalloc(&P->ws, lay.total) != hipSuccess) {
      (void)hipGetLastError();
      P->ws = nullptr;
      return bail(fail(c, GEER_ERR_OOM, "plan workspace of %zu bytes", lay.total));
    }
    P->owns_ws = true;
    P->bytes = (int64_t)lay.total;
  }
  char* w = (char*)P->ws;
  const PlanLayout& F = lay.fwd;
  P->meta = w + F.meta;
  P->stats = (uint64_t*)(w + lay.stats);
  FwdBufs b;
  b.recs = (Record*)(w + F.recs);
  b.rects = (uint2*)(w + F.rects);
  b.keys = (uint32_t*)(w + F.keys);
  b.counts = (uint32_t*)(w + F.counts);
  b.ka = (uint32_t*)(w + F.ka);
  b.va = (uint32_t*)(w + F.va);
  b.kb = (uint32_t*)(w + F.kb);
  b.vb = (uint32_t*)(w + F.vb);
  b.hist = (uint32_t*)(w + F.hist);
  b.twork = (uint32_t*)(w + F.twork);
  b.cnt_sorted = (uint32_t*)(w + F.cnt_sorted);
  b.tiles_a = (uint32_t*)(w + F.tiles_a);
  b.tiles_b = (uint32_t*)(w + F.tiles_b);
  b.items_b = (uint32_t*)(w + F.items_b);
  b.list = (uint32_t*)(w + F.list);
  b.ranges = (uint32_t*)(w + F.ranges);
  b.heavy_list = (uint32_t*)(w + F.heavy_list);
  b.heavy_flag = (uint32_t*)(w + F.heavy_flag);
  b.tcones = (float4*)(w + F.tcones);
  b.owners = (uint32_t*)(w + F.owners);
  b.owners_n = owner_words(entry_capacity);
  b.hmax = heavy_capacity(S.ntiles_max);
  b.nlast = (uint32_t*)(w + lay.nlast);
  b.tfinal = (float*)(w + lay.tfinal);
  float* dl = (float*)(w + lay.dl);
  float* acc = (float*)(w + lay.acc);
  float2* partial = (float2*)(w + lay.partial);
  float* scale = (float*)(partial + l1_partial_count(S.npix_max) + 1);
  float* loss_views = (float*)(w + lay.loss_views);
  uint8_t* ones = (uint8_t*)(w + lay.mask);
  if (!mask) PHIP(hipMemset(ones, 1, (size_t)S.npix_max));  // every ray valid (set once, outside the graph)
  for (int k = 0; k < 2; ++k) {
    PHIP(hipHostMalloc(&P->staging[k], std::max<size_t>(S.meta_bytes, 64), hipHostMallocDefault));
    PHIP(hipEventCreateWithFlags(&P->staged[k], hipEventDisableTiming));
  }
  PHIP(hipEventCreateWithFlags(&P->done, hipEventDisableTiming));
  PHIP(hipHostMalloc((void**)&P->host_stats, 64 * (size_t)n_views, hipHostMallocDefault));

  // Capture: per view, forward (keeping T_final and the last blended index),
  // weighted L1, backward accumulated into the gradients; then the loss sum.
  // The views' associations run on a second captured stream, one after the
  // other, each as soon as its list buffers are free: view v's association
  // overlaps view v - 1's render and backward (the two lists alternate).  So
  // at most one look-back pass runs at a time, and no tickets are needed.
  hipStream_t cs = nullptr, as = nullptr;
  PHIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  PHIP(hipStreamCreateWithFlags(&as, hipStreamNonBlocking));
  std::vector<hipEvent_t> evs(2 * (size_t)n_views + 1, nullptr);
  for (auto& ev : evs) PHIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  auto drop_streams = [&]() {
    for (auto& ev : evs)
      if (ev) (void)hipEventDestroy(ev);
    (void)hipStreamDestroy(as);
  };
  uint32_t* const lists[2] = {b.list, (uint32_t*)(w + lay.list2)};
  uint32_t* const rangess[2] = {b.ranges, (uint32_t*)(w + lay.ranges2)};
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    const double weight = 1.0 / (double)n_views;
    const ViewDev* all_views = (const ViewDev*)((char*)P->meta + S.all_off);
    // one preprocess for every view: the scene is read once, item v n + g
    // holds Gaussian g in view v, view v's counters are P->stats + 8 v
    b.views = all_views;
    b.edges = (const float*)P->meta;
    b.stats = P->stats;
    auto ok = [&](hipError_t r) {
      if (e == hipSuccess && r != hipSuccess) e = r;
    };
    // the association stream forks off after the preprocess's geometry; the
    // views' colour (the records' rgb, which no association kernel reads) and
    // the accumulators' clear follow on this stream meanwhile
    enqueue_preprocess(cs, P->scene, n_views, P->op, lt.dev, b, true, nullptr, true);
    ok(hipEventRecord(evs[0], cs));
    ok(hipStreamWaitEvent(as, evs[0], 0));
    launch_colour(cs, n, n_views, scene->sh_degree, scene->mean, scene->sh, all_views, b.counts, b.recs);
    launch_zero_acc(cs, acc, b.counts, n * (int64_t)n_views);  // the visible items' accumulators
    Record* const recs0 = b.recs;
    uint2* const rects0 = b.rects;
    uint32_t *const keys0 = b.keys, *const counts0 = b.counts;
    for (int v = 0; v < n_views && e == hipSuccess; ++v) {
      hipEvent_t assoc_done = evs[1 + 2 * v], bwd_done = evs[2 + 2 * v];
      const ViewTables& T = S.tabs[v];
      char* mv = (char*)P->meta + S.seg_off[v];
      b.views = (const ViewDev*)mv;
      b.edges = (const float*)(mv + T.edges_off);
      b.dtab = (const float2*)(mv + T.dtab_off);
      b.stats = P->stats + 8 * v;
      const int64_t io = (int64_t)v * n;
      b.recs = recs0 + io;
      b.rects = rects0 + io;
      b.keys = keys0 + io;
      b.counts = counts0 + io;
      const int64_t po = S.pix_off[v];
      float* rgb_v = rgb + 3 * po;
      b.list = lists[v & 1];
      b.ranges = rangess[v & 1];
      // this list was last read by view v - 2's backward
      if (v >= 2) ok(hipStreamWaitEvent(as, evs[2 + 2 * (v - 2)], 0));
      enqueue_association(as, P->op, n, n, n, entry_capacity, T.ntiles, true, b);
      ok(hipEventRecord(assoc_done, as));
      ok(hipStreamWaitEvent(cs, assoc_done, 0));
      enqueue_render(cs, P->op, T.ntiles, 1, b, rgb_v, nullptr, nullptr);
      launch_l1(cs, T.npix, rgb_v, target + 3 * po, mask ? mask + po : ones, dl, loss_views + v, partial, scale,
                weight);
      // ray-wise backward of this view into its own accumulator slice
      launch_render_backward(cs, P->op.lambda_mode == 1, T.ntiles, 1, b.views, b.dtab, P->op, b.heavy(), b.ranges,
                             b.list, b.rects, b.recs, b.nlast, b.tfinal, dl, acc + (size_t)v * (size_t)n * 16);
      ok(hipEventRecord(bwd_done, cs));
    }
    // Gaussian-wise backward once, summing every view
    launch_preprocess_backward(cs, n, n_views, scene->sh_degree, scene->mean, scene->scale, scene->quat,
                               scene->opacity, scene->sh, all_views,
                               (const float*)P->meta, lt.dev, P->op, counts0, acc, recs0, 0, g_mean, g_scale,
                               g_quat, g_opacity, g_sh);
    launch_sum_f32(cs, n_views, loss_views, loss);
    hipError_t e2 = hipStreamEndCapture(cs, &P->graph);
    if (e == hipSuccess) e = e2 != hipSuccess ? e2 : hipGetLastError();
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0);
  (void)hipStreamDestroy(cs);
  drop_streams();
  if (e != hipSuccess) return bail(fail(c, GEER_ERR_HIP, "graph capture: %s", hipGetErrorString(e)));
  *out = P;
  return GEER_OK;
#undef PHIP
}

geer_status geer_plan_launch(geer_plan* P, const geer_view* views, void* stream) {
  if (!P || !views) return GEER_ERR_INVALID_ARG;
  geer_ctx* c = P->ctx;
  geer_status s;
  for (int i = 0; i < P->nviews; ++i) {
    if ((s = check_view(c, views[i], i)) != GEER_OK) return s;
    if (views[i].width != P->shapes[i].width || views[i].height != P->shapes[i].height)
      return fail(c, GEER_ERR_INVALID_ARG, "view %d: grid %dx%d differs from the plan's %dx%d", i, views[i].width,
                  views[i].height, P->shapes[i].width, P->shapes[i].height);
  }
  HIP_TRY(c, hipSetDevice(c->device));
  ViewTables tab;
  TrainShape S;
  if (P->nseg) {
    if ((s = train_shape(c, P->nseg, views, S)) != GEER_OK) return s;
    if (S.meta_bytes != P->meta_bytes) return fail(c, GEER_ERR_INVALID_ARG, "view tables changed size");
  } else {
    if ((s = build_tables(c, P->nviews, views, tab)) != GEER_OK) return s;
    if (tab.bytes != P->meta_bytes) return fail(c, GEER_ERR_INVALID_ARG, "view tables changed size");
  }
  hipStream_t st = (hipStream_t)stream;
  // the previous launch (possibly on another stream) still reads the tables
  if (P->launched) HIP_TRY(c, hipStreamWaitEvent(st, P->done, 0));
  const int k = P->next;
  if (P->staged_used[k]) HIP_TRY(c, hipEventSynchronize(P->staged[k]));  // its previous upload has left the buffer
  if (P->nseg) pack_train_tables(S, P->staging[k]);
  else pack_tables(tab, P->staging[k]);
  HIP_TRY(c, hipMemcpyAsync(P->meta, P->staging[k], P->meta_bytes, hipMemcpyHostToDevice, st));
  HIP_TRY(c, hipEventRecord(P->staged[k], st));
  P->staged_used[k] = true;
  P->next = 1 - k;
  HIP_TRY(c, hipGraphLaunch(P->exec, st));
  HIP_TRY(c, hipMemcpyAsync(P->host_stats, P->stats, 64 * (size_t)P->nstat, hipMemcpyDeviceToHost, st));
  HIP_TRY(c, hipEventRecord(P->done, st));
  P->launched = true;
  return GEER_OK;
}

geer_status geer_plan_entries(geer_plan* P, int64_t* entries, int64_t* capacity) {
  if (!P) return GEER_ERR_INVALID_ARG;
  geer_ctx* c = P->ctx;
  if (capacity) *capacity = P->ecap;
  if (!P->launched) {
    if (entries) *entries = 0;
    return GEER_OK;
  }
  HIP_TRY(c, hipEventSynchronize(P->done));
  int64_t E = 0;
  bool stalled = false;
  for (int i = 0; i < P->nstat; ++i) {
    E = std::max<int64_t>(E, (int64_t)P->host_stats[8 * i + 3]);
    stalled |= P->host_stats[8 * i + 4] != 0;
  }
  if (entries) *entries = E;
  if (stalled)
    return fail(c, GEER_ERR_STALLED, "association sort stalled (look-back spin limit); the launch's outputs are invalid");
  if (E > P->ecap)
    return fail(c, GEER_ERR_CAPACITY, "association list of %lld entries exceeds the plan's %lld", (long long)E,
                (long long)P->ecap);
  return GEER_OK;
}

geer_status geer_plan_get_stats(geer_plan* P, geer_frame_stats* out) {
  if (!P || !out) return GEER_ERR_INVALID_ARG;
  geer_ctx* c = P->ctx;
  std::memset(out, 0, sizeof *out);
  out->n_items = P->items * (P->nseg ? P->nseg : 1);
  out->n_tiles = P->ntiles;
  out->n_pixels = P->npix;
  if (!P->launched) return GEER_OK;
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipEventSynchronize(P->done));
  int64_t tiles = 0;
  for (int i = 0; i < P->nstat; ++i) {
    const uint64_t* h = P->host_stats + 8 * i;
    out->n_visible += (int64_t)h[1];
    out->n_evaluated += (int64_t)h[2];
    out->n_candidates += (int64_t)h[3];
    out->n_entries += h[0] ? (int64_t)h[5] : 0;
  }
  if (P->nseg) {
    for (const geer_view& v : P->shapes) tiles += (int64_t)((v.width + 15) / 16) * ((v.height + 15) / 16);
    out->n_tiles = tiles;
  }
  return GEER_OK;
}

int64_t geer_plan_device_bytes(const geer_plan* P) { return P ? P->bytes : -1; }

void geer_plan_destroy(geer_plan* P) {
  if (!P) return;
  (void)hipSetDevice(P->ctx->device);
  if (P->launched) (void)hipEventSynchronize(P->done);
  if (P->exec) (void)hipGraphExecDestroy(P->exec);
  if (P->graph) (void)hipGraphDestroy(P->graph);
  for (int k = 0; k < 2; ++k) {
    if (P->staged[k]) {
      if (P->staged_used[k]) (void)hipEventSynchronize(P->staged[k]);
      (void)hipEventDestroy(P->staged[k]);
    }
    if (P->staging[k]) (void)hipHostFree(P->staging[k]);
  }
  if (P->done) (void)hipEventDestroy(P->done);
  if (P->host_stats) (void)hipHostFree(P->host_stats);
  if (P->owns_ws && P->ws) (void)hipFree(P->ws);
  delete P;
}

bool same_camera(const geer_view& a, const geer_view& b) {
  if (a.model != b.model || a.grid != b.grid || a.width != b.width || a.height != b.height || a.fx != b.fx ||
      a.fy != b.fy ||
      a.cx != b.cx || a.cy != b.cy || a.fov_x != b.fov_x || a.fov_y != b.fov_y)
    return false;
  for (int i = 0; i < 4; ++i)
    if (a.k[i] != b.k[i]) return false;
  return true;
}

geer_status geer_reproject(geer_ctx* c, const geer_view* view, int32_t native_width, int32_t native_height,
                           int32_t channels, const float* beap, float* native, uint8_t* valid, void* stream) {
  if (!c) return GEER_ERR_INVALID_ARG;
  if (!view || !beap || !native) return fail(c, GEER_ERR_INVALID_ARG, "null argument");
  geer_status s = check_view(c, *view, 0);
  if (s != GEER_OK) return s;
  if (view->grid != GEER_GRID_BEAP) return fail(c, GEER_ERR_INVALID_ARG, "reprojection takes a BEAP grid");
  const int nw = native_width > 0 ? native_width : view->width;
  const int nh = native_height > 0 ? native_height : view->height;
  if (nw > 65536 || nh > 65536 || native_width < 0 || native_height < 0)
    return fail(c, GEER_ERR_INVALID_ARG, "native size %dx%d out of range", native_width, native_height);
  if (channels < 1 || channels > 64) return fail(c, GEER_ERR_INVALID_ARG, "channels %d out of range", channels);
  if (!(view->fx > 0 && view->fy > 0)) return fail(c, GEER_ERR_INVALID_ARG, "focal lengths must be positive");
  HIP_TRY(c, hipSetDevice(c->device));
  void* map = nullptr;
  {
    std::lock_guard<std::mutex> lk(c->mu);
    for (size_t i = 0; i < c->maps.size(); ++i)
      if (c->maps[i].nw == nw && c->maps[i].nh == nh && same_camera(c->maps[i].key, *view)) {
        ReprojMap m = c->maps[i];
        c->maps.erase(c->maps.begin() + i);
        c->maps.push_back(m);
        map = m.dev;
        break;
      }
  }
  if (!map) {
    std::vector<int32_t> host;
    reproject_map(*view, nw, nh, host);
    const size_t bytes = host.size() * sizeof(int32_t);
    if (hipMalloc(&map, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return fail(c, GEER_ERR_OOM, "sampling map of %zu bytes", bytes);
    }
    HIP_TRY(c, hipMemcpy(map, host.data(), bytes, hipMemcpyHostToDevice));
    std::lock_guard<std::mutex> lk(c->mu);
    if (c->maps.size() >= 16) {  // drop the least recently used map once nothing can still read it
      (void)hipDeviceSynchronize();
      (void)hipFree(c->maps.front().dev);
      c->maps.erase(c->maps.begin());
    }
    ReprojMap m;
    m.key = *view;
    m.nw = nw;
    m.nh = nh;
    m.dev = map;
    c->maps.push_back(m);
  }
  launch_reproject((hipStream_t)stream, (const int4*)map, (int64_t)nw * nh, view->width, view->height, channels, beap,
                   native, valid);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, GEER_ERR_HIP, "reprojection launch: %s", hipGetErrorString(e));
  return GEER_OK;
}

geer_status check_train_state(geer_ctx* c, const geer_train_state* t, bool stats) {
  if (!t) return fail(c, GEER_ERR_INVALID_ARG, "null training state");
  if (t->n < 0 || t->n > ((int64_t)1 << 28) || t->sh_degree < 0 || t->sh_degree > 3 || t->reserved != 0)
    return fail(c, GEER_ERR_INVALID_ARG, "training state: n %lld, sh_degree %d", (long long)t->n, t->sh_degree);
  if (t->n > 0 && (!t->raw || !t->scale || !t->opacity || !t->m || !t->v || (stats && (!t->accum || !t->count))))
    return fail(c, GEER_ERR_INVALID_ARG, "training state: null array");
  return GEER_OK;
}

geer_status geer_activate(geer_ctx* c, const geer_train_state* t, void* stream) {
  if (!c) return GEER_ERR_INVALID_ARG;
  if (!t) return fail(c, GEER_ERR_INVALID_ARG, "null training state");
  if (t->n < 0 || (t->n > 0 && (!t->raw || !t->scale || !t->opacity)))
    return fail(c, GEER_ERR_INVALID_ARG, "training state: null array");
  HIP_TRY(c, hipSetDevice(c->device));
  launch_activate((hipStream_t)stream, t->n, t->raw, t->scale, t->opacity);
  HIP_TRY(c, hipGetLastError());
  return GEER_OK;
}

geer_status geer_adam_step(geer_ctx* c, const geer_train_state* t, const geer_adam_opts* o, const float* g_mean,
                           const float* g_scale, const float* g_quat, const float* g_opacity, const float* g_sh,
                           void* stream) {
  if (!c) return GEER_ERR_INVALID_ARG;
  geer_status s = check_train_state(c, t, false);
  if (s != GEER_OK) return s;
  if (!o || o->step < 1 || o->reserved != 0 || !(o->beta1 >= 0 && o->beta1 < 1) || !(o->beta2 >= 0 && o->beta2 < 1) ||
      !(o->eps >= 0))
    return fail(c, GEER_ERR_INVALID_ARG, "bad Adam options");
  if (t->n > 0 && (!g_mean || !g_scale || !g_quat || !g_opacity || !g_sh))
    return fail(c, GEER_ERR_INVALID_ARG, "null gradient array");
  if ((t->accum == nullptr) != (t->count == nullptr))
    return fail(c, GEER_ERR_INVALID_ARG, "accum and count go together");
  HIP_TRY(c, hipSetDevice(c->device));
  AdamParams ap;
  ap.lr[0] = o->lr_mean;
  ap.lr[1] = o->lr_scale;
  ap.lr[2] = o->lr_quat;
  ap.lr[3] = o->lr_opacity;
  ap.lr[4] = o->lr_sh;
  ap.b1 = (float)o->beta1;
  ap.b2 = (float)o->beta2;
  ap.eps = (float)o->eps;
  ap.omb1 = (float)(1.0 - o->beta1);
  ap.omb2 = (float)(1.0 - o->beta2);
  ap.c1 = (float)(1.0 / (1.0 - std::pow(o->beta1, (double)o->step)));
  ap.c2 = (float)(1.0 / (1.0 - std::pow(o->beta2, (double)o->step)));
  launch_adam((hipStream_t)stream, t->n, t->sh_degree, t->raw, g_mean, g_scale, g_quat, g_opacity, g_sh, t->m, t->v,
              t->scale, t->opacity, t->accum, t->count, ap);
  HIP_TRY(c, hipGetLastError());
  return GEER_OK;
}

geer_status geer_densify(geer_ctx* c, const geer_train_state* in, const geer_densify_opts* o, const float* noise,
                         geer_train_state* out, void* stream) {
  if (!c) return GEER_ERR_INVALID_ARG;
  geer_status s = check_train_state(c, in, true);
  if (s != GEER_OK) return s;
  if (!out || !o || (in->n > 0 && !noise)) return fail(c, GEER_ERR_INVALID_ARG, "null argument");
  if ((s = check_train_state(c, out, true)) != GEER_OK) return s;
  if (out->sh_degree != in->sh_degree) return fail(c, GEER_ERR_INVALID_ARG, "SH degrees differ");
  if (!(o->min_opacity > 0 && o->min_opacity < 1) || !(o->split_scale > 0) || !(o->split_shrink >= 1) ||
      !(o->grad_threshold >= 0))
    return fail(c, GEER_ERR_INVALID_ARG, "bad densification options");
  const int64_t n = in->n;
  const int64_t cap = out->n;
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(c, hipSetDevice(c->device));
  Block kind, offs, scratch;
  auto done = [&](geer_status r) {
    release(c, kind);
    release(c, offs);
    release(c, scratch);
    return r;
  };
  const int64_t n1 = std::max<int64_t>(n, 1);
  if ((s = acquire(c, 4 * (size_t)n1, st, kind)) != GEER_OK) return done(s);
  if ((s = acquire(c, 4 * (size_t)(n1 + 1), st, offs)) != GEER_OK) return done(s);
  if ((s = acquire(c, 4 * (size_t)scan_scratch_words(n1 + 1), st, scratch)) != GEER_OK) return done(s);
  DensifyParams dp;
  const double mo = o->min_opacity;
  dp.prune_logit = (float)std::log(mo / (1.0 - mo));
  dp.grad_threshold = o->grad_threshold;
  dp.split_log_scale = (float)std::log((double)o->split_scale);
  uint32_t* cnt = (uint32_t*)offs.p;  // counts, scanned in place into offsets; entry n is the total
  launch_fill_u32(st, cnt + n, 1, 0u);
  launch_densify_count(st, n, in->raw, in->accum, in->count, dp, cnt, (uint32_t*)kind.p);
  scan_exclusive(st, cnt, cnt, n + 1, (uint32_t*)scratch.p);
  uint32_t total = 0;
  hipError_t e = hipMemcpyAsync(&total, cnt + n, 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return done(fail(c, GEER_ERR_HIP, "densify count: %s", hipGetErrorString(e)));
  if ((int64_t)total > cap)
    return done(fail(c, GEER_ERR_CAPACITY, "densification gives %u Gaussians, capacity %lld", total, (long long)cap));
  launch_densify_apply(st, n, in->sh_degree, in->raw, in->m, in->v, (const uint32_t*)kind.p, cnt, noise, total,
                       out->raw, out->m, out->v, out->scale, out->opacity, out->accum, out->count,
                       (float)std::log((double)o->split_shrink));
  e = hipGetLastError();
  if (e != hipSuccess) return done(fail(c, GEER_ERR_HIP, "densify launch: %s", hipGetErrorString(e)));
  out->n = total;
  return done(GEER_OK);
}

geer_status geer_check(geer_ctx* c, void* stream) {
  if (!c) return GEER_ERR_INVALID_ARG;
  HIP_TRY(c, hipSetDevice(c->device));
  return take_stall(c, (hipStream_t)stream);
}

geer_status geer_debug_set_spin_limit(geer_ctx* c, int64_t limit) {
  if (!c) return GEER_ERR_INVALID_ARG;
  c->spin_limit = limit < 0 ? kDefaultSpinLimit : (uint32_t)std::min<int64_t>(limit, 0xffffffffll);
  return GEER_OK;
}

geer_status geer_debug_mark_stalled(geer_ctx* c, geer_plan* P) {
  if (!c) return GEER_ERR_INVALID_ARG;
  HIP_TRY(c, hipSetDevice(c->device));
  if (P) {
    if (P->ctx != c || !P->launched) return fail(c, GEER_ERR_INVALID_ARG, "plan from another context or not launched");
    HIP_TRY(c, hipEventSynchronize(P->done));
    P->host_stats[4] = 1;  // the first segment's stall word, as read back by the launch
    return GEER_OK;
  }
  const uint64_t one = 1;
  HIP_TRY(c, hipDeviceSynchronize());
  HIP_TRY(c, hipMemcpy(c->dev_err, &one, 8, hipMemcpyHostToDevice));
  return GEER_OK;
}

}  // extern "C"
