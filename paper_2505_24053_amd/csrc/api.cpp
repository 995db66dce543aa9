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
};

struct geer_ctx {
  int device = 0;
  bool profiling = false;
  std::vector<ProfSlot> prof;  // ring of stage-timing records
  int prof_next = 0, prof_count = 0;
  std::mutex mu;
  std::vector<Block> cache;  // released device blocks, reusable on the same stream
  std::string err;
  float lam_amin = -1.0f;
  float* lam_dev = nullptr;
  int lam_lo = 0, lam_n = 0;
  void* pinned = nullptr;  // host staging for table uploads and read-backs
  size_t pinned_bytes = 0;
  int64_t live_frames = 0;
};

struct geer_frame {
  geer_ctx* ctx = nullptr;
  hipStream_t stream = nullptr;
  geer_scene scene{};
  Opts op{};
  int32_t nviews = 0;
  int64_t n = 0, items = 0, ntiles = 0, npix = 0, entries = 0, visible = 0;
  size_t edges_off = 0, dtab_off = 0;  // sub-buffers of meta
  std::vector<geer_view> views;
  std::vector<ViewDev> hviews;
  Block meta, recs, rects, keys, counts, list, ranges, nlast, tfinal, stats;
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
  if (v.reserved != 0) return fail(c, GEER_ERR_INVALID_ARG, "view %d: reserved field must be 0", i);
  if (!(v.fov_x > 0 && v.fov_x <= 2 * M_PI) || !(v.fov_y > 0 && v.fov_y <= M_PI))
    return fail(c, GEER_ERR_INVALID_ARG, "view %d: fov (%g, %g) outside (0, 2pi] x (0, pi]", i, v.fov_x, v.fov_y);
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
  if (o.reserved != 0) return fail(c, GEER_ERR_INVALID_ARG, "opts.reserved must be 0");
  return GEER_OK;
}

geer_status lambda_dev(geer_ctx* c, float amin, hipStream_t st) {
  if (c->lam_dev && c->lam_amin == amin) return GEER_OK;
  std::vector<float> tab;
  int lo, n;
  lambda_table(amin, tab, lo, n);
  if (c->lam_dev) {
    HIP_TRY(c, hipStreamSynchronize(st));
    (void)hipFree(c->lam_dev);
    c->lam_dev = nullptr;
  }
  HIP_TRY(c, hipMalloc(&c->lam_dev, tab.size() * sizeof(float)));
  HIP_TRY(c, hipMemcpy(c->lam_dev, tab.data(), tab.size() * sizeof(float), hipMemcpyHostToDevice));
  c->lam_amin = amin;
  c->lam_lo = lo;
  c->lam_n = n;
  return GEER_OK;
}

void free_frame_buffers(geer_frame* f) {
  geer_ctx* c = f->ctx;
  for (Block* b : {&f->meta, &f->recs, &f->rects, &f->keys, &f->counts, &f->list, &f->ranges, &f->nlast,
                   &f->tfinal, &f->stats})
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

int bytes_for_tiles(int64_t max_tile) {
  int passes = 0;
  while (max_tile > 0) {
    ++passes;
    max_tile >>= 8;
  }
  return passes;
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
  if (c->lam_dev) (void)hipFree(c->lam_dev);
  if (c->pinned) (void)hipHostFree(c->pinned);
  delete c;
}

const char* geer_last_error(const geer_ctx* c) { return c ? c->err.c_str() : "null context"; }

geer_status geer_render(geer_ctx* c, const geer_scene* scene, int32_t n_views, const geer_view* views,
                        const geer_opts* opts, float* rgb, float* depth, float* trans, geer_frame** frame_out,
                        void* stream) {
  if (!c) return GEER_ERR_INVALID_ARG;
  if (frame_out) *frame_out = nullptr;
  if (!scene || !views || !opts || !rgb) return fail(c, GEER_ERR_INVALID_ARG, "null argument");
  if (n_views < 1 || n_views > 4096) return fail(c, GEER_ERR_INVALID_ARG, "n_views %d out of range", n_views);
  const int64_t n = scene->n;
  if (n < 0 || n > ((int64_t)1 << 28)) return fail(c, GEER_ERR_INVALID_ARG, "scene size %lld", (long long)n);
  if (scene->sh_degree < 0 || scene->sh_degree > 3) return fail(c, GEER_ERR_INVALID_ARG, "sh_degree must be 0..3");
  if (scene->reserved != 0) return fail(c, GEER_ERR_INVALID_ARG, "scene.reserved must be 0");
  if (n > 0 && (!scene->mean || !scene->scale || !scene->quat || !scene->opacity || !scene->sh))
    return fail(c, GEER_ERR_INVALID_ARG, "null scene array");
  geer_status s;
  if ((s = check_opts(c, *opts)) != GEER_OK) return s;
  const int64_t items = n * n_views;
  if (items >= ((int64_t)1 << 32) - 16) return fail(c, GEER_ERR_CAPACITY, "Gaussians x views exceeds 2^32");
  for (int i = 0; i < n_views; ++i)
    if ((s = check_view(c, views[i], i)) != GEER_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(c, hipSetDevice(c->device));

  // ---- per-view constants and tables, one upload ----
  std::vector<ViewDev> hv(n_views);
  std::vector<float> edges, dtab;
  int64_t ntiles = 0, npix = 0;
  for (int i = 0; i < n_views; ++i) {
    view_constants(views[i], hv[i]);
    std::vector<float> ex, ey, dx, dy;
    edge_tables(views[i], ex, ey);
    direction_tables(views[i], dx, dy);
    hv[i].tile_base = (int32_t)ntiles;
    hv[i].pix_base = (int32_t)npix;
    hv[i].ex_off = (int32_t)edges.size();
    edges.insert(edges.end(), ex.begin(), ex.end());
    hv[i].ey_off = (int32_t)edges.size();
    edges.insert(edges.end(), ey.begin(), ey.end());
    hv[i].dx_off = (int32_t)(dtab.size() / 2);
    dtab.insert(dtab.end(), dx.begin(), dx.end());
    hv[i].dy_off = (int32_t)(dtab.size() / 2);
    dtab.insert(dtab.end(), dy.begin(), dy.end());
    ntiles += (int64_t)hv[i].tiles_x * hv[i].tiles_y;
    npix += (int64_t)views[i].width * views[i].height;
    if (ntiles >= ((int64_t)1 << 31) || npix >= ((int64_t)1 << 31))
      return fail(c, GEER_ERR_CAPACITY, "batch exceeds 2^31 tiles or pixels");
  }
  Opts op{};
  op.alpha_min = opts->alpha_min;
  op.alpha_max = opts->alpha_max;
  op.t_min = opts->t_min;
  op.lambda_fixed = opts->lambda_fixed;
  op.lambda_mode = opts->lambda_mode;
  op.lam2_fixed = lambda_fixed_hat(opts->lambda_fixed);
  op.kmax_fixed = opts->lambda_fixed * opts->lambda_fixed;
  if ((s = lambda_dev(c, opts->alpha_min, st)) != GEER_OK) return s;
  op.lam_lo = c->lam_lo;
  op.lam_n = c->lam_n;

  geer_frame* f = new (std::nothrow) geer_frame();
  if (!f) return fail(c, GEER_ERR_OOM, "frame allocation");
  f->ctx = c;
  f->stream = st;
  f->scene = *scene;
  f->op = op;
  f->nviews = n_views;
  f->n = n;
  f->items = items;
  f->ntiles = ntiles;
  f->npix = npix;
  f->views.assign(views, views + n_views);
  f->hviews = hv;

  // Temporaries of the sort; released at the end of the call.
  Block ka, va, kb, vb, hist, scratch, tiles_a, tiles_b, items_b, cnt_sorted;
  auto cleanup = [&](geer_status st_) {
    for (Block* b : {&ka, &va, &kb, &vb, &hist, &scratch, &tiles_a, &tiles_b, &items_b, &cnt_sorted}) release(c, *b);
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

  const size_t views_bytes = sizeof(ViewDev) * hv.size();
  const size_t edges_off = round_up(views_bytes, 256);
  const size_t dtab_off = round_up(edges_off + edges.size() * sizeof(float), 256);
  const size_t meta_bytes = dtab_off + dtab.size() * sizeof(float);
  TRY(acquire(c, meta_bytes, st, f->meta));
  TRY(ensure_pinned(c, std::max<size_t>(meta_bytes, 64)));
  // The previous call's read-back synchronised the stream, so the staging
  // buffer is free again.
  std::memcpy(c->pinned, hv.data(), views_bytes);
  std::memcpy((char*)c->pinned + edges_off, edges.data(), edges.size() * sizeof(float));
  std::memcpy((char*)c->pinned + dtab_off, dtab.data(), dtab.size() * sizeof(float));
  HTRY(hipMemcpyAsync(f->meta.p, c->pinned, meta_bytes, hipMemcpyHostToDevice, st));
  f->edges_off = edges_off;
  f->dtab_off = dtab_off;
  const ViewDev* d_views = (const ViewDev*)f->meta.p;
  const float* d_edges = (const float*)((char*)f->meta.p + edges_off);
  const float2* d_dtab = (const float2*)((char*)f->meta.p + dtab_off);

  // ---- stage (a): preprocess + PBF ----
  const int64_t it1 = std::max<int64_t>(items, 1);
  TRY(acquire(c, sizeof(Record) * it1, st, f->recs));
  TRY(acquire(c, sizeof(uint2) * it1, st, f->rects));
  TRY(acquire(c, 4 * it1, st, f->keys));
  TRY(acquire(c, 4 * it1, st, f->counts));
  TRY(acquire(c, 64, st, f->stats));  // [0] entries, [1] visible, [2] evaluated, [3] spare
  uint64_t* d_stats = (uint64_t*)f->stats.p;
  launch_fill_u32(st, (uint32_t*)d_stats, 8, 0u);
  ProfSlot* ps = prof_slot(c);
  prof_mark(ps, 0, st);
  launch_preprocess(st, n, n_views, scene->sh_degree, scene->mean, scene->scale, scene->quat, scene->opacity,
                    scene->sh, d_views, op, c->lam_dev, d_edges, (Record*)f->recs.p, (uint2*)f->rects.p,
                    (uint32_t*)f->keys.p, (uint32_t*)f->counts.p, (unsigned long long*)d_stats);
  HTRY(hipGetLastError());
  prof_mark(ps, 1, st);
  HTRY(hipMemcpyAsync(c->pinned, d_stats, 16, hipMemcpyDeviceToHost, st));
  HTRY(hipStreamSynchronize(st));
  uint64_t totals[2];
  std::memcpy(totals, c->pinned, 16);
  const int64_t E = (int64_t)totals[0], nvis = (int64_t)totals[1];
  if (totals[0] >= ((uint64_t)1 << 32) - 16)
    return cleanup(fail(c, GEER_ERR_CAPACITY, "association list of %llu entries exceeds 2^32",
                        (unsigned long long)totals[0]));
  f->entries = E;
  f->visible = nvis;

  // ---- stage (b): depth sort, expansion, tile sort, ranges ----
  const int64_t nv1 = std::max<int64_t>(nvis, 1), e1 = std::max<int64_t>(E, 1);
  const int64_t hist_words = radix_hist_words(std::max(items, E));
  TRY(acquire(c, 4 * nv1, st, ka));
  TRY(acquire(c, 4 * nv1, st, va));
  TRY(acquire(c, 4 * nv1, st, kb));
  TRY(acquire(c, 4 * nv1, st, vb));
  TRY(acquire(c, 4 * (size_t)hist_words, st, hist));
  TRY(acquire(c, 4 * (size_t)scan_scratch_words(std::max<int64_t>(hist_words, nv1)), st, scratch));
  TRY(acquire(c, 4 * nv1, st, cnt_sorted));
  TRY(acquire(c, 4 * (e1 + 8), st, tiles_a));
  TRY(acquire(c, 4 * (e1 + 8), st, tiles_b));
  TRY(acquire(c, 4 * (e1 + 8), st, f->list));
  TRY(acquire(c, 4 * (e1 + 8), st, items_b));
  TRY(acquire(c, 4 * (ntiles + 1), st, f->ranges));
  prof_mark(ps, 2, st);
  uint32_t* H = (uint32_t*)hist.p;
  uint32_t* SC = (uint32_t*)scratch.p;
  if (nvis > 0) {
    radix_pass(st, (const uint32_t*)f->keys.p, nullptr, (const uint32_t*)f->counts.p, items, 0, (uint32_t*)ka.p,
               (uint32_t*)va.p, H, SC);
    radix_pass(st, (uint32_t*)ka.p, (uint32_t*)va.p, nullptr, nvis, 8, (uint32_t*)kb.p, (uint32_t*)vb.p, H, SC);
    radix_pass(st, (uint32_t*)kb.p, (uint32_t*)vb.p, nullptr, nvis, 16, (uint32_t*)ka.p, (uint32_t*)va.p, H, SC);
    radix_pass(st, (uint32_t*)ka.p, (uint32_t*)va.p, nullptr, nvis, 24, (uint32_t*)kb.p, (uint32_t*)vb.p, H, SC);
    const uint32_t* sorted_items = (const uint32_t*)vb.p;
    launch_gather_counts(st, sorted_items, nvis, (const uint32_t*)f->counts.p, (uint32_t*)cnt_sorted.p);
    scan_exclusive(st, (uint32_t*)cnt_sorted.p, (uint32_t*)cnt_sorted.p, nvis, SC);
    // Expansion writes (tile, item) entries in depth order into buffer pair A
    // or B, chosen so that after the tile passes (alternating A <-> B) the
    // items end in f->list (pair B).
    uint32_t* tA = (uint32_t*)tiles_a.p;
    uint32_t* iA = (uint32_t*)items_b.p;
    uint32_t* tB = (uint32_t*)tiles_b.p;
    uint32_t* iB = (uint32_t*)f->list.p;
    const int passes = bytes_for_tiles(ntiles - 1);
    uint32_t* tc = (passes % 2 == 1) ? tA : tB;
    uint32_t* ic = (passes % 2 == 1) ? iA : iB;
    launch_expand(st, sorted_items, (const uint32_t*)cnt_sorted.p, nvis, E, (const uint2*)f->rects.p, d_views, n,
                  tc, ic);
    for (int p = 0; p < passes; ++p) {
      uint32_t* to = (tc == tA) ? tB : tA;
      uint32_t* io = (ic == iA) ? iB : iA;
      radix_pass(st, tc, ic, nullptr, E, 8 * p, to, io, H, SC);
      tc = to;
      ic = io;
    }
    const uint32_t* final_tiles = tc;
    uint32_t* i_out = iB;
    launch_fill_u32(st, i_out + E, 8, 0u);  // padding read by the 8-wide batches
    launch_ranges(st, final_tiles, E, ntiles, (uint32_t*)f->ranges.p);
  } else {
    launch_fill_u32(st, (uint32_t*)f->list.p, 8, 0u);
    launch_ranges(st, nullptr, 0, ntiles, (uint32_t*)f->ranges.p);
  }
  HTRY(hipGetLastError());

  // ---- stage (c): render ----
  const bool keep = frame_out != nullptr;
  if (keep) {
    TRY(acquire(c, 4 * npix, st, f->nlast));
    TRY(acquire(c, 4 * npix, st, f->tfinal));
  }
  prof_mark(ps, 3, st);
  launch_render(st, op.lambda_mode == 1, ntiles, d_views, n_views, d_dtab, (const uint32_t*)f->ranges.p,
                (const uint32_t*)f->list.p, (const uint2*)f->rects.p, (const Record*)f->recs.p, op, rgb, depth,
                trans, keep ? (uint32_t*)f->nlast.p : nullptr, keep ? (float*)f->tfinal.p : nullptr,
                (unsigned long long*)(d_stats + 2));
  HTRY(hipGetLastError());
  prof_mark(ps, 4, st);
  if (ps) HTRY(hipMemcpyAsync(ps->host_stats, d_stats, 32, hipMemcpyDeviceToHost, st));
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
  if (!f->nlast.p || !f->tfinal.p) return fail(c, GEER_ERR_INVALID_ARG, "frame holds no forward state");
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(c, hipSetDevice(c->device));
  if ((f->op.lambda_mode == 0) && (!c->lam_dev || c->lam_amin != f->op.alpha_min)) {
    geer_status s = lambda_dev(c, f->op.alpha_min, st);
    if (s != GEER_OK) return s;
  }
  Block acc;
  geer_status s = acquire(c, sizeof(float) * 16 * (size_t)std::max<int64_t>(f->items, 1), st, acc);
  if (s != GEER_OK) return s;
  const char* meta = (const char*)f->meta.p;
  const ViewDev* d_views = (const ViewDev*)meta;
  const float* d_edges = (const float*)(meta + f->edges_off);
  const float2* d_dtab = (const float2*)(meta + f->dtab_off);
  const geer_scene& sc = f->scene;
  launch_backward(st, f->op.lambda_mode == 1, f->ntiles, f->n, f->nviews, sc.sh_degree, sc.mean, sc.scale, sc.quat,
                  sc.opacity, sc.sh, d_views, d_dtab, d_edges, c->lam_dev, f->op, (const uint32_t*)f->ranges.p,
                  (const uint32_t*)f->list.p, (const uint2*)f->rects.p, (const Record*)f->recs.p,
                  (const uint32_t*)f->nlast.p, (const float*)f->tfinal.p, dl_drgb, (float*)acc.p, accumulate != 0,
                  g_mean, g_scale, g_quat, g_opacity, g_sh);
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

geer_status geer_frame_get_stats(const geer_frame* f, geer_frame_stats* out) {
  if (!f || !out) return GEER_ERR_INVALID_ARG;
  geer_ctx* c = f->ctx;
  uint64_t st[4];
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipMemcpyAsync(st, f->stats.p, sizeof st, hipMemcpyDeviceToHost, f->stream));
  HIP_TRY(c, hipStreamSynchronize(f->stream));
  out->n_items = f->items;
  out->n_visible = (int64_t)st[1];
  out->n_entries = (int64_t)st[0];
  out->n_tiles = f->ntiles;
  out->n_pixels = f->npix;
  out->n_evaluated = (int64_t)st[2];
  out->n_composited = -1;
  return GEER_OK;
}

int64_t geer_frame_buffer_bytes(const geer_frame* f, int32_t which) {
  if (!f) return -1;
  switch (which) {
    case GEER_BUF_RECT: return 8 * f->items;
    case GEER_BUF_COUNT: return 4 * f->items;
    case GEER_BUF_KEY: return 4 * f->items;
    case GEER_BUF_LIST: return 4 * f->entries;
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
      HIP_TRY(c, hipHostMalloc((void**)&ps.host_stats, 32, hipHostMallocDefault));
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
    float t01 = 0, t23 = 0, t34 = 0, t04 = 0;
    (void)hipEventElapsedTime(&t01, ps.ev[0], ps.ev[1]);
    (void)hipEventElapsedTime(&t23, ps.ev[2], ps.ev[3]);
    (void)hipEventElapsedTime(&t34, ps.ev[3], ps.ev[4]);
    (void)hipEventElapsedTime(&t04, ps.ev[0], ps.ev[4]);
    out[i].ms_preprocess = t01;
    out[i].ms_sort = t23;
    out[i].ms_render = t34;
    out[i].ms_total = t04;
    out[i].n_entries = (int64_t)ps.host_stats[0];
    out[i].n_evaluated = (int64_t)ps.host_stats[2];
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
  launch_l1(st, pixels, rgb, target, mask, dl_drgb, loss, partial, scale);
  hipError_t e = hipGetLastError();
  release(c, scratch);
  if (e != hipSuccess) return fail(c, GEER_ERR_HIP, "loss launch: %s", hipGetErrorString(e));
  return GEER_OK;
}

}  // extern "C"
