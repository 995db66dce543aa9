// Host-side tables and kernel launchers of libgeer (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <vector>

#include "geer.h"
#include "geer_common.h"

namespace geer {

// static_scratch.hip: the fixed device array of geer_render_static
hipError_t static_scratch_init(int device);  // with `device` current; looks its address up once
void* static_scratch_addr(int device);        // null until static_scratch_init succeeded
std::mutex& static_scratch_lock(int device);  // held by a call for as long as it uses the array

// tables.cpp
void lambda_table(float alpha_min, std::vector<float>& tab, int& lo, int& n);
float lambda_fixed_hat(float lambda_fixed);
void edge_tables(const geer_view& v, std::vector<float>& ex, std::vector<float>& ey);
void direction_tables(const geer_view& v, std::vector<float>& dx, std::vector<float>& dy);
void view_constants(const geer_view& v, ViewDev& d);
void valid_mask(const geer_view& v, uint8_t* mask);
// native-sensor sampling map of a view's BEAP grid: 4 int32 per native pixel
void reproject_map(const geer_view& v, int nw, int nh, std::vector<int32_t>& map);

// reproject.hip
void launch_reproject(hipStream_t st, const int4* map, int64_t npix, int W, int H, int C, const float* beap,
                      float* native, uint8_t* valid);

// preprocess.hip
void launch_preprocess(hipStream_t st, int64_t n, int32_t n_views, int32_t sh_degree, const float* mean,
                       const float* scale, const float* quat, const float* opacity, const float* sh,
                       const ViewDev* views, const Opts& op, const float* lam_tab, const float* edges,
                       Record* recs, uint2* rects, uint32_t* keys, uint32_t* counts, unsigned long long* totals,
                       int totals_stride, const unsigned long long* err_in = nullptr, bool defer_colour = false);
// The colour of a batch of views that launch_preprocess deferred (no-op when
// it had none to defer: one view, or SH degree 0).  Touches only the records'
// rgb, which the association never reads.
void launch_colour(hipStream_t st, int64_t n, int32_t n_views, int32_t sh_degree, const float* mean,
                   const float* sh, const ViewDev* views, const uint32_t* counts, Record* recs);

// sort.hip
int64_t scan_scratch_words(int64_t n);
void scan_exclusive(hipStream_t st, const uint32_t* in, uint32_t* out, int64_t n, uint32_t* scratch);
// Depth order of the visible items (four 8-bit passes over the depth keys;
// pass 0 keeps items with counts[i] != 0 out of all n0 items, later passes
// read the live visible count dyn1, or n1_cap): the items in depth order end
// in vb, offs[j] = exclusive prefix of their tile counts.  work:
// depth_work_words(n0) words whose first depth_zero_words(n0) are zero unless
// `zeroed` is false (then the call clears them).
int64_t depth_work_words(int64_t n0);
int64_t depth_zero_words(int64_t n0);
// Polls of a radix pass's look-back before it gives up and sets the error
// word (about a second of waiting).
constexpr uint32_t kDefaultSpinLimit = 1u << 22;
void depth_order(hipStream_t st, const uint32_t* keys, const uint32_t* counts, int64_t n0, int64_t n1_cap,
                 const unsigned long long* dyn1, uint32_t* work, bool zeroed, uint32_t* ka, uint32_t* va,
                 uint32_t* kb, uint32_t* vb, uint32_t* offs, uint32_t* owners, int64_t owners_n,
                 unsigned long long* err, bool tickets, uint32_t spin_limit);
// words of the table of expansion-block owners for lists of up to ecap entries
int64_t owner_words(int64_t ecap);
// Work of the expansion and the tile sort for up to ecap entries:
// tile_work_words(ecap) words whose first tile_zero_words(ecap) must be zero
// before the expansion.
int64_t tile_work_words(int64_t ecap);
int64_t tile_zero_words(int64_t ecap);
// Stable sort of the entries (tile ids tin, items iin; the live count dE, or
// ecap) by `passes` digits of `bits` bits, leaving out the entries the
// expansion marked as culled; the number kept goes to *kept.  Passes write
// (at, ai), (bt, bi), (at, ai), ...  With hpass, the expansion counted the
// digits of the first hpass passes into twork.
void tile_sort(hipStream_t st, const uint32_t* tin, const uint32_t* iin, int64_t ecap,
               const unsigned long long* dE, unsigned long long* kept, int passes, int bits, uint32_t* at,
               uint32_t* ai, uint32_t* bt, uint32_t* bi, uint32_t* twork, int hpass, unsigned long long* err,
               bool tickets, uint32_t spin_limit);
// Bytes of the expansion's per-tile cull table; its launch also sets
// zero[0 .. nzero) = 0.
size_t tile_cone_bytes(int64_t ntiles);
void launch_tile_cones(hipStream_t st, const ViewDev* views, int nviews, const float2* dtab, int64_t ntiles,
                       float4* out, uint32_t* zero, int64_t nzero);
// Expansion of the depth-ordered items into their tile entries in depth
// order; the culled ones get the tile id 0xffffffff.  With hpass, the kept
// entries' tile digits are counted into the partial histograms of twork.
void launch_expand(hipStream_t st, const uint32_t* items, const uint32_t* offs, int64_t m_cap,
                   const unsigned long long* dyn_m, int64_t total_cap, const unsigned long long* dyn_total,
                   const uint2* rects, const ViewDev* views, int64_t n, const float4* tcones, const Record* recs,
                   const Opts& op, uint32_t* tiles_out, uint32_t* items_out, uint32_t* twork, int hpass,
                   int hbits, int64_t nitems, int64_t ntiles, const uint32_t* owners);
int hist_parts_words();
// with list: also zeroes the 8 words of padding after the list; with err:
// every range is empty when the sort's error word is set
void launch_ranges(hipStream_t st, const uint32_t* tiles, int64_t total_cap, const unsigned long long* dyn,
                   int64_t ntiles, uint32_t* ranges, uint32_t* list = nullptr,
                   const unsigned long long* err = nullptr);
void launch_zero2_u32(hipStream_t st, uint32_t* p1, int64_t n1, uint32_t* p2, int64_t n2);
void launch_capacity_guard(hipStream_t st, unsigned long long* stats, int64_t cap);
void launch_fill_u32(hipStream_t st, uint32_t* p, int64_t n, uint32_t v);

// render.hip
int heavy_capacity(int64_t ntiles);
int64_t heavy_evals_offset(int hmax);     // u32 words from the list to the evaluated-pair counters
int64_t heavy_list_words(int64_t ntiles);  // u32 words of the list buffer
int heavy_slots(int hmax);
void launch_mark_heavy(hipStream_t st, const uint32_t* ranges, int64_t ntiles, const ViewDev* views, int nviews,
                       const HeavyTiles& h);
void launch_render(hipStream_t st, bool fixed_lambda, int64_t ntiles, const ViewDev* views, int nviews,
                   const float2* dtab, const uint32_t* ranges, const uint32_t* list, const uint2* rects,
                   const Record* recs, const Opts& op, const HeavyTiles& heavy, float* rgb, float* depth,
                   float* trans, uint32_t* nlast, float* tfinal, unsigned long long* stats);

void launch_render_splat(hipStream_t st, int64_t ntiles, const ViewDev* views, int nviews, const float2* dtab,
                         const uint32_t* ranges, const uint32_t* list, const uint2* rects, const Record* recs,
                         const Opts& op, float* rgb, float* depth, float* trans);

// backward.hip
void launch_backward(hipStream_t st, bool fixed_lambda, int64_t ntiles, int64_t n, int32_t n_views,
                     int32_t sh_degree, const float* mean, const float* scale, const float* quat,
                     const float* opacity, const float* sh, const ViewDev* views, const float2* dtab,
                     const float* edges, const float* lam_tab, const Opts& op, const HeavyTiles& heavy,
                     const uint32_t* ranges, const uint32_t* list, const uint2* rects, const Record* recs,
                     const uint32_t* counts, const uint32_t* nlast,
                     const float* tfinal, const float* dl_drgb, float* acc, int accumulate, float* g_mean,
                     float* g_scale, float* g_quat, float* g_opacity, float* g_sh,
                     unsigned long long* counters = nullptr);

// counters: optional replay pair counters (kEvalSlots slots kEvalStride apart,
// then the total), cleared here and filled by launch_render_backward
void launch_zero_acc(hipStream_t st, float* acc, const uint32_t* counts, int64_t nitems,
                     unsigned long long* counters = nullptr);
void launch_render_backward(hipStream_t st, bool fixed_lambda, int64_t ntiles, int32_t n_views, const ViewDev* views,
                            const float2* dtab, const Opts& op, const HeavyTiles& heavy, const uint32_t* ranges,
                            const uint32_t* list, const uint2* rects, const Record* recs, const uint32_t* nlast,
                            const float* tfinal, const float* dl_drgb, float* acc,
                            unsigned long long* counters = nullptr);
void launch_preprocess_backward(hipStream_t st, int64_t n, int32_t n_views, int32_t sh_degree, const float* mean,
                                const float* scale, const float* quat, const float* opacity, const float* sh,
                                const ViewDev* views, const float* edges, const float* lam_tab, const Opts& op,
                                const uint32_t* counts, const float* acc, const Record* recs, int accumulate,
                                float* g_mean, float* g_scale, float* g_quat, float* g_opacity, float* g_sh);

// train.hip (raw parameter rows: mean 3, log scale 3, quaternion 4, opacity logit 1, SH 3K)
void launch_activate(hipStream_t st, int64_t n, const float* raw, float* scale_out, float* opac_out);
void launch_adam(hipStream_t st, int64_t n, int sh_degree, float* raw, const float* g_mean, const float* g_scale,
                 const float* g_quat, const float* g_opac, const float* g_sh, float* m, float* v, float* scale_out,
                 float* opac_out, float* accum, float* count, const AdamParams& ap);
void launch_densify_count(hipStream_t st, int64_t n, const float* raw, const float* accum, const float* count,
                          const DensifyParams& dp, uint32_t* nout, uint32_t* kind);
void launch_densify_apply(hipStream_t st, int64_t n, int sh_degree, const float* raw, const float* m, const float* v,
                          const uint32_t* kind, const uint32_t* offs, const float* noise, int64_t n_out, float* raw_o,
                          float* m_o, float* v_o, float* scale_o, float* opac_o, float* accum_o, float* count_o,
                          float split_shrink);

// loss.hip
int64_t l1_partial_count(int64_t P);
void launch_l1(hipStream_t st, int64_t P, const float* rgb, const float* target, const uint8_t* mask, float* dl,
               float* loss, float2* partial, float* scale, double weight);
void launch_sum_f32(hipStream_t st, int n, const float* in, float* out);

}  // namespace geer
