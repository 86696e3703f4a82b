// C ABI of the gfx950 omnidirectional rasterizer: plan / workspace layout, argument checks and
// the entry points declared in include/odgs.h.  No allocation, no synchronisation, no global
// mutable state: every entry point validates on the host and enqueues kernels on the stream.
#include <string.h>

#include "common.h"

namespace odgs {
namespace {

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

int check_ws(const odgs_plan* p, const void* ws, size_t ws_bytes) {
  if (!p) return ODGS_EINVAL;
  if (p->ws_bytes > 0 && (!ws || !aligned(ws, 256))) return ODGS_EINVAL;
  if (ws_bytes < p->ws_bytes) return ODGS_ENOSPACE;
  return ODGS_OK;
}

int check_params(const odgs_plan* p, const float* means, const float* scales, const float* quats, const float* opac,
                 const float* sh, const float* cams) {
  if (!cams || !aligned(cams, 4)) return ODGS_EINVAL;
  if (p->n == 0) return ODGS_OK;
  const float* ptrs[5] = {means, scales, quats, opac, sh};
  for (const float* q : ptrs)
    if (!q || !aligned(q, 4)) return ODGS_EINVAL;
  return ODGS_OK;
}

int hip_status(hipError_t e) { return e == hipSuccess ? ODGS_OK : ODGS_EHIP; }

// Default threshold of coarse binning.  Measured at tile 16: one 4096x2048 view (32,768 tiles)
// bins in 0.29 instead of 0.38 ms and eight 2048x1024 views (65,536) in 0.84 instead of 0.97 ms;
// one 2048x1024 view (8,192) gains nothing, and a 256x128 view (128) pays for the extra launches.
constexpr int64_t kCoarseMinTiles = 16384;

bool batch_ok(int tile, int batch) {
  if (tile == 8 || tile == 16) return batch == 32 || batch == 64 || batch == 128 || batch == 256;
  if (tile == 32) return batch == 64 || batch == 128 || batch == 256;
  return false;
}

}  // namespace
}  // namespace odgs

using namespace odgs;

extern "C" {

size_t odgs_plan_size(void) { return sizeof(odgs_plan); }

int odgs_plan_set_pinhole(odgs_plan* plan, int32_t view, float fx, float fy, float cx, float cy) {
  if (!plan || view < 0 || view >= plan->n_views) return ODGS_EINVAL;
  if (plan_spherical(plan)) return ODGS_EINVAL;  // the spherical footprint is defined for ERP views
  if (!(fx > 0.0f) || !(fy > 0.0f) || !std::isfinite(fx) || !std::isfinite(fy) || !std::isfinite(cx) ||
      !std::isfinite(cy))
    return ODGS_EINVAL;
  plan->pinhole[view][0] = fx;
  plan->pinhole[view][1] = fy;
  plan->pinhole[view][2] = cx;
  plan->pinhole[view][3] = cy;
  return ODGS_OK;
}

int odgs_plan_init(odgs_plan* plan, int64_t n, int32_t sh_degree, int32_t n_views, const int32_t* wh,
                   const odgs_settings* s, int64_t pair_capacity) {
  if (!plan || !wh || !s) return ODGS_EINVAL;
  if (n < 0 || sh_degree < 0 || sh_degree > 3 || n_views < 1 || n_views > ODGS_MAX_VIEWS) return ODGS_EINVAL;
  if (pair_capacity < 0 || pair_capacity >= (int64_t(1) << 31)) return ODGS_EINVAL;
  if (n * (int64_t)n_views >= (int64_t(1) << 31)) return ODGS_EINVAL;
  odgs_settings st = *s;
  if (st.tile != 8 && st.tile != 16 && st.tile != 32) return ODGS_EINVAL;
  // one-wavefront compositors (16x16 blocks) stage 64 entries at a time; the spherical footprint's
  // 32x32 compositors have a workgroup of 1024 threads to fill
  const bool sph32 = st.tile == 32 && (st.flags & ODGS_FLAG_SPHERICAL);
  if (st.batch == 0) st.batch = sph32 ? 256 : 64;
  if (st.batch_bwd == 0) st.batch_bwd = st.tile == 8 ? 32 : (sph32 ? 256 : 64);
  if (!batch_ok(st.tile, st.batch) || !batch_ok(st.tile, st.batch_bwd)) return ODGS_EINVAL;
  if (st.flags & ~(ODGS_FLAG_COUNT_WORK | ODGS_FLAG_SPHERICAL | ODGS_FLAG_SCHED_PERSISTENT | ODGS_FLAG_SCHED_TILE_ID |
                   ODGS_FLAG_BIN_COARSE | ODGS_FLAG_BIN_DIRECT))
    return ODGS_EINVAL;
  if ((st.flags & ODGS_FLAG_SCHED_PERSISTENT) && (st.flags & ODGS_FLAG_SCHED_TILE_ID)) return ODGS_EINVAL;
  if ((st.flags & ODGS_FLAG_BIN_COARSE) && (st.flags & ODGS_FLAG_BIN_DIRECT)) return ODGS_EINVAL;
  if ((st.flags & ODGS_FLAG_COUNT_WORK) && (st.flags & ODGS_FLAG_SPHERICAL)) return ODGS_EINVAL;
  if (!(st.near_r >= 0.0f) || !(st.far_r > st.near_r) || !(st.dilation >= 0.0f) || !(st.pole_eps >= 0.0f))
    return ODGS_EINVAL;
  memset(plan, 0, sizeof(*plan));
  plan->n = n;
  plan->sh_degree = sh_degree;
  plan->n_views = n_views;
  plan->s = st;
  int64_t tiles = 0, pixels = 0;
  for (int v = 0; v < n_views; ++v) {
    const int W = wh[2 * v], H = wh[2 * v + 1];
    if (W <= 0 || H <= 0 || W % st.tile || H % st.tile || W / st.tile > 65535 || H / st.tile > 65535)
      return ODGS_EINVAL;
    plan->width[v] = W;
    plan->height[v] = H;
    plan->tile_base[v] = (int32_t)tiles;
    plan->pix_base[v] = pixels;
    tiles += (int64_t)(W / st.tile) * (H / st.tile);
    pixels += (int64_t)W * H;
    // up to four compositing tasks per tile must fit a launch grid
    if (tiles >= (int64_t(1) << 29) || pixels >= (int64_t(1) << 40)) return ODGS_EINVAL;
  }
  plan->tile_base[n_views] = (int32_t)tiles;
  plan->pix_base[n_views] = pixels;
  plan->items = n * n_views;
  plan->pair_capacity = pair_capacity;
  int bits = 1;
  while ((int64_t(1) << bits) < tiles) ++bits;
  plan->tile_bits = bits;
  plan->item_blocks = (int32_t)((plan->items + kSortBlockItems - 1) / kSortBlockItems);
  if (plan->item_blocks < 1) plan->item_blocks = 1;
  plan->pair_blocks = (int32_t)((pair_capacity + kSortBlockItems - 1) / kSortBlockItems);
  if (plan->pair_blocks < 1) plan->pair_blocks = 1;
  plan->depth_final = (4 % 2);                  // 4 passes of 8 bits over 32-bit depths
  plan->pair_final = ((bits + 7) / 8) % 2;      // passes over the tile bits
  // Coarse binning at 16x16 tiles: pairs by 32x32 tile (about half as many), sorted, then split
  // into the four 16x16 tiles' lists, which land in the other pair buffer.  By default from
  // kCoarseMinTiles tiles on (below, its three extra launches cost more than the sort saves).
  int64_t tiles32 = 0;
  bool coarse = st.tile == 16 && !(st.flags & ODGS_FLAG_BIN_DIRECT) &&
                ((st.flags & ODGS_FLAG_BIN_COARSE) || tiles >= kCoarseMinTiles);
  for (int v = 0; v < n_views; ++v) coarse = coarse && wh[2 * v] % 32 == 0 && wh[2 * v + 1] % 32 == 0;
  for (int v = 0; v < n_views; ++v) {
    plan->tile_base32[v] = (int32_t)tiles32;
    if (coarse) tiles32 += (int64_t)(wh[2 * v] / 32) * (wh[2 * v + 1] / 32);
  }
  plan->tile_base32[n_views] = (int32_t)tiles32;
  int cbits = 1;
  while ((int64_t(1) << cbits) < tiles32) ++cbits;
  if (cbits > 24) coarse = false;  // the sort passes must leave the mask bits (28..31) of the keys alone
  plan->coarse = coarse ? 1 : 0;
  plan->coarse_bits = coarse ? cbits : 0;
  if (coarse) plan->pair_final = (((cbits + 7) / 8) % 2) ^ 1;
  const int64_t I = plan->items;
  const int64_t sblocks = (I + 1023) / 1024 + 1;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes, 256);
    return o;
  };
  plan->off_status = take(256);
  plan->off_rec = take((size_t)I * sizeof(Rec));
  plan->off_rect = take((size_t)I * sizeof(Rect));
  plan->off_count = take((size_t)I * 4);
  plan->off_depth = take((size_t)I * 4);
  plan->off_dkey[0] = take((size_t)I * 4);
  plan->off_dkey[1] = take((size_t)I * 4);
  plan->off_did[0] = take((size_t)I * 4);
  plan->off_did[1] = take((size_t)I * 4);
  plan->off_srect = take((size_t)I * sizeof(Rect));
  plan->off_blocksum = take(align_up((size_t)sblocks, 64) * 4 + (size_t)sblocks * 8);
  plan->off_pkey[0] = take((size_t)pair_capacity * 4);
  plan->off_pkey[1] = take((size_t)pair_capacity * 4);
  plan->off_pval[0] = take((size_t)pair_capacity * 4);
  plan->off_pval[1] = take((size_t)pair_capacity * 4);
  const int64_t hb = plan->item_blocks > plan->pair_blocks ? plan->item_blocks : plan->pair_blocks;
  // radix histograms; before binning the preprocess workgroups' item counts, after the pair sort
  // the coarse refinement's per-chunk counts (16 bytes per sort block), then the tile queue's
  // per-(block, bucket) counts
  const int64_t qwords = (tiles + 4095) / 4096 * 1024;
  int64_t hwords = 256 * hb > qwords ? 256 * hb : qwords;
  if (hwords < preprocess_blocks(n, n_views)) hwords = preprocess_blocks(n, n_views);
  plan->off_hist = take((size_t)hwords * 4);
  plan->off_digit = take(256 * 4);
  plan->off_ranges = take((size_t)tiles * 8);
  plan->off_T = take((size_t)pixels * 4);
  plan->off_last = take((size_t)pixels * 4);
  plan->off_ncontrib = take((size_t)pixels * 4);
  plan->off_neval = take((size_t)pixels * 4);
  plan->off_lasteval = take((size_t)pixels * 4);
  const bool sph = (st.flags & ODGS_FLAG_SPHERICAL) != 0;
  plan->g2d_stride = sph ? 13 : 9;
  plan->off_g2d = take((size_t)plan->g2d_stride * I * 8);  // double
  plan->off_queue = take(64 + (size_t)tiles * 4);  // counters (forward, reverse), then the tile queue
  int64_t dirs = 0;
  for (int v = 0; v < n_views; ++v) dirs += plan->width[v] + plan->height[v];
  plan->off_srec = take(sph ? (size_t)I * sizeof(SphRec) : 0);
  plan->off_cone = take(sph ? (size_t)I * sizeof(SphCull) : 0);
  plan->off_dirs = take(sph ? (size_t)dirs * 16 : 0);
  plan->ws_bytes = off;
  return ODGS_OK;
}

size_t odgs_workspace_bytes(const odgs_plan* plan) { return plan ? plan->ws_bytes : 0; }

size_t odgs_status_offset(const odgs_plan* plan) { return plan ? plan->off_status : 0; }

int odgs_preprocess(const odgs_plan* plan, const float* means, const float* scales, const float* quats,
                    const float* opacities, const float* sh, const float* cams, void* ws, size_t ws_bytes,
                    void* stream) {
  int rc = check_ws(plan, ws, ws_bytes);
  if (rc != ODGS_OK) return rc;
  rc = check_params(plan, means, scales, quats, opacities, sh, cams);
  if (rc != ODGS_OK) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = launch_status_reset(plan, ws, st);
  if (e == hipSuccess) e = launch_preprocess(plan, means, scales, quats, opacities, sh, cams, ws, st);
  return hip_status(e);
}

int odgs_bin_sort(const odgs_plan* plan, void* ws, size_t ws_bytes, void* stream) {
  const int rc = check_ws(plan, ws, ws_bytes);
  if (rc != ODGS_OK) return rc;
  return hip_status(launch_bin_sort(plan, ws, static_cast<hipStream_t>(stream)));
}

int odgs_render_fwd(const odgs_plan* plan, void* ws, size_t ws_bytes, float* out_rgb, float* out_T, float* out_depth,
                    void* stream) {
  const int rc = check_ws(plan, ws, ws_bytes);
  if (rc != ODGS_OK) return rc;
  if (!out_rgb || !aligned(out_rgb, 4) || (out_T && !aligned(out_T, 4)) || (out_depth && !aligned(out_depth, 4)))
    return ODGS_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (plan_spherical(plan)) return hip_status(launch_render_sph_fwd(plan, ws, out_rgb, out_T, out_depth, st));
  return hip_status(launch_render_fwd(plan, ws, out_rgb, out_T, out_depth, st));
}

int odgs_composite_bwd(const odgs_plan* plan, void* ws, size_t ws_bytes, const float* dL_drgb, void* stream) {
  const int rc = check_ws(plan, ws, ws_bytes);
  if (rc != ODGS_OK) return rc;
  if (!dL_drgb || !aligned(dL_drgb, 4)) return ODGS_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (plan_spherical(plan)) return hip_status(launch_render_sph_bwd(plan, ws, dL_drgb, st));
  return hip_status(launch_render_bwd(plan, ws, dL_drgb, st));
}

int odgs_project_bwd(const odgs_plan* plan, const float* means, const float* scales, const float* quats,
                     const float* opacities, const float* sh, const float* cams, void* ws, size_t ws_bytes,
                     float* d_means, float* d_scales, float* d_quats, float* d_opacities, float* d_sh,
                     const odgs_densify_acc* acc, void* stream) {
  int rc = check_ws(plan, ws, ws_bytes);
  if (rc != ODGS_OK) return rc;
  rc = check_params(plan, means, scales, quats, opacities, sh, cams);
  if (rc != ODGS_OK) return rc;
  if (plan->n > 0) {
    float* outs[5] = {d_means, d_scales, d_quats, d_opacities, d_sh};
    for (float* q : outs)
      if (!q || !aligned(q, 4)) return ODGS_EINVAL;
    if (acc) {
      if (plan_spherical(plan)) return ODGS_EINVAL;  // statistics are defined on the 2D mean
      if (!acc->grad_sum || !acc->tau_sum || !acc->count) return ODGS_EINVAL;
      if (!aligned(acc->grad_sum, 4) || !aligned(acc->tau_sum, 4) || !aligned(acc->count, 4)) return ODGS_EINVAL;
      if (!std::isfinite(acc->tau_min) || !std::isfinite(acc->tau_max)) return ODGS_EINVAL;
    }
  }
  return hip_status(launch_preprocess_bwd(plan, means, scales, quats, opacities, sh, cams, ws, d_means, d_scales,
                                          d_quats, d_opacities, d_sh, acc, static_cast<hipStream_t>(stream)));
}

size_t odgs_l1_loss_workspace_bytes(int64_t count) { return count < 0 ? 0 : l1_workspace_bytes(count); }

int odgs_l1_loss(const float* rgb, const float* target, int64_t count, float* dL, float* loss, void* ws,
                 size_t ws_bytes, void* stream) {
  if (count < 0 || !loss || !aligned(loss, 4) || !ws || !aligned(ws, 256)) return ODGS_EINVAL;
  if (count > 0 && (!rgb || !target || !dL || !aligned(rgb, 4) || !aligned(target, 4) || !aligned(dL, 4)))
    return ODGS_EINVAL;
  if (ws_bytes < l1_workspace_bytes(count)) return ODGS_ENOSPACE;
  return hip_status(launch_l1(rgb, target, count, dL, loss, ws, static_cast<hipStream_t>(stream)));
}

int odgs_l1_loss_noalloc(const float* rgb, const float* target, int64_t count, float* dL, float* loss, void* stream) {
  if (count < 0 || !loss || !aligned(loss, 4)) return ODGS_EINVAL;
  if (count > 0 && (!rgb || !target || !dL || !aligned(rgb, 4) || !aligned(target, 4) || !aligned(dL, 4)))
    return ODGS_EINVAL;
  if (count > l1_noalloc_max_count()) return ODGS_ETOOBIG;
  return hip_status(launch_l1_noalloc(rgb, target, count, dL, loss, static_cast<hipStream_t>(stream)));
}

namespace {
bool params_ok(const odgs_param_ptrs* p) {
  if (!p) return false;
  const float* a[5] = {p->means, p->scales, p->quats, p->opacities, p->sh};
  for (const float* q : a)
    if (!q || !aligned(q, 4)) return false;
  return true;
}
}  // namespace

int odgs_adam_step(int64_t n, int32_t sh_degree, const odgs_param_ptrs* raw, const odgs_param_ptrs* act,
                   const odgs_param_ptrs* grad, const odgs_param_ptrs* m, const odgs_param_ptrs* v, const float* lr,
                   int32_t* step, const odgs_adam_hyper* hp, void* stream) {
  if (n < 0 || sh_degree < 0 || sh_degree > 3 || !hp || !lr || !step || !aligned(lr, 4) || !aligned(step, 4))
    return ODGS_EINVAL;
  if (!(hp->beta1 >= 0.0f && hp->beta1 < 1.0f && hp->beta2 >= 0.0f && hp->beta2 < 1.0f && hp->eps >= 0.0f))
    return ODGS_EINVAL;
  if (!raw || !act || !grad || !m || !v) return ODGS_EINVAL;
  if (n > 0 && !(params_ok(raw) && params_ok(act) && params_ok(grad) && params_ok(m) && params_ok(v)))
    return ODGS_EINVAL;
  return hip_status(launch_adam_step(n, sh_degree, *raw, *act, *grad, *m, *v, lr, step, *hp,
                                     static_cast<hipStream_t>(stream)));
}

size_t odgs_densify_workspace_bytes(int64_t n) { return n < 0 ? 0 : densify_workspace_bytes(n); }

int odgs_densify(int64_t n, int32_t sh_degree, const float* means, const float* scales, const float* quats,
                 const float* opacities, const float* sh, const float* grad_sum, const float* tau_sum,
                 const int32_t* count, const float* noise, const odgs_densify_params* dp, int64_t capacity,
                 float* out_means, float* out_scales, float* out_quats, float* out_opacities, float* out_sh,
                 int32_t* out_src, int64_t* out_counts, void* ws, size_t ws_bytes, void* stream) {
  if (n < 0 || n >= ((int64_t)1 << 30) || sh_degree < 0 || sh_degree > 3 || !dp) return ODGS_EINVAL;
  if (!out_counts || !aligned(out_counts, 8) || !ws || !aligned(ws, 256)) return ODGS_EINVAL;
  if (capacity < 2 * n) return ODGS_EINVAL;
  if (!std::isfinite(dp->extent) || !std::isfinite(dp->percent_dense) || !std::isfinite(dp->min_opacity) ||
      !std::isfinite(dp->max_scale_frac) || dp->max_scale_frac < 0.0f)
    return ODGS_EINVAL;
  if (ws_bytes < densify_workspace_bytes(n)) return ODGS_ENOSPACE;
  if (n > 0) {
    const void* in[10] = {means, scales, quats, opacities, sh, grad_sum, tau_sum, count, noise, nullptr};
    for (int k = 0; k < 9; ++k)
      if (!in[k] || !aligned(in[k], 4)) return ODGS_EINVAL;
    const void* out[6] = {out_means, out_scales, out_quats, out_opacities, out_sh, out_src};
    for (const void* q : out)
      if (!q || !aligned(q, 4)) return ODGS_EINVAL;
  }
  return hip_status(launch_densify(n, sh_degree, means, scales, quats, opacities, sh, grad_sum, tau_sum, count, noise,
                                   *dp, capacity, out_means, out_scales, out_quats, out_opacities, out_sh, out_src,
                                   out_counts, ws, static_cast<hipStream_t>(stream)));
}

int odgs_render_bwd(const odgs_plan* plan, const float* means, const float* scales, const float* quats,
                    const float* opacities, const float* sh, const float* cams, void* ws, size_t ws_bytes,
                    const float* dL_drgb, float* d_means, float* d_scales, float* d_quats, float* d_opacities,
                    float* d_sh, const odgs_densify_acc* acc, void* stream) {
  int rc = check_ws(plan, ws, ws_bytes);
  if (rc != ODGS_OK) return rc;
  rc = check_params(plan, means, scales, quats, opacities, sh, cams);
  if (rc != ODGS_OK) return rc;
  if (!dL_drgb || !aligned(dL_drgb, 4)) return ODGS_EINVAL;
  if (acc && plan_spherical(plan)) return ODGS_EINVAL;
  rc = odgs_composite_bwd(plan, ws, ws_bytes, dL_drgb, stream);
  if (rc != ODGS_OK) return rc;
  return odgs_project_bwd(plan, means, scales, quats, opacities, sh, cams, ws, ws_bytes, d_means, d_scales, d_quats,
                          d_opacities, d_sh, acc, stream);
}

const char* odgs_strerror(int code) {
  switch (code) {
    case ODGS_OK: return "success";
    case ODGS_EINVAL: return "invalid argument";
    case ODGS_ENOSPACE: return "workspace too small";
    case ODGS_EHIP: return "HIP kernel launch failed";
    case ODGS_ETOOBIG: return "input larger than the static scratch of a no-allocation entry point";
    default: return "unknown error";
  }
}

int odgs_debug_records(const odgs_plan* plan, const void* ws, float* out, void* stream) {
  if (!plan || !ws || !out) return ODGS_EINVAL;
  return hip_status(launch_debug_records(plan, ws, out, static_cast<hipStream_t>(stream)));
}

int odgs_debug_g2d(const odgs_plan* plan, const void* ws, double* out, void* stream) {
  if (!plan || !ws || (plan->items > 0 && !out)) return ODGS_EINVAL;
  return hip_status(launch_debug_g2d(plan, ws, out, static_cast<hipStream_t>(stream)));
}

int odgs_debug_pixel_counts(const odgs_plan* plan, const void* ws, int32_t* out, void* stream) {
  if (!plan || !ws || !out) return ODGS_EINVAL;
  return hip_status(launch_debug_pixel_counts(plan, ws, out, static_cast<hipStream_t>(stream)));
}

int odgs_debug_keys(const odgs_plan* plan, const void* ws, int64_t cap, uint64_t* keys, uint32_t* gauss,
                    void* stream) {
  if (!plan || !ws || cap < 0 || (cap > 0 && (!keys || !gauss))) return ODGS_EINVAL;
  return hip_status(launch_debug_keys(plan, ws, cap, keys, gauss, static_cast<hipStream_t>(stream)));
}

}  // extern "C"
