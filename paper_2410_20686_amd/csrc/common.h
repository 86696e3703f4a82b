// Shared device-side definitions of the gfx950 rasterizer (kernels + C ABI glue).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

#include "../../include/odgs.h"

namespace odgs {

constexpr int kWave = 64;  // CDNA wavefront width

inline bool plan_spherical(const odgs_plan* p) { return (p->s.flags & ODGS_FLAG_SPHERICAL) != 0; }

// Per-view geometry passed to kernels by value (kernel arguments are captured by HIP graphs).
struct ViewTable {
  int32_t n_views;
  int32_t W[ODGS_MAX_VIEWS];
  int32_t H[ODGS_MAX_VIEWS];
  int32_t tile_base[ODGS_MAX_VIEWS + 1];
  int64_t pix_base[ODGS_MAX_VIEWS + 1];
  float pin[ODGS_MAX_VIEWS][4];  // fx, fy, cx, cy of pinhole views; fx == 0: equirectangular
  int32_t dir_base[ODGS_MAX_VIEWS + 1];  // first entry of each view's ray table (W columns, then H rows)
  int32_t tile_base32[ODGS_MAX_VIEWS + 1];  // first global 32x32 tile id of each view (coarse binning)
};

// Half width at which horizontal offsets wrap round the +-pi seam: W/2 for ERP views, none
// (infinite) for pinhole views.
__device__ inline float wrap_half(const ViewTable& vt, int v) {
  return vt.pin[v][0] > 0.0f ? INFINITY : (float)vt.W[v] * 0.5f;
}

// Compositor record of one (Gaussian, view) item, three 16-byte words:
//   r0 = (u, v, l0, l1)        exponent -((l0 du + l1 dv)^2 + (l2 dv)^2), du = px - u, dv = py - v
//   r1 = (l2, opacity, p_min, eu)
//   r2 = (red, green, blue, ev)  eu, ev: padded half extents of the alpha >= 1/255 footprint
struct Rec {
  float4 r0, r1, r2;
};

// Compositor record of the spherical footprint, four 16-byte words:
//   s0 = (u1x, u1y, u1z, u2x), s1 = (u2y, u2z, wx, wy), s2 = (wz, k2, opacity, p_min), s3 = (r, g, b, 0)
// For a pixel ray d: t1 = u1 . d, t2 = u2 . d, h = w . d, qh = t1^2 + t2^2, D = h^2 + k2 qh; the
// Gaussian reaches the pixel iff h > 0 and p_min D + qh <= 0, with exponent -qh / D.
struct SphRec {
  float4 s0, s1, s2, s3;
};

// Culling data of a spherical-footprint item, read only while staging:
//   c0 = (mu^, beta)  the cone that holds every ray reaching alpha >= 1/255 (beta = pi: all rays);
//   c1 = (e1x, e1z, e2x, e2y), c2 = (e2z, p0x, p0y, M11), c3 = (M12, M22, rho, sqrt(lambda_max(M))):
//   in the gnomonic coordinates p = (d . e1, d . e2) / (d . mu^) of the tangent plane those rays
//   satisfy (p - p0)^T M (p - p0) <= rho^2 (rho < 0: no such ellipse, cone only).
struct SphCull {
  float4 c0, c1, c2, c3;
};

// Packed tile rectangle of an item: first column (may wrap), column count, first row, rows.
struct Rect {
  uint16_t col0, ncols, row0, nrows;
};

__host__ __device__ inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

__device__ inline int view_of_tile(const ViewTable& vt, int32_t g) {
  int v = 0;
  while (v + 1 < vt.n_views && g >= vt.tile_base[v + 1]) ++v;
  return v;
}

__device__ inline int view_of_item(int64_t item, int64_t n) { return (int)(item / n); }

// Tile scheduling of the compositors (one launch covers the tiles of every view).  Binning ends
// by building a work queue of all global tile ids, longest list first.  Persistent launches (as
// many workgroups as fit on the device at once) claim queue entries one at a time with an atomic
// counter, the last workgroup to find the queue empty clearing the counters for the next launch;
// otherwise one workgroup per task takes task blockIdx.x (order == nullptr: tile id blockIdx.x, no
// queue).
//
// A task is a whole tile or, for compositors that take them (split_cap > 0), one of four parts of
// a tile: binning counts the tiles whose lists reach the split length (at most split_cap of them,
// all at the front of the queue), and each of those becomes four tasks, so that a single long list
// is composited by four wavefronts at once instead of setting the launch's length by itself.
// Tasks 0 .. 4 nsplit - 1 are those parts (task e: part e % 4 of queue entry e / 4; of tile
// e / 4 without a queue), then come the remaining queue entries as whole tiles.  With split_all
// every tile is split (32x32 tiles composited as four 16x16 parts).
struct TileSched {
  const uint32_t* order;  // tile ids by descending list length, or nullptr
  uint32_t* ctr;          // persistent: {next task, finished workgroups}; nullptr: one task each
  odgs_status* status;
  uint32_t* split;        // {tiles split by binning, tiles split by the last forward}
  int32_t tiles;
  int32_t split_cap;      // 0: whole tiles only
  int32_t split_all;      // every tile in four parts (split_cap == tiles)
};

// Upper bound of the task count of a launch (its grid without a persistent launch).
inline int sched_tasks(const TileSched& s) { return s.tiles + 3 * s.split_cap; }

// Next task of this workgroup (uniform): returns its tile and sets `sel` to the part it covers
// (1 << part; 0xF: the whole tile), or returns -1 when the workgroup is done.  `nsplit` (uniform,
// at most split_cap) is the number of split tiles; `round` starts at 0; `slot` is a
// workgroup-shared word.  Contains barriers in persistent mode.
__device__ inline int claim_task(const TileSched& s, int nsplit, uint32_t& round, uint32_t* slot, uint32_t& sel) {
  const uint32_t total = (uint32_t)(s.tiles + 3 * nsplit);
  uint32_t e;
  if (!s.ctr) {
    if (round++) return -1;
    e = blockIdx.x;
    // The dispatcher hands workgroups to the 8 XCDs in turn, each with its own L2: the four parts
    // of a split tile (which stage the same list) go to four consecutive workgroups of one XCD
    // (groups of eight tiles, in queue order; the tail of an incomplete group stays in order).
    constexpr uint32_t kXcds = 8;
    if (e < (uint32_t)(nsplit / kXcds) * 4u * kXcds) {
      const uint32_t k = e / kXcds;
      e = 4u * ((k / 4u) * kXcds + e % kXcds) + k % 4u;
    }
  } else {
    __syncthreads();  // every thread has read the previous claim
    if (threadIdx.x == 0) {
      const uint32_t c = atomicAdd(&s.ctr[0], 1u);
      // queue drained: every workgroup passes here once, so the last one resets the counters
      if (c >= total && atomicAdd(&s.ctr[1], 1u) == gridDim.x - 1) {
        atomicExch(&s.ctr[0], 0u);
        atomicExch(&s.ctr[1], 0u);
      }
      *slot = c;
    }
    __syncthreads();
    e = *slot;
  }
  if (e >= total) return -1;
  uint32_t idx;
  if (e < 4u * (uint32_t)nsplit) {
    sel = 1u << (e & 3u);
    idx = e >> 2;
  } else {
    sel = 0xFu;
    idx = e - 3u * (uint32_t)nsplit;
  }
  return s.order ? (int)s.order[idx] : (int)idx;
}

// Next whole tile of this workgroup (compositors that take no quadrant tasks).
__device__ inline int claim_tile(const TileSched& s, uint32_t& round, uint32_t* slot) {
  uint32_t sel;
  return claim_task(s, 0, round, slot, sel);
}

// Split tiles of a forward launch (uniform): every tile with split_all, else what binning chose
// (within this launch's cap; none without the queue, which names the longest tiles).
__device__ inline int forward_split(const TileSched& s) {
  if (s.split_all) return s.tiles;
  return s.split_cap > 0 && s.order ? (int)min(s.split[0], (uint32_t)s.split_cap) : 0;
}
// Split tiles of a reverse launch: every tile with split_all, else those of the forward it follows
// (which wrote the culling masks of the split tiles' parts separately), within this launch's cap.
__device__ inline int reverse_split(const TileSched& s) {
  if (s.split_all) return s.tiles;
  return s.split_cap > 0 && s.order ? (int)min(s.split[1], (uint32_t)s.split_cap) : 0;
}

// The forward marks the pair list it composited, and how many tiles it split; the reverse
// compositor runs only on that list.
__device__ inline void mark_forward(const TileSched& s, int nsplit = 0) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    s.status->fwd_gen = s.status->bin_gen;
    s.split[1] = (uint32_t)nsplit;
  }
}
__device__ inline bool forward_is_stale(const TileSched& s) {
  const bool stale = s.status->fwd_gen != s.status->bin_gen;
  if (stale && blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&s.status->flags, ODGS_STATUS_STALE_FORWARD);
  return stale;
}

inline ViewTable make_view_table(const odgs_plan* p) {
  ViewTable vt{};
  vt.n_views = p->n_views;
  for (int v = 0; v < p->n_views; ++v) {
    vt.W[v] = p->width[v];
    vt.H[v] = p->height[v];
    for (int k = 0; k < 4; ++k) vt.pin[v][k] = p->pinhole[v][k];
  }
  for (int v = 0; v <= p->n_views; ++v) {
    vt.tile_base[v] = p->tile_base[v];
    vt.pix_base[v] = p->pix_base[v];
  }
  vt.dir_base[0] = 0;
  for (int v = 0; v < p->n_views; ++v) vt.dir_base[v + 1] = vt.dir_base[v] + p->width[v] + p->height[v];
  for (int v = 0; v <= p->n_views; ++v) vt.tile_base32[v] = p->tile_base32[v];
  return vt;
}

template <typename T>
inline T* ws_ptr(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}
template <typename T>
inline const T* ws_ptr(const void* ws, size_t off) {
  return reinterpret_cast<const T*>(static_cast<const char*>(ws) + off);
}

// Launchers implemented in the kernel translation units.
hipError_t launch_preprocess(const odgs_plan* p, const float* means, const float* scales, const float* quats,
                             const float* opac, const float* sh, const float* cams, void* ws, hipStream_t st);
hipError_t launch_bin_sort(const odgs_plan* p, void* ws, hipStream_t st);
hipError_t launch_render_fwd(const odgs_plan* p, void* ws, float* out_rgb, float* out_T, float* out_depth,
                             hipStream_t st);
hipError_t launch_render_bwd(const odgs_plan* p, void* ws, const float* dL_drgb, hipStream_t st);
hipError_t launch_render_sph_fwd(const odgs_plan* p, void* ws, float* out_rgb, float* out_T, float* out_depth,
                                 hipStream_t st);
hipError_t launch_render_sph_bwd(const odgs_plan* p, void* ws, const float* dL_drgb, hipStream_t st);
hipError_t launch_preprocess_bwd(const odgs_plan* p, const float* means, const float* scales, const float* quats,
                                 const float* opac, const float* sh, const float* cams, void* ws, float* d_means,
                                 float* d_scales, float* d_quats, float* d_opac, float* d_sh,
                                 const odgs_densify_acc* acc, hipStream_t st);
hipError_t launch_densify(int64_t n, int32_t sh_degree, const float* means, const float* scales, const float* quats,
                          const float* opac, const float* sh, const float* grad_sum, const float* tau_sum,
                          const int32_t* count, const float* noise, const odgs_densify_params& dp, int64_t capacity,
                          float* out_means, float* out_scales, float* out_quats, float* out_opac, float* out_sh,
                          int32_t* out_src, int64_t* out_counts, void* ws, hipStream_t st);
size_t densify_workspace_bytes(int64_t n);
size_t l1_workspace_bytes(int64_t count);
hipError_t launch_l1(const float* rgb, const float* tgt, int64_t count, float* dL, float* loss, void* ws,
                     hipStream_t st);
int64_t l1_noalloc_max_count();
hipError_t launch_l1_noalloc(const float* rgb, const float* tgt, int64_t count, float* dL, float* loss,
                             hipStream_t st);
hipError_t launch_adam_step(int64_t n, int32_t sh_degree, const odgs_param_ptrs& raw, const odgs_param_ptrs& act,
                            const odgs_param_ptrs& grad, const odgs_param_ptrs& m, const odgs_param_ptrs& v,
                            const float* lr, int32_t* step, const odgs_adam_hyper& hp, hipStream_t st);
hipError_t launch_fill_u32(uint32_t* ptr, uint32_t value, int64_t n, hipStream_t st);
hipError_t launch_status_reset(const odgs_plan* p, void* ws, hipStream_t st);
// Scheduling of a compositor launch: the queue, and for persistent launches the counter pair
// (which = 0 forward, 1 reverse) and the grid that fits `per_cu` workgroups on every CU.  Whole
// tiles only (split_cap 0); split_tile_cap gives the cap of compositors that take quadrant tasks.
TileSched make_sched(const odgs_plan* p, void* ws, int which);
int split_tile_cap(int tiles);
// The schedule of a compositor that takes quadrant tasks (only with the queue, which names the
// longest tiles).
inline TileSched with_split(TileSched s) {
  if (s.order) s.split_cap = split_tile_cap(s.tiles);
  return s;
}
// The schedule of a compositor that takes every tile in four parts.
inline TileSched with_parts(TileSched s) {
  s.split_cap = s.tiles;
  s.split_all = 1;
  return s;
}
int sched_grid(const TileSched& s, int per_cu);

// Launch of a compositor kernel whose last parameter is its TileSched: a persistent launch sizes
// its grid from the kernel's occupancy (workgroups resident per CU); otherwise one workgroup per
// tile.
template <typename... KArgs, typename... Args>
inline void launch_sched(void (*kernel)(KArgs...), const TileSched& s, int threads, hipStream_t st, Args&&... args) {
  int grid = sched_tasks(s);
  if (s.ctr) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess) per_cu = 1;
    grid = sched_grid(s, per_cu);
  }
  hipLaunchKernelGGL(kernel, dim3(grid), dim3(threads), 0, st, std::forward<Args>(args)..., s);
}
hipError_t launch_debug_records(const odgs_plan* p, const void* ws, float* out, hipStream_t st);
hipError_t launch_debug_pixel_counts(const odgs_plan* p, const void* ws, int32_t* out, hipStream_t st);
hipError_t launch_debug_g2d(const odgs_plan* p, const void* ws, double* out, hipStream_t st);
hipError_t launch_debug_keys(const odgs_plan* p, const void* ws, int64_t cap, uint64_t* keys, uint32_t* gauss,
                             hipStream_t st);

// Preprocess workgroups: one per (256-Gaussian chunk, group of views), the chunks padded to a
// multiple of 8 (the XCDs), each leaving one word of item counts in the radix histograms' region
// (at most n_views groups).
inline int64_t preprocess_blocks(int64_t n, int32_t groups) { return (n + 8 * 256 - 1) / (8 * 256) * 8 * groups; }

// Sort sizes: 256 threads x kSortIpt keys per block.
constexpr int kSortThreads = 256;
constexpr int kSortIpt = 16;
constexpr int kSortBlockItems = kSortThreads * kSortIpt;

}  // namespace odgs
