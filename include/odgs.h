/*
 * odgs.h -- C ABI of the MI355X (gfx950) omnidirectional Gaussian rasterizer.
 *
 * Implements the rasterizer of ODGS (Lee et al., NeurIPS 2024, arXiv 2410.20686): every 3D
 * Gaussian is projected perspectively onto the plane tangent to the unit sphere along the ray
 * to its centre and mapped into equirectangular (ERP) pixel space (Sec. 3.2, Eq. equirec_proj,
 * Eq. omni_rotation, Eq. omni_J, Eq. omni_QS, Eq. omni_Jacobian); pixels alpha-composite their
 * depth-ordered Gaussians front to back (Sec. 3.1, Eq. gaussian2d, Eq. alphablending); the
 * backward pass differentiates all of it (Sec. 3.2 last paragraph, Appendix C).
 *
 * General rules for every entry point:
 *   - Pointers are DEVICE pointers unless marked [host].  All device buffers are owned by the
 *     caller; the library never allocates, frees or synchronises, and keeps no global mutable
 *     state.  Every call only enqueues work on `stream` (a hipStream_t; NULL = legacy stream)
 *     and is therefore capturable in a HIP graph.
 *   - float arrays are FP32, structure-of-arrays, with N = plan->n Gaussians:
 *       means [3][N] world-space centres;  scales [3][N] linear axis scales (> 0);
 *       quats [4][N] rotations (w, x, y, z), normalised inside;  opacities [N] in (0, 1);
 *       sh [K*3][N] real spherical-harmonic colour coefficients, plane index k*3 + channel,
 *       K = (sh_degree + 1)^2, basis order (l, m = -l..l);
 *       cams [V][12] per view: world-to-camera rotation R (row-major 3x3) then t (3), so
 *       x_cam = R x_world + t with OpenCV axes (z forward, x right, y down).
 *   - Images of all views are concatenated view after view: rgb [V][3][H_v][W_v] (planar),
 *     per-pixel planes [V][H_v][W_v].  Pixel (x, y) samples the point (x + 0.5, y + 0.5).
 *   - Return value: ODGS_OK or a negative error code (argument errors are detected on the host,
 *     before anything is enqueued).  Data-dependent conditions found on the device (pair-list
 *     overflow) are written to the status record inside the workspace, which the caller reads
 *     after its own synchronisation.
 *   - Calls for one plan must use one workspace, in the order preprocess -> bin_sort ->
 *     render_fwd -> render_bwd, on one stream (or with the caller ordering the streams).
 */
#ifndef ODGS_H
#define ODGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ODGS_OK = 0,
  ODGS_EINVAL = -1,    /* invalid argument (null or misaligned pointer, size out of range) */
  ODGS_ENOSPACE = -2,  /* workspace smaller than odgs_workspace_bytes(plan) */
  ODGS_EHIP = -3,      /* a kernel launch failed */
  ODGS_ETOOBIG = -4    /* input beyond the fixed scratch of a no-allocation entry point */
};

#define ODGS_MAX_VIEWS 64
#define ODGS_STATUS_OVERFLOW 1 /* more Gaussian-tile pairs than plan->pair_capacity */
#define ODGS_STATUS_STALE_FORWARD 2 /* odgs_composite_bwd found no odgs_render_fwd of the current pair
                                       list (none since the last odgs_bin_sort): it accumulated
                                       nothing, so the 2D gradients stay zero */
#define ODGS_FLAG_COUNT_WORK 1 /* settings flag: odgs_render_fwd also records the per-pixel work
                                  counters of odgs_debug_pixel_counts (slower; for measurement) */
#define ODGS_FLAG_SPHERICAL 2  /* settings flag: spherical footprint instead of the local affine
                                  approximation, see below (not with pinhole views, not with
                                  ODGS_FLAG_COUNT_WORK, no densification statistics) */
/* Scheduling of the two compositing launches, which cover the tiles of every view.  odgs_bin_sort
 * ends by queueing all (view, tile) pairs by descending list length (its compositing cost).
 * Default: one workgroup per task, workgroup b taking task b, so the longest tiles of all views
 * are dispatched first and the short ones fill the tail (the hardware dispatcher starts
 * workgroups in id order as slots free up).  A task is a tile, or at 16x16 tiles one 8x8 quadrant
 * of a tile whose list is long against the launch (at least 1/4096 of all pairs and, with 4096
 * tiles or more, at least 1024 pairs; at most max(1024, tiles / 8) tiles): those are split into four
 * tasks at the front of the queue, so that one list does not set the launch's length.  The two
 * flags below select the alternatives: */
#define ODGS_FLAG_SCHED_PERSISTENT 4 /* persistent launches: as many workgroups as fit on the device,
                                        each claiming the next task when it finishes one */
#define ODGS_FLAG_SCHED_TILE_ID 8    /* one workgroup per tile in global tile id order (no queue, no
                                        split tiles) */

/* Binning at 16x16 tiles when every view's width and height is a multiple of 32.  By default a
 * plan of 16384 tiles or more bins coarsely: its pairs are sorted by 32x32 tile, each carrying the
 * mask of the four 16x16 tiles its rectangle covers, and the sorted list is then split into the
 * 16x16 tiles' lists (about half as many keys to sort; the lists are the same either way).  Smaller
 * plans sort by 16x16 tile directly (fewer launches).  The flags select one of the two regardless
 * of size (coarse binning still needs tile 16 and the multiples of 32; setting both is an error): */
#define ODGS_FLAG_BIN_COARSE 16
#define ODGS_FLAG_BIN_DIRECT 32

/* Spherical footprint (ODGS_FLAG_SPHERICAL).  The paper names its local affine approximation
 * of the projected Gaussian as its limitation (Sec. 5).  With this flag every pixel ray t d
 * (t > 0, d the unit direction through the pixel centre, Eq. equirec_proj inverted) receives the
 * largest value the 3D Gaussian takes along the ray, exp(-m / 2) with
 *   m(d) = min_t (t d - mu^)^T Sigma~^-1 (t d - mu^),  mu^ = mu / |mu|,
 *   Sigma~ = W Sigma W^T / |mu|^2 + dilation (pi / H)^2 I,
 * so the footprint follows the curved image of the Gaussian exactly (the low-pass term becomes an
 * isotropic angular variance of `dilation` squared pixels at the vertical pixel pitch).  Sorting,
 * culling, compositing and the 3DGS constants are unchanged.  The tile rectangle bounds the cone
 * of rays through the ball of radius k sqrt(lambda_max(Sigma~)) around mu^ (k^2 = -2 p_min).
 * The kernels decide in float with the form described at SphRec in the sources (exponent
 * -qh / D, accepted iff h > 0 and p_min D + qh <= 0). */

/* Rasterization settings.  The paper fixes none of these constants; the defaults follow the
 * 3DGS rasterizer the method builds on (Sec. 3.2). */
typedef struct odgs_settings {
  int32_t tile;     /* tile edge in pixels: 8, 16 or 32; every W and H must be a multiple */
  int32_t batch;    /* Gaussians the forward compositor stages in LDS per round: 32, 64, 128 or 256
                       (64..256 at tile 32); 0 = default (256 for the spherical footprint at
                       tile 32, else 64) */
  int32_t batch_bwd; /* the same for the reverse compositor; 0 = default (32 at tile 8, 256 for the
                        spherical footprint at tile 32, else 64) */
  float near_r;     /* spherical-shell culling radii (Sec. 3.2): keep near_r < |mu| < far_r */
  float far_r;
  float dilation;   /* added to the 2D covariance's diagonal (3DGS low-pass), e.g. 0.3 */
  float pole_eps;   /* cull when sqrt(mu_x^2 + mu_z^2) <= pole_eps * |mu|, e.g. 1e-4 */
  float bg[3];      /* background colour behind the final transmittance */
  int32_t flags;    /* ODGS_FLAG_* bits, 0 for none */
} odgs_settings;

/* Device status record at byte offset plan->off_status of the workspace.  odgs_preprocess resets
 * every field except bin_gen. */
typedef struct odgs_status {
  int32_t flags;      /* ODGS_STATUS_* bits */
  int32_t n_pairs_stored; /* min(n_pairs, pair_capacity): pairs actually sorted and rendered */
  int64_t n_pairs;    /* Gaussian-tile pairs P of the last odgs_preprocess (with coarse binning, when
                         the 32x32 tiles' pairs already overflow: four times their number, an upper
                         bound of P to grow the capacity to) */
  int64_t n_visible;  /* (Gaussian, view) items that survived culling */
  uint32_t bin_gen;   /* incremented by every odgs_bin_sort (wraps) */
  uint32_t fwd_gen;   /* bin_gen of the pair list the last odgs_render_fwd composited; set to
                         ~bin_gen by odgs_preprocess and odgs_bin_sort.  The reverse compositor
                         reads the forward's per-entry culling masks and per-pixel state, so it
                         runs only when fwd_gen == bin_gen (else ODGS_STATUS_STALE_FORWARD) */
  int64_t n_culled;   /* (Gaussian, view) items culled: outside the shell, at a pole, degenerate
                         2D covariance, opacity below 1/255, no tile reached, or non-finite */
  int64_t n_nonfinite; /* Gaussians with a NaN or infinite parameter (mean, scale, quaternion,
                          opacity or SH coefficient) or a zero quaternion; all their items are
                          culled */
} odgs_status;

/* Plain-data description of one workload and of its workspace layout.  Filled by
 * odgs_plan_init; callers treat it as opaque, keep it in host memory and pass it by pointer. */
typedef struct odgs_plan {
  int64_t n;               /* Gaussians */
  int32_t sh_degree;       /* 0..3 */
  int32_t n_views;         /* 1..ODGS_MAX_VIEWS */
  odgs_settings s;
  int32_t width[ODGS_MAX_VIEWS];
  int32_t height[ODGS_MAX_VIEWS];
  int32_t tile_base[ODGS_MAX_VIEWS + 1];  /* first global tile id of each view; [n_views] = total */
  int64_t pix_base[ODGS_MAX_VIEWS + 1];   /* first pixel of each view; [n_views] = total */
  float pinhole[ODGS_MAX_VIEWS][4];       /* fx, fy, cx, cy of a perspective view; fx == 0: ERP view */
  int64_t items;           /* n * n_views (Gaussian, view) items, item id = view * n + gaussian */
  int64_t pair_capacity;   /* maximum Gaussian-tile pairs the workspace holds */
  int32_t tile_bits;       /* significant bits of a global tile id */
  int32_t item_blocks;     /* sort / scan blocks over items */
  int32_t pair_blocks;     /* sort blocks over pair_capacity */
  int32_t g2d_stride;      /* per-item gradient values of the reverse compositor: 9, or 13 (spherical) */
  /* workspace layout, byte offsets */
  size_t off_status, off_rec, off_rect, off_count, off_depth, off_dkey[2], off_did[2], off_srect, off_blocksum, off_pkey[2],
      off_pval[2],
      off_hist, off_digit, off_ranges, off_T, off_last, off_ncontrib, off_neval,
      off_lasteval, off_g2d, off_srec, off_cone, off_dirs, off_queue;
  int32_t depth_final;     /* which of the two depth-sort buffers holds the sorted result */
  int32_t pair_final;      /* which of the two pair buffers holds the sorted result (coarse binning:
                              the item buffer of that pair holds the refined lists) */
  int32_t coarse;          /* 1: pairs are binned and sorted by 32x32 tiles, then refined into the 16x16
                              tiles' lists (tile 16 with every W and H a multiple of 32) */
  int32_t coarse_bits;     /* significant bits of a global 32x32 tile id (coarse binning) */
  int32_t tile_base32[ODGS_MAX_VIEWS + 1];  /* first global 32x32 tile id of each view (coarse) */
  size_t ws_bytes;
} odgs_plan;

/* Fill `plan` for n Gaussians of SH degree sh_degree seen by n_views views of sizes
 * wh [host] = {W0, H0, W1, H1, ...}, with room for pair_capacity Gaussian-tile pairs
 * (pair_capacity < 2^31; fewer than 2^29 tiles over all views).  Pure host computation. */
int odgs_plan_init(odgs_plan* plan /*[host]*/, int64_t n, int32_t sh_degree, int32_t n_views, const int32_t* wh /*[host]*/,
                   const odgs_settings* s /*[host]*/, int64_t pair_capacity);

/* Densification statistics (Sec. 3.3), optionally accumulated by the reverse projection stage
 * for every (Gaussian, view) that is visible (kept by the culling tests and covering at least
 * one tile).  All three arrays have n entries and are ADDED to, so they can gather several
 * steps; the caller clears them (e.g. after odgs_densify).
 *   grad_sum += |(dL/du * W/2, dL/dv * H/2)|: the length of the gradient of the loss with
 *               respect to the Gaussian's 2D mean in normalised image units;
 *   tau_sum  += tau_min + (1 - cos theta) (tau_max - tau_min), theta the elevation of the mean
 *               seen from that view (the paper's elevation-dependent threshold; the paper uses
 *               tau_min = 2e-5, tau_max = 1e-4);
 *   count    += 1. */
typedef struct odgs_densify_acc {
  float* grad_sum;
  float* tau_sum;
  int32_t* count;
  float tau_min, tau_max;
} odgs_densify_acc;

/* Parameters of one clone / split / prune step (the 3DGS rules the method keeps, with the
 * threshold of Sec. 3.3 and percent_dense = 1e-3 of the paper's implementation details). */
typedef struct odgs_densify_params {
  float extent;          /* scene extent: the clone / split boundary is percent_dense * extent */
  float percent_dense;   /* e.g. 1e-3 */
  float min_opacity;     /* prune below this opacity, e.g. 0.005 */
  float max_scale_frac;  /* > 0: also prune a largest scale above max_scale_frac * extent; 0: off */
} odgs_densify_params;

/* Make view `view` of an initialised plan a perspective (pinhole) camera, the 3DGS model of
 * Sec. 3.1: pixel position pi(mu) = (fx mu_x / mu_z + cx, fy mu_y / mu_z + cy) (pixel (x, y)
 * samples (x + 0.5, y + 0.5) as in ERP views), Jacobian Eq. jacob_pers, sort depth mu_z, culling
 * to near_r < mu_z < far_r with the projected mean inside 1.3 times the field of view
 * (|mu_x / mu_z| <= 1.3 W / (2 fx), likewise y), tile columns clamped at the image edges (no
 * seam).  Such views share every other step with the ERP views of the same plan (e.g. the six
 * faces of a cubemap next to panoramas).  Pure host computation; fx, fy > 0. */
int odgs_plan_set_pinhole(odgs_plan* plan /*[host]*/, int32_t view, float fx, float fy, float cx, float cy);

/* Bytes of device workspace a plan needs (256-byte aligned base pointer required). */
size_t odgs_workspace_bytes(const odgs_plan* plan /*[host]*/);

/* Per (Gaussian, view): view transform, shell and pole culling, ERP position (Eq. equirec_proj),
 * 3D covariance R S S^T R^T (Sec. 3.1), tangent-plane Jacobian J_omni (Eq. omni_Jacobian),
 * 2D covariance J_omni W Sigma W^T J_omni^T plus dilation, its inverse, SH colour, radial
 * depth, and the footprint's tile rectangle.  Binning decisions are taken in FP64.
 * Resets the status record and clears the per-item 2D-gradient accumulators of odgs_composite_bwd. */
int odgs_preprocess(const odgs_plan* plan, const float* means, const float* scales, const float* quats,
                    const float* opacities, const float* sh, const float* cams, void* ws, size_t ws_bytes,
                    void* stream);

/* Bin and sort: depth-sort the items, count and emit Gaussian-tile pairs, radix-sort them by
 * global tile (stable, so each tile's list stays in (radial depth, Gaussian index) order, i.e.
 * the pairs end up ordered by the 64-bit key (tile << 32 | depth bits)), and build each tile's
 * [start, end) range.  P stays on the device; P > pair_capacity sets ODGS_STATUS_OVERFLOW and
 * leaves the pair list truncated (the images are then invalid). */
int odgs_bin_sort(const odgs_plan* plan, void* ws, size_t ws_bytes, void* stream);

/* Front-to-back compositing of every pixel of every view in one launch (Eq. gaussian2d and
 * Eq. alphablending, 3DGS constants alpha <= 0.99, alpha >= 1/255, stop below T = 1e-4).
 * out_rgb [V][3][H][W] receives C + T_final * bg; out_T [V][H][W] (may be NULL) the final
 * transmittance (accumulated alpha = 1 - T); out_depth [V][H][W] (may be NULL) the
 * alpha-weighted depth sum_j alpha_j T_j d_j with d_j the sort depth (radial distance in ERP
 * views, camera z in pinhole views; divide by 1 - T for the expected depth of the covered part).
 * Keeps per-pixel T, the list position after the last contributor, each staged list entry's
 * culling mask (all three read by the backward) and the work counters of
 * odgs_debug_pixel_counts in the workspace. */
int odgs_render_fwd(const odgs_plan* plan, void* ws, size_t ws_bytes, float* out_rgb, float* out_T, float* out_depth,
                    void* stream);

/* Gradient of L = sum(dL_drgb * out_rgb) with respect to every parameter, summed over the
 * views (reverse compositing, then the adjoint of the tangent-plane projection and of the SH
 * colour; Sec. 3.2 and Appendix C).  The parameters must be those given to odgs_preprocess.
 * The five gradient arrays (same shapes as the parameters) are OVERWRITTEN.
 * Equivalent to odgs_composite_bwd followed by odgs_project_bwd (acc as there). */
int odgs_render_bwd(const odgs_plan* plan, const float* means, const float* scales, const float* quats,
                    const float* opacities, const float* sh, const float* cams, void* ws, size_t ws_bytes,
                    const float* dL_drgb, float* d_means, float* d_scales, float* d_quats, float* d_opacities,
                    float* d_sh, const odgs_densify_acc* acc, void* stream);

/* First backward stage: reverse compositing of every pixel of every view (Eq. alphablending
 * differentiated), accumulating per-(Gaussian, view) gradients of the ERP position, the 2D
 * covariance Sigma_2D (dilation included), the opacity and the colour into the workspace (which
 * odgs_preprocess leaves cleared).  dL_drgb has the layout of out_rgb.
 * Requires odgs_render_fwd on this workspace after its last odgs_bin_sort (the compositing state
 * it reads is the forward's). */
int odgs_composite_bwd(const odgs_plan* plan, void* ws, size_t ws_bytes, const float* dL_drgb, void* stream);

/* Second backward stage: adjoint of the per-(Gaussian, view) projection (Eq. omni_Jacobian and
 * its derivative, Sigma = R S S^T R^T with the quaternion normalisation, SH colour), summed over
 * views into the five gradient arrays (OVERWRITTEN); the workspace's 2D gradients stay as they
 * are (odgs_debug_g2d can read them) until the next odgs_preprocess clears them.
 * acc [host] (may be NULL): densification statistics to accumulate, see odgs_densify_acc. */
int odgs_project_bwd(const odgs_plan* plan, const float* means, const float* scales, const float* quats,
                     const float* opacities, const float* sh, const float* cams, void* ws, size_t ws_bytes,
                     float* d_means, float* d_scales, float* d_quats, float* d_opacities, float* d_sh,
                     const odgs_densify_acc* acc, void* stream);

/* Device workspace bytes odgs_densify needs for n Gaussians (256-byte aligned base). */
size_t odgs_densify_workspace_bytes(int64_t n);

/* One densification step (Sec. 3.3): Gaussian i is selected when count[i] > 0 and
 * grad_sum[i] >= tau_sum[i] (its mean gradient reaches its mean threshold; FP32 compare).
 * Selected Gaussians whose largest scale is <= percent_dense * extent are cloned; the others are
 * split into two children at m + R(q) (s * xi_c) with scales s / 1.6 and all other parameters
 * copied, xi_c = noise[c][3][n] (c = 0, 1: standard normal draws supplied by the caller), and
 * the parent is removed.  Every resulting Gaussian with opacity < min_opacity (or, if
 * max_scale_frac > 0, largest scale > max_scale_frac * extent) is pruned.
 * Inputs are the parameter arrays (layouts as above, n Gaussians) and the statistics of
 * odgs_densify_acc.  Outputs have the same layouts with column stride `capacity` (>= 2 n, the
 * largest possible result): out_means [3][capacity], ..., out_sh [K*3][capacity]; out_src
 * [capacity] the parent index of each output; out_counts [4] (int64, device) the numbers of
 * surviving originals, clones, first children and second children, which appear in that order,
 * each group in parent order.  Entries past the total are left untouched. */
int odgs_densify(int64_t n, int32_t sh_degree, const float* means, const float* scales, const float* quats,
                 const float* opacities, const float* sh, const float* grad_sum, const float* tau_sum,
                 const int32_t* count, const float* noise, const odgs_densify_params* dp /*[host]*/,
                 int64_t capacity, float* out_means, float* out_scales, float* out_quats, float* out_opacities,
                 float* out_sh, int32_t* out_src, int64_t* out_counts, void* ws, size_t ws_bytes, void* stream);

/* ---- training step around the rasterizer (the 3DGS recipe the paper keeps) ---------------- */

/* Device pointers to the five parameter arrays (layouts as above). */
typedef struct odgs_param_ptrs {
  float* means;
  float* scales;
  float* quats;
  float* opacities;
  float* sh;
} odgs_param_ptrs;

typedef struct odgs_adam_hyper {
  float beta1, beta2, eps;  /* 3DGS: 0.9, 0.999, 1e-15 */
} odgs_adam_hyper;

/* Device workspace bytes odgs_l1_loss needs for `count` image values (256-byte aligned base). */
size_t odgs_l1_loss_workspace_bytes(int64_t count);

/* Image loss L = mean |rgb - target| over `count` values (any layout, both arrays alike):
 * writes dL/drgb = sign(rgb - target) / count (0 where equal) into dL (may feed
 * odgs_render_bwd) and L into loss[0] (device float), summed in double in a fixed order. */
int odgs_l1_loss(const float* rgb, const float* target, int64_t count, float* dL, float* loss, void* ws,
                 size_t ws_bytes, void* stream);

/* odgs_l1_loss without a workspace, for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the same kernels and
 * results (bit-identical), with the per-block partial sums in a fixed 512 KiB device array of the
 * library (one per GPU, held until the process ends; its address is looked up on the first call
 * on each device).  Calls nothing that allocates.  count <= ODGS_L1_NOALLOC_MAX_COUNT, else
 * ODGS_ETOOBIG before anything is enqueued.  Every call on one GPU shares that array: calls that
 * overlap on one GPU (different streams, or host threads) race and must be serialised by the
 * caller.  `stream` must belong to the current device. */
#define ODGS_L1_NOALLOC_MAX_COUNT (65536LL * 4096LL)
int odgs_l1_loss_noalloc(const float* rgb, const float* target, int64_t count, float* dL, float* loss, void* stream);

/* One Adam step (Kingma & Ba; PyTorch's placement of eps) over parameters kept before their
 * activations: raw scales are log-scales (scale = exp(raw)), raw opacities logits (opacity =
 * sigmoid(raw)); means, quaternions and SH coefficients are their own raw values.
 *   grad: gradients w.r.t. the ACTIVATED parameters (as odgs_render_bwd writes them); chained
 *         through the activations with the activated values in `act`;
 *   m, v: first and second moments (same layouts), updated;
 *   raw:  updated in place; act: overwritten with the new activated values (for identity groups
 *         act may alias raw);
 *   lr:   device float[6], learning rates of means, raw scales, quaternions, raw opacities, SH DC
 *         planes (k = 0) and the other SH planes;
 *   step: device int32 step counter t (read as t, the update uses t + 1, then incremented), so a
 *         captured HIP graph can be replayed step after step. */
int odgs_adam_step(int64_t n, int32_t sh_degree, const odgs_param_ptrs* raw /*[host]*/,
                   const odgs_param_ptrs* act /*[host]*/, const odgs_param_ptrs* grad /*[host]*/,
                   const odgs_param_ptrs* m /*[host]*/, const odgs_param_ptrs* v /*[host]*/, const float* lr,
                   int32_t* step, const odgs_adam_hyper* hp /*[host]*/, void* stream);

/* Byte offset of the odgs_status record inside the workspace. */
size_t odgs_status_offset(const odgs_plan* plan /*[host]*/);

/* Static description of an error code. */
const char* odgs_strerror(int code);

/* Size of odgs_plan, so bindings can allocate it without the struct definition. */
size_t odgs_plan_size(void);

/* ---- inspection (tests): copy internal results out of the workspace ---------------------- */

/* Per-item FP32 record [items][12]: u, v, l0, l1, l2, opacity, p_min, depth, r, g, b, tile count,
 * where the compositor's exponent -d^T Sigma_2D^-1 d / 2 is evaluated as
 * -((l0 du + l1 dv)^2 + (l2 dv)^2) (a Cholesky factor of Sigma_2D^-1 / 2); culled items have
 * tile count 0. */
int odgs_debug_records(const odgs_plan* plan, const void* ws, float* out, void* stream);

/* Per-pixel int32 [pixels][4] of the last odgs_render_fwd: list position after the last
 * contributor; number of contributors; list entries evaluated (up to and including the one that
 * ended the pixel by early termination, else the whole list); and entries evaluated up to the
 * last contributor.  The last three are only recorded by a forward whose plan has
 * ODGS_FLAG_COUNT_WORK set (otherwise they hold whatever an earlier counting forward left).  The last two count only entries whose padded footprint rectangle reaches
 * the pixel's 8x8 quadrant (the others are skipped for the whole wavefront). */
int odgs_debug_pixel_counts(const odgs_plan* plan, const void* ws, int32_t* out, void* stream);

/* Per-item 2D gradients accumulated by odgs_composite_bwd and not yet consumed by
 * odgs_project_bwd, double [items][9]: d/du, d/dv, d/dSigma_uu, d/dSigma_uv (the off-diagonal as
 * one shared variable), d/dSigma_vv (Sigma_2D with dilation), d/dopacity, d/dr, d/dg, d/db.
 * Spherical footprint: double [items][13]: d/dmu^ (3), d/dSigma~ (xx, xy, xz, yy, yz, zz; the
 * off-diagonals as one shared variable), d/dopacity, d/dr, d/dg, d/db.  Each tile's float sum
 * over its pixels is added in double, so the cross-tile total does not depend on the order in
 * which tiles finish (to double rounding, far below float resolution). */
int odgs_debug_g2d(const odgs_plan* plan, const void* ws, double* out, void* stream);

/* The sorted pair list as 64-bit keys (global tile << 32 | depth bits) and Gaussian indices,
 * first min(P, cap) entries (P from the status record, read by the caller). */
int odgs_debug_keys(const odgs_plan* plan, const void* ws, int64_t cap, uint64_t* keys, uint32_t* gauss,
                    void* stream);

#ifdef __cplusplus
}
#endif

#endif /* ODGS_H */
