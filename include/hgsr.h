/*
 * hgsr -- MI355X (gfx950) tile rasterizer of 3D Gaussian splats: RGB, depth,
 * alpha and feature maps of a Gaussian scene at one or many camera poses, and
 * the gradient of a loss on those maps with respect to the poses and the
 * Gaussian parameters.
 *
 * What it computes (Hi^2-GSLoc, arXiv 2507.15683):
 *   - the scene is a set of Gaussian primitives with centre, rotation, scale,
 *     opacity, colour and feature vector (Sec. 3.1);
 *   - colour and feature are alpha-blended front to back by the same tile
 *     rasterization (Sec. 3.1, the joint radiance/feature field);
 *   - the renderer is called as rasterization(means, opacity, q, c, s, K, T)
 *     (Algorithm 1) and, in the dense stage, renders dense feature and depth
 *     maps at a candidate pose (Sec. 3.4), repeated at every refinement step;
 *   - its backward gives the per-Gaussian gradients whose non-zero pattern is
 *     the render-visibility test of Algorithm 1.
 * The paper takes the rasterizer from 3D Gaussian Splatting and does not
 * restate it; this library fixes it as follows.  Per Gaussian: EWA
 * projection Sigma' = J R Sigma R^T J^T + 0.3 I with the pinhole Jacobian J
 * evaluated at x/z, y/z clamped to 1.3x the half field of view; colour =
 * max(0, sum_lm k_lm Y_lm(d) + 0.5) with d the unit vector from the camera
 * centre; culled when z <= near_z or opacity < 1/255; its pixel support is
 * the bounding box of the ellipse where o exp(-q/2) >= 1/255.  Per pixel,
 * Gaussians in ascending (camera z, index) order: alpha = min(0.99,
 * o exp(-q/2)) with q the conic distance; skipped when alpha < 1/255; the
 * walk stops (without blending) at the first Gaussian that would take the
 * transmittance T below 1e-4; rgb = sum w c + T bg, alpha = 1 - T,
 * depth = sum w z / (1 - T) (0 when nothing is blended), feat = sum w f,
 * with w = alpha T.
 *
 * Conventions
 *   - Every data pointer is a DEVICE pointer, owned by the caller, unless the
 *     comment says "host".  The library never frees caller memory.
 *   - Gaussians: structure of arrays, FP32, feature vectors as bfloat16 bits.
 *   - Poses: P x 12 floats, row-major [R | t], world -> camera, x_c = R x_w + t;
 *     camera axes x right, y down, z forward.  Pixel (i, j) has its centre
 *     at (i + 0.5, j + 0.5).
 *   - Images are planar per pose: rgb P x 3 x H x W, depth/alpha P x H x W,
 *     feat P x D x H x W (the D x H' x W' feature map of Sec. 3.1).
 *   - Pose gradients are in the left-perturbation tangent T <- Exp(xi) T,
 *     xi = (rho, phi), translation first.
 *   - Every call returns an hgsr_status and never throws; arguments are
 *     validated on the host before anything is enqueued.  HIP failures return
 *     HGSR_ERR_HIP; hgsr_last_error() gives a thread-local message.
 *   - All calls except hgsr_check_overflow, hgsr_stats, hgsr_debug_*,
 *     hgsr_autotune, hgsr_validate, the partition cache (hgsr_pcache_*, which
 *     plans on the host) and the host-only helpers are asynchronous on the
 *     given stream and can be captured into a HIP graph (after hgsr_reserve:
 *     a call that would grow the workspace while capturing fails).
 */
#ifndef HGSR_H_
#define HGSR_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* hgsr_stream;  /* a hipStream_t; NULL = default stream */

typedef enum {
  HGSR_OK = 0,
  HGSR_ERR_INVALID_ARG = 1, /* bad sizes, null required pointer, NaN input (validate) */
  HGSR_ERR_HIP = 2,         /* a HIP runtime call failed */
  HGSR_ERR_CAPACITY = 3,    /* workspace too small: the overflow flag was raised */
  HGSR_ERR_UNSUPPORTED = 4, /* a combination this build does not implement */
  HGSR_ERR_STATE = 5        /* call out of order (backward without render, ...) */
} hgsr_status;

typedef struct hgsr_ctx hgsr_ctx;

/* The Gaussian scene (Sec. 3.1: centre, rotation, scale, opacity, colour,
 * feature).  means n x 3; log_scales n x 3 (log of per-axis std. dev.);
 * quats n x 4 in (w, x, y, z) order, normalised by the renderer; opacities n,
 * already in [0, 1]; sh n x (sh_degree+1)^2 x 3 real spherical-harmonic
 * coefficients (degree 0..3), colour = max(0, SH + 0.5); feat n x feat_dim
 * bfloat16 bit patterns, feat_dim in {0, 8, 16, 32, 64}.
 * Optional spatial partitions (VastGaussian cells, Sec. 3.1): the Gaussians
 * of partition k are the contiguous range [part_offsets[k], part_offsets[k+1])
 * (device int64, n_parts + 1 entries) and part_bounds (device, n_parts x 6:
 * min xyz, max xyz) bound every point of those Gaussians' support; fill it
 * with hgsr_partition_bounds.  n_parts = 0: unpartitioned. */
typedef struct {
  int64_t n;
  const float* means;
  const float* log_scales;
  const float* quats;
  const float* opacities;
  const float* sh;
  int32_t sh_degree;
  int32_t feat_dim;
  const uint16_t* feat;
  int32_t n_parts;
  const int64_t* part_offsets;
  const float* part_bounds;
} hgsr_gaussians;

/* Pinhole intrinsics (the K of Algorithm 1), host struct. */
typedef struct {
  float fx, fy, cx, cy;
  int32_t width, height;
} hgsr_intrinsics;

enum { HGSR_SORT_BUCKET = 0, HGSR_SORT_LSD = 1 };
enum { HGSR_SCHED_GRID = 0, HGSR_SCHED_POSE_MAJOR = 1, HGSR_SCHED_TILE_MAJOR = 2, HGSR_SCHED_AUTO = -1 };

/* Render options (host struct).  tile: 8, 16 or 32 pixels, or 0 for the
 * autotuned choice (16 when none).  sort_mode: HGSR_SORT_BUCKET (counting
 * sort on the tile id, then a per-tile LDS sort on (depth, index)) or
 * HGSR_SORT_LSD (device LSD radix sort of (tile, depth, index) keys); both
 * give the same order.  schedule: blend launch shape (HGSR_SCHED_*).
 * bg: background colour added with the final transmittance.  near_z: camera
 * z below which a Gaussian is culled (0.2).  feat_out_bf16: write the feature
 * image as bfloat16 (FP32 accumulation).  lds_sort_cap: largest per-tile list
 * sorted in LDS (0 = default 4096; larger lists take a global-memory path).
 * feat_accum: how 32-channel features are summed at tile 8 and 16 --
 * HGSR_FEAT_AUTO (the autotuned choice, else the VALU), HGSR_FEAT_VALU
 * (per-pixel FMAs in blend order) or HGSR_FEAT_MFMA (per group of 8 splats,
 * a 32x8 by 8x64 matrix-core product of the bf16 features and the per-pixel
 * FP32 weights, each weight split exactly into three bf16 parts; the same
 * sum in another association order, colour, depth and alpha unchanged).  HGSR_FEAT_MFMA also moves the
 * backward's per-pair feature term (the pixel's feature gradient dotted with
 * the splat's feature) onto the matrix cores, per group of 32 splats; the
 * other settings keep it on the VALU. */
enum { HGSR_FEAT_AUTO = 0, HGSR_FEAT_VALU = 1, HGSR_FEAT_MFMA = 2 };

typedef struct {
  int32_t tile;
  int32_t sort_mode;
  int32_t schedule;
  float bg[3];
  float near_z;
  int32_t feat_out_bf16;
  int32_t lds_sort_cap;
  int32_t feat_accum;
} hgsr_opts;

/* Output images (device, caller-allocated).  rgb, depth and alpha are
 * required; feat may be NULL (not written).  feat is float or bfloat16 bits
 * per hgsr_opts.feat_out_bf16. */
typedef struct {
  float* rgb;
  float* depth;
  float* alpha;
  void* feat;
} hgsr_outputs;

/* Loss gradients with respect to the outputs (device, FP32, same layouts);
 * any may be NULL meaning zero. */
typedef struct {
  const float* rgb;
  const float* depth;
  const float* alpha;
  const float* feat;
} hgsr_grad_outputs;

/* Gradients written by hgsr_render_backward (device, FP32, overwritten; NULL
 * = not computed).  pose: P x 6 (rho, phi); means n x 3; opacities n;
 * log_scales n x 3; quats n x 4 (with respect to the stored, unnormalised
 * quaternion); sh n x K x 3; feat n x feat_dim.  Gaussian gradients are summed
 * over poses. */
typedef struct {
  float* pose;
  float* means;
  float* opacities;
  float* log_scales;
  float* quats;
  float* sh;
  float* feat;
  /* Which render these gradients are for: 0 = the context's last render;
   * otherwise an id hgsr_render_id returned, and the call fails with
   * HGSR_ERR_STATE (nothing enqueued) unless that render is still the
   * context's last one (a later render or scoring pass replaced the saved
   * lists, transmittances and pose pointers the backward replays). */
  int64_t render_id;
} hgsr_grads;

/* Per-render counters (host struct, from hgsr_stats). */
typedef struct {
  int64_t visible;       /* (pose, Gaussian) pairs with a non-empty support */
  int64_t keys;          /* (pose, tile, Gaussian) entries */
  int64_t max_tile_list; /* longest per-tile list */
  int32_t overflow;      /* bit 0 records, bit 1 keys */
  int32_t tile;          /* tile size used */
} hgsr_render_stats;

/* Result of hgsr_autotune (host struct). */
typedef struct {
  int32_t tile;
  int32_t schedule;
  int32_t feat_accum;
  float ms;              /* best time per render */
  int32_t proj_group;    /* Gaussians culled per thread by the projection of up to 4 poses: 1 or 4 */
} hgsr_tune_result;

/* Create a context on the current HIP device.  The context owns the
 * workspace (projected splats, keys, per-tile lists, the per-pixel final
 * transmittance and list length saved for the backward).  Capacity hints may
 * be 0. */
hgsr_status hgsr_ctx_create(hgsr_ctx** ctx, int64_t record_hint, int64_t key_hint);
hgsr_status hgsr_ctx_destroy(hgsr_ctx* ctx);

/* Pre-size the workspace for P poses of W x H at tile size `tile` with
 * room for `records_per_pose` visible Gaussians per pose and `keys` tile
 * entries in total.  Required before graph capture (no allocation is
 * allowed while capturing). */
hgsr_status hgsr_reserve(hgsr_ctx* ctx, int32_t P, int32_t width, int32_t height, int32_t tile,
                         int64_t records_per_pose, int64_t keys, int64_t n_gaussians);

/* Render P poses (device pointer, P x 12) of the scene:
 * out = {rgb, depth, alpha, feat} per pose.  Enqueues the projection, tile
 * binning, sort and blend kernels on `stream`; no host synchronisation.  The
 * context keeps what the backward needs until the next hgsr_render.  When
 * the workspace is too small the overflow flag is raised on the device, the
 * outputs are undefined, and hgsr_check_overflow reports it. */
hgsr_status hgsr_render(hgsr_ctx* ctx, const hgsr_gaussians* g, const float* poses, int32_t P,
                        const hgsr_intrinsics* K, const hgsr_opts* opts, const hgsr_outputs* out,
                        hgsr_stream stream);

/* hgsr_render for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, kernels and results as hgsr_render (bit for bit: the
 * tile lists' order does not depend on the capacities), but no context: the workspace (projected splats, keys,
 * per-tile lists, per-pixel transmittance and list length) is laid out in a
 * static device array of 128 MiB that each GPU the library runs on holds
 * from the library's load until the process ends.  The call allocates
 * nothing, host or device, and does not synchronise.
 *   records_per_pose, keys: capacities (visible Gaussians per pose, tile
 *     entries in total), both > 0, or both 0 to split the space the
 *     per-pixel (8 B) and per-tile (20 B) buffers leave evenly between
 *     records (60 B each) and keys (28 B each).
 *   flags_out: device int32 (may be NULL) that receives the overflow bits
 *     after the render (bit 0 records, bit 1 keys; 0 = complete).  When
 *     non-zero the outputs are undefined: render again with larger
 *     capacities, or with hgsr_render.
 * HGSR_ERR_CAPACITY (nothing enqueued) when the layout would exceed 128 MiB
 * (for example 16 poses at 1920x1080: 8 B per pixel alone is 265 MB).
 * Every call on one GPU shares that GPU's array and leaves its contents
 * behind (each render clears what must start at zero): calls that overlap on
 * one GPU -- on different streams, or a graph replayed while another call
 * runs -- race, and the array holds nothing a backward can use.  The HIP
 * device current at the call must be the one `stream` belongs to. */
hgsr_status hgsr_render_noalloc(const hgsr_gaussians* g, const float* poses, int32_t P, const hgsr_intrinsics* K,
                                const hgsr_opts* opts, const hgsr_outputs* out, int64_t records_per_pose,
                                int64_t keys, int32_t* flags_out, hgsr_stream stream);

/* Backward of the last hgsr_render on this context: the gradient of a loss
 * on the rendered maps with respect to the poses and the Gaussian parameters
 * (Algorithm 1 back-propagates the summed rendered RGB and keeps the
 * Gaussians whose mean gradient is non-zero; the dense stage's refinement,
 * Sec. 3.4, descends the residual of the rendered package against the
 * query).  grad_out holds dL/d{rgb, depth, alpha, feat} (device, FP32, the
 * layouts of hgsr_outputs; NULL = zero).  Replays each pixel's blend in
 * reverse from the saved final transmittance and list length (no per-pixel
 * lists are stored) and writes the requested gradients (see hgsr_grads,
 * including its render_id check).  The forward's inputs and its depth/alpha
 * outputs must still hold the values of that render.  HGSR_ERR_STATE before
 * any render or after a scoring pass. */
hgsr_status hgsr_render_backward(hgsr_ctx* ctx, const hgsr_grad_outputs* grad_out, const hgsr_grads* grads,
                                 hgsr_stream stream);

/* Id of the context's last render (host, no synchronisation): 1, 2, ... in
 * the order of the context's renders, 0 when the last call that built tile
 * lists was not a render (or there was none).  Pass it in hgsr_grads.render_id
 * to have a backward refuse gradients for a render that is no longer the
 * last one. */
hgsr_status hgsr_render_id(hgsr_ctx* ctx, int64_t* id);

/* Left retraction of P poses: out = Exp(xi) T per pose, xi (device, P x 6,
 * (rho, phi), translation first) in the tangent every pose gradient of this
 * library uses; poses and out P x 12 (may alias).  Evaluated in FP64, stored
 * in FP32.  Asynchronous on `stream`. */
hgsr_status hgsr_pose_retract(const float* poses, const float* xi, int32_t P, float* out, hgsr_stream stream);

/* Chain rule through the retraction: given g = dL/d(delta) at delta = 0 for
 * Exp(delta) Exp(xi) T (what hgsr_render_backward returns for a render at
 * the retracted pose), writes dL/dxi = J_l(xi)^T g with J_l the left Jacobian
 * of SE(3), Exp(xi + dxi) = Exp(J_l(xi) dxi) Exp(xi) to first order.  J_l is
 * the series sum_n ad(xi)^n / (n + 1)!, summed to 40 terms in FP64 (its
 * truncation is below double rounding for |phi| <= 2 pi; rho enters
 * linearly).  xi, g, g_xi: device, P x 6 (g_xi may alias g).  J_l(0) is the
 * identity, so at xi = 0 g_xi equals g bit for bit. */
hgsr_status hgsr_pose_tangent_grad(const float* xi, const float* g, int32_t P, float* g_xi, hgsr_stream stream);

/* Refinement residual of P rendered poses against targets (Sec. 3.4 compares
 * the rendered package with the query): per pose
 *   L = 1/(H W) sum_p [ sum_c |rgb - rgb*| + lam_f (1 - cos(F, F*)) ],
 * cos(a, b) = a.b / (|a| |b| + 1e-8).  Writes loss (P floats), dL/drgb
 * (P x 3 x H x W) and, when D > 0, dL/dfeat (P x D x H x W).  feat is float
 * or bfloat16 bits per feat_bf16; targets are float. */
hgsr_status hgsr_residual(const float* rgb, const void* feat, int32_t feat_bf16, const float* rgb_target,
                          const float* feat_target, int32_t P, int32_t H, int32_t W, int32_t D, float lam_f,
                          float* loss, float* grad_rgb, float* grad_feat, hgsr_stream stream);

/* Targets of the refinement residual (the one hgsr_residual defines), as
 * device pointers: rgb_target 3 x H x W and feat_target D x H x W per target
 * image (feat_target NULL when D == 0).  shared_target = 0: one target
 * image per pose; nonzero: every pose is compared with the same single
 * target (the candidate poses of one query).  lam_f weighs the feature
 * term. */
typedef struct {
  const float* rgb_target;
  const float* feat_target;
  float lam_f;
  int32_t shared_target;
} hgsr_residual_targets;

/* Gradient of the refinement residual of the last hgsr_render on this
 * context (Sec. 3.4: the dense stage refines the pose by comparing renders
 * with the query), without materialising dL/d(outputs): the blend backward
 * forms each pixel's residual gradient from the render's rgb and feature
 * outputs (which must still hold that render's values) and the targets, then
 * replays the blend as hgsr_render_backward does.  Writes loss (device, P
 * floats, overwritten; summed per tile, then per pose, in a fixed order) and
 * the requested gradients; equal to hgsr_residual followed by
 * hgsr_render_backward up to the order in which the loss is summed. */
hgsr_status hgsr_residual_backward(hgsr_ctx* ctx, const hgsr_residual_targets* targets, float* loss,
                                   const hgsr_grads* grads, hgsr_stream stream);

/* One Adam step on the pose tangents and the left update T <- Exp(-step) T.
 * poses P x 12 (updated in place), grad P x 6, m and v P x 6 (state),
 * step_count: device int32 incremented by the call (so graph replays
 * advance it); lr_rho in metres, lr_phi in radians. */
hgsr_status hgsr_pose_adam(float* poses, const float* grad, float* m, float* v, int32_t* step_count, int32_t P,
                           float lr_rho, float lr_phi, float beta1, float beta2, float eps, hgsr_stream stream);

/* 2D feature maps of the views scored by hgsr_significance (device, FP32):
 * one D x height x width map per view, D = the scene's feature_dim.  The
 * map covers the image: the projected mean (U, V) reads the cell
 * (floor(U width / W), floor(V height / H)) that contains it (nearest, no
 * interpolation).  layout HGSR_MAP_PLANAR: view-major, then channel, row,
 * column (P x D x height x width, the layout of the rendered feature maps);
 * HGSR_MAP_INTERLEAVED: P x height x width x D (one contiguous vector per
 * cell). */
enum { HGSR_MAP_PLANAR = 0, HGSR_MAP_INTERLEAVED = 1 };
typedef struct {
  const float* maps;
  int32_t width;
  int32_t height;
  int32_t layout;
} hgsr_feature_maps;

/* Significance scoring (Sec. 3.2, Eq. 4-6) of every Gaussian against P
 * training views with poses `poses` (device, P x 12) and 2D feature maps
 * `maps`.  For each view the call renders the visibility of the render-mask
 * algorithm of Sec. 3.2: a Gaussian j is visible when it is blended (weight
 * alpha T > 0, the condition under which its mean receives a gradient from
 * the rendered RGB) at one pixel at least, and its projected mean (U, V) =
 * K (X/Z) lies in [0, W) x [0, H).  For each visible j it adds
 *   cos_j = F_j . F^t(U, V) / (|F_j| |F^t(U, V)| + 1e-8)      (Eq. 4)
 * to score_sum[j] (Eq. 5) and 1 to vis_count[j] (device, n floats and n
 * uint32, accumulated: the caller zeroes them once and calls once per batch
 * of views).  Views are added in order, so results do not depend on
 * scheduling.  visible (device, P x n bytes, or NULL) receives the mask per
 * view (1 = visible).  The Gaussians' features must be present
 * (feature_dim > 0).  Uses the context's workspace: a following
 * hgsr_render_backward is refused until the next hgsr_render.  Overflow is
 * reported as for hgsr_render (the sums are then undefined). */
hgsr_status hgsr_significance(hgsr_ctx* ctx, const hgsr_gaussians* g, const float* poses, int32_t P,
                              const hgsr_intrinsics* K, const hgsr_opts* opts, const hgsr_feature_maps* maps,
                              float* score_sum, uint32_t* vis_count, uint8_t* visible, hgsr_stream stream);

/* Final significance score S(g_j) = score_sum[j] / vis_count[j] (Eq. 6), 0
 * where vis_count[j] == 0 (device, n floats). */
hgsr_status hgsr_significance_final(const float* score_sum, const uint32_t* vis_count, int64_t n, float* score,
                                    hgsr_stream stream);

/* Query and rendered feature maps for hgsr_match (device, bfloat16 bits,
 * planar D x H x W).  The coarse maps are coarse_width x coarse_height
 * positions; the fine maps, when given, 8 times that in each direction
 * (the window w = H_f / H_c = 8 of Sec. 3.4).  D: 8, 16, 32 or 64. */
typedef struct {
  const uint16_t* query_coarse;
  const uint16_t* render_coarse;
  const uint16_t* query_fine;   /* NULL: coarse level only */
  const uint16_t* render_fine;
  int32_t D;
  int32_t coarse_width;
  int32_t coarse_height;
} hgsr_match_maps;

/* Outputs of hgsr_match (device, caller-allocated).  n_coarse: one uint32,
 * the number of coarse correspondences K.  coarse_query / coarse_render /
 * coarse_p: capacity coarse_width x coarse_height entries; entry k < K is
 * the k-th correspondence in query order: the query's and the render's
 * coarse position (row-major index) and its probability P.  fine_query /
 * fine_render / fine_p (needed when fine maps are given): capacity
 * coarse_width x coarse_height x 64; slot 64 k + t describes query window
 * position t (row-major in the 8 x 8 window) of coarse correspondence k: its
 * fine position and the matched rendered fine position (row-major indices
 * in the fine maps) and P, or -1, -1, 0 when position t has no mutual
 * match.  Slots of k >= K are left unchanged. */
typedef struct {
  uint32_t* n_coarse;
  int32_t* coarse_query;
  int32_t* coarse_render;
  float* coarse_p;
  int32_t* fine_query;
  int32_t* fine_render;
  float* fine_p;
} hgsr_match_out;

/* Coarse-to-fine probabilistic mutual matching of a query's feature maps
 * with rendered ones (Sec. 3.4, Eq. 11).  Coarse level: M_ij = cosine of
 * query position i and rendered position j (a.b / (|a| |b| + 1e-8)),
 * P = softmax over j of M/tau times softmax over i of M/tau (element by
 * element), and (i, j) is a correspondence when j maximises row i of P and
 * i maximises column j (ties: lowest index).  Fine level: the same on the
 * 8 x 8 fine windows of coarse cell i in the query and cell j in the render,
 * for every coarse correspondence.  tau_coarse and tau_fine must be at least
 * 1/40.  The M matrix is never stored; the workspace grows with the number
 * of coarse positions.  Asynchronous on `stream`. */
hgsr_status hgsr_match(hgsr_ctx* ctx, const hgsr_match_maps* maps, float tau_coarse, float tau_fine,
                       const hgsr_match_out* out, hgsr_stream stream);

/* A 2D-3D pose problem for hgsr_pnp (device arrays): query pixel coordinates
 * p2d (n x 2, pixel centres at +0.5) and world points x3d (n x 3), e.g. the
 * fine correspondences with hgsr_backproject's points; samples (n_hyp x 3)
 * are the RANSAC draws, indices into the n correspondences (given by the
 * caller, so that runs are reproducible); tau the inlier threshold in
 * pixels; gn_iters Gauss-Newton steps per hypothesis, refine_iters steps of
 * the final refinement. */
typedef struct {
  const float* p2d;
  const float* x3d;
  int64_t n;
  const int32_t* samples;
  int32_t n_hyp;
  float tau;
  int32_t gn_iters;
  int32_t refine_iters;
} hgsr_pnp_problem;

/* Results of hgsr_pnp (device, caller-allocated): pose (12 floats, the
 * refined world -> camera [R|t]); best (1 int32, the winning hypothesis, -1
 * when no sample was valid); counts (n_hyp int32: inliers per hypothesis, -1
 * for a degenerate sample); hyp_poses (n_hyp x 12, or NULL); inliers (n
 * bytes, or NULL: 1 for the final pose's inliers); n_inliers (1 int32). */
typedef struct {
  float* pose;
  int32_t* best;
  int32_t* counts;
  float* hyp_poses;
  uint8_t* inliers;
  int32_t* n_inliers;
} hgsr_pnp_result;

/* Pose from 2D-3D correspondences (Sec. 3.4, Eq. 10): argmin over [R|t] of
 * sum_i rho(|p_i - pi(K [R|t] X_i)|, tau), rho the truncated quadratic
 * min(e^2, tau^2), by RANSAC.  Each sample of 3 correspondences is solved by
 * gn_iters Gauss-Newton steps from the prior pose pose0 (device, 12 floats:
 * the render pose) with the left update T <- Exp(delta) T; a sample with a
 * singular normal matrix is invalid; every hypothesis is scored by its
 * number of correspondences with positive depth and reprojection error
 * below tau (ties: lowest index); the best is refined by refine_iters
 * Gauss-Newton steps on its inlier set, re-taken before every step.
 * Everything runs on the device (capturable). */
hgsr_status hgsr_pnp(hgsr_ctx* ctx, const hgsr_pnp_problem* problem, const hgsr_intrinsics* K, const float* pose0,
                     const hgsr_pnp_result* result, hgsr_stream stream);

/* World points of rendered pixels (Sec. 3.4 lifts the rendered matches with
 * the rendered depth): x3d[i] = R^T (d K^-1 [u, v, 1]^T - t) for pixel pix[i]
 * (row-major index into the width x height depth map, centre (u, v) =
 * (x + 0.5, y + 0.5)), its depth d and the render pose [R|t] (device, 12
 * floats).  Out-of-range pixels give (0, 0, 0). */
hgsr_status hgsr_backproject(const float* depth, int32_t width, int32_t height, const float* pose,
                             const hgsr_intrinsics* K, const int32_t* pix, int64_t n, float* x3d,
                             hgsr_stream stream);

/* Pose consistency verification (Algorithm 2): for the n dense results
 * poses (device, n x 12), the rotation angle of R_i R_{i+1}^T (trace clamped
 * to [-1, 3]) for every consecutive pair; reliable (device int32) is 1 when
 * none exceeds tau_deg; max_angle (device float, or NULL) the largest. */
hgsr_status hgsr_pose_consistency(const float* poses, int32_t n, float tau_deg, int32_t* reliable,
                                  float* max_angle, hgsr_stream stream);

/* Fill part_bounds (device, n_parts x 6) with a box containing, for every
 * Gaussian of each partition, the ball of radius 3.33 x its largest scale
 * around its mean (the 1/255 support of the most opaque Gaussian). */
hgsr_status hgsr_partition_bounds(const hgsr_gaussians* g, float* part_bounds, hgsr_stream stream);

/* ---------------------------------------------------------------- partition streaming
 * Scenes larger than device memory (Sec. 3.1: the scene is trained and kept
 * as spatial cells; Sec. 3.2: batches are processed under a memory budget
 * and their intermediate data released).  A partition cache keeps the whole
 * partitioned scene in library-owned pinned host memory and a fixed device
 * budget of n_slots slots, each holding one partition; per batch of poses it
 * makes resident the partitions that may be seen, evicting the least
 * recently used slots the batch does not need, and hands back a scene
 * descriptor for hgsr_render / hgsr_render_backward / hgsr_significance.
 *
 * The descriptor's Gaussians are the slots laid end to end
 * (n = n_slots x slot_capacity; slot s is partition s of the descriptor,
 * [s x capacity, (s + 1) x capacity)); a slot's unused tail has opacity 0
 * and an empty slot an empty box, so neither is ever projected.  Renders
 * through the descriptor equal renders of the whole resident scene up to
 * the order of Gaussians at exactly equal depth (the index that breaks such
 * ties is the slot index, not the scene index).  Gaussian indices in
 * per-Gaussian outputs (gradients, visibility) are descriptor indices. */

/* Host-side scene of a partition cache: every array in host memory, the
 * layouts of hgsr_gaussians; part_offsets host int64, n_parts + 1 entries,
 * partition k = [part_offsets[k], part_offsets[k+1]). */
typedef struct {
  int64_t n;
  const float* means;
  const float* log_scales;
  const float* quats;
  const float* opacities;
  const float* sh;
  int32_t sh_degree;
  int32_t feat_dim;
  const uint16_t* feat;
  int32_t n_parts;
  const int64_t* part_offsets;
} hgsr_host_scene;

typedef struct hgsr_pcache hgsr_pcache;

#define HGSR_MAX_SLOTS 64

/* One partition upload of a batch: partition `part` into device slot `slot`.
 * `release` is the batch whose start the copy waits for before it overwrites
 * the slot: the first batch after the slot's previous use (work enqueued on
 * the render stream before that batch's prepare may still read the slot's
 * old partition), or the oldest of the last 16 batches when that use is
 * older still (a conservative, later release); -1 when the slot was never
 * used (no wait).  `ahead` is 1 for an upload made for upcoming views only. */
typedef struct {
  int32_t part;
  int32_t slot;
  int64_t release;
  int32_t ahead;
  int32_t reserved;
} hgsr_slot_upload;

typedef struct {
  int32_t needed;          /* partitions the last batch's rendered views may see */
  int32_t hits;            /* of those, already resident */
  int32_t uploads;         /* copied from host memory for the last batch */
  int32_t evictions;       /* resident partitions dropped for the last batch */
  int64_t bytes_uploaded;  /* by the last batch */
  int64_t total_uploads;   /* since creation */
  int64_t total_bytes;     /* since creation */
  int32_t n_slots;
  int64_t slot_capacity;   /* Gaussians per slot (the largest partition) */
  int64_t device_bytes;    /* the device budget in use (slots + tables) */
  int32_t prefetched;      /* of the last batch's uploads, those for upcoming views only */
  hgsr_slot_upload upload[HGSR_MAX_SLOTS]; /* the last batch's uploads, in enqueue order (`uploads` entries) */
} hgsr_pcache_stats;

/* Create a cache on the current device: copies the host scene into pinned
 * host memory (hipHostMalloc; the caller's arrays may be freed afterwards),
 * computes the partition boxes (hgsr_host_partition_bounds) and allocates
 * n_slots slots (1..64, at most n_parts).  Synchronous.  Errors:
 * HGSR_ERR_INVALID_ARG for bad sizes or NULL arrays, HGSR_ERR_HIP when an
 * allocation fails. */
hgsr_status hgsr_pcache_create(hgsr_pcache** out, const hgsr_host_scene* scene, int32_t n_slots);
hgsr_status hgsr_pcache_destroy(hgsr_pcache* pc);

/* Make the partitions that the first n_render of the P poses (host, P x 12)
 * may see at intrinsics K resident, and fill *out with the device
 * descriptor through which those views are rendered.  Poses n_render..P-1
 * are upcoming views: the partitions only they may see are uploaded ahead,
 * into free or least recently used slots the rendered views cannot see (best
 * effort, skipped when no such slot is left), behind this batch's slot table,
 * so that the uploads overlap this batch's renders; they become visible to
 * renders from the next prepare on.  A partition may be seen when its box,
 * grown by motion_margin metres (room for poses that move during refinement
 * without a new call), passes the conservative frustum test of
 * hgsr_partition_plan.  Uploads run on the cache's own copy stream from
 * pinned memory; `stream` -- the stream the renders using *out run on, the
 * same on every call -- waits for the rendered views' uploads, and a slot is
 * only overwritten after the work enqueued on `stream` before the call that
 * last needed it (no host synchronisation).  The descriptor stays valid
 * until the next prepare on this cache.  Returns HGSR_ERR_CAPACITY (nothing
 * enqueued) when the rendered views may see more partitions than the cache
 * has slots.  stats may be NULL. */
hgsr_status hgsr_pcache_prepare(hgsr_pcache* pc, const float* poses, int32_t P, int32_t n_render,
                                const hgsr_intrinsics* K, float near_z, float motion_margin, hgsr_gaussians* out,
                                hgsr_pcache_stats* stats, hgsr_stream stream);

/* Drop every resident partition (the slots stay allocated); the next
 * prepare uploads what it needs.  Synchronises the copy stream. */
hgsr_status hgsr_pcache_evict_all(hgsr_pcache* pc);

/* Host-only helpers (no device work; usable without a GPU).
 * hgsr_host_partition_bounds: per partition (host out, n_parts x 6, min xyz
 * then max xyz) the box containing every Gaussian's ball of radius 3.33 x its
 * largest scale around its mean (the same box as hgsr_partition_bounds,
 * rounded outward); an empty partition gets min > max.
 * hgsr_partition_plan: per (pose, partition) (host out, P x n_parts bytes)
 * 1 when the box grown by motion_margin may reach the image: rejected only
 * when all 8 corners lie behind the near plane or outside one of the four
 * side planes through the camera centre, pushed out by 9 + 0.05 max(W, H)
 * pixels (a pixel more than the renderer's own partition test, so that every
 * partition the renderer would draw is planned).  Empty boxes are never
 * seen. */
hgsr_status hgsr_host_partition_bounds(const hgsr_host_scene* scene, float* bounds);

/* The partition cache's slot policy on its own (host only; the policy
 * hgsr_pcache_prepare applies, exposed so that it can be checked without a
 * GPU).  A step takes, per partition (host, n_parts bytes), 1 when the
 * batch's rendered views may see it, 2 when only its upcoming views may, 0
 * otherwise.  Missing partitions of the rendered views take an empty slot
 * (least recently used first), else the least recently used slot the batch
 * does not need (ties to the lower slot); then the upcoming views' missing
 * partitions take the slots left over, while any remain.  It fills needed,
 * hits, uploads, evictions, prefetched and upload[] of *st (the byte
 * counters are left alone).  HGSR_ERR_CAPACITY, with the state unchanged,
 * when the rendered views need more partitions than there are slots. */
typedef struct hgsr_slot_policy hgsr_slot_policy;
hgsr_status hgsr_slot_policy_create(hgsr_slot_policy** out, int32_t n_parts, int32_t n_slots);
hgsr_status hgsr_slot_policy_destroy(hgsr_slot_policy* policy);
hgsr_status hgsr_slot_policy_step(hgsr_slot_policy* policy, const uint8_t* need, hgsr_pcache_stats* st);
hgsr_status hgsr_slot_policy_evict_all(hgsr_slot_policy* policy);
hgsr_status hgsr_partition_plan(const float* bounds, int32_t n_parts, const float* poses, int32_t P,
                                const hgsr_intrinsics* K, float near_z, float motion_margin, uint8_t* seen);

/* Spatial order of a scene (host only, no device work): perm (host, n int64)
 * lists the Gaussians sorted by the Morton code of their means (21 bits per
 * axis over the bounding box, one scale for all axes; ties by index), within
 * each partition when part_offsets (host, n_parts + 1) is given, so that
 * partitions stay contiguous.  A scene stored in this order renders the same
 * images (up to the order of Gaussians at exactly equal depth) with denser
 * projection waves, tile counts aggregated per workgroup and tile lists
 * whose records lie close together; Gaussian i of the reordered scene is
 * Gaussian perm[i] of the input.  Non-finite coordinates sort as the box
 * minimum. */
hgsr_status hgsr_host_spatial_order(const float* means, int64_t n, const int64_t* part_offsets, int32_t n_parts,
                                    int64_t* perm);

/* Check the Gaussian arrays for NaN/Inf (means, log-scales, quaternions, SH
 * coefficients and bfloat16 features), opacities outside [0, 1] and zero
 * quaternions.  Allocates a 4-byte device flag and synchronises `stream`, so
 * it cannot be captured: HGSR_ERR_STATE when `stream` is capturing.  Returns
 * HGSR_ERR_INVALID_ARG when any entry fails. */
hgsr_status hgsr_validate(const hgsr_gaussians* g, hgsr_stream stream);

/* Graph capture of everything enqueued on `stream` between begin and end;
 * launch replays it `replays` times on `stream`. */
hgsr_status hgsr_graph_begin(hgsr_ctx* ctx, hgsr_stream stream);
hgsr_status hgsr_graph_end(hgsr_ctx* ctx);
hgsr_status hgsr_graph_launch(hgsr_ctx* ctx, int32_t replays, hgsr_stream stream);

/* Synchronise `stream` and report whether the last render overflowed its
 * workspace (*overflowed = bit mask, 0 = fine).  When it did, the workspace
 * is grown to the sizes the device measured so that a re-render fits. */
hgsr_status hgsr_check_overflow(hgsr_ctx* ctx, int32_t* overflowed, hgsr_stream stream);

/* Counters of the last render (synchronises `stream`). */
hgsr_status hgsr_stats(hgsr_ctx* ctx, hgsr_render_stats* out, hgsr_stream stream);

/* Copy pose `pose`'s per-tile lists of the last render to host memory:
 * ranges (host, tiles x 2: begin, end offsets into gids) and gids (host,
 * capacity cap) holding Gaussian indices in blend order.  *n receives the
 * number of entries.  Synchronises `stream`. */
hgsr_status hgsr_debug_tile_lists(hgsr_ctx* ctx, int32_t pose, uint32_t* ranges, uint32_t* gids, int64_t cap,
                                  int64_t* n, hgsr_stream stream);

/* Time the renderer on this input for tile sizes 8/16/32, the blend
 * schedules and (32 channels) both feature accumulations, then (up to 4 poses) the
 * projection's grouping (1 Gaussian per thread, the default, suited to scenes
 * in spatial order -- hgsr_host_spatial_order --, or 4, often faster for
 * scenes in arbitrary order); keep the fastest as
 * the context's default (opts->tile == 0, opts->schedule == HGSR_SCHED_AUTO,
 * opts->feat_accum == HGSR_FEAT_AUTO) and append it to the JSON-lines cache
 * file `cache_path` (host string, may be NULL), which later calls on the same
 * shape read instead of timing.  with_backward != 0 times each render
 * followed by the pose backward (dL/drgb and, for FP32 feature maps,
 * dL/dfeat taken as the rendered maps themselves), the cost of a refinement
 * step, instead of the render alone.  Synchronises `stream`. */
hgsr_status hgsr_autotune(hgsr_ctx* ctx, const hgsr_gaussians* g, const float* poses, int32_t P,
                          const hgsr_intrinsics* K, const hgsr_opts* opts, const hgsr_outputs* out,
                          int32_t with_backward, const char* cache_path, hgsr_tune_result* result,
                          hgsr_stream stream);

/* Measured VALU issue rate, for rooflines of instruction-bound kernels: the
 * device's rate of wave64 FP32 fused multiply-add instructions (independent
 * chains, no packed forms) over all its compute units, from one timed
 * launch on `stream`.  Allocates a small buffer and synchronises the stream
 * (HGSR_ERR_STATE while it is being captured). */
hgsr_status hgsr_probe_valu_rate(double* wave_fma_per_s, hgsr_stream stream);


/* Stage timing.  While enabled, hgsr_render records HIP events on its
 * stream around its stages (0: projection, 1: tile binning and sort,
 * 2: blend), hgsr_render_backward around its stages (3: blend backward,
 * 4: projection backward) and hgsr_significance around stages 0 and 1, its
 * visibility walk (2) and its scoring pass (5); nothing is recorded while a
 * graph is captured.
 * hgsr_profile_read synchronises, returns the milliseconds accumulated per
 * stage (host array of 6 doubles) and the number of timed calls per stage
 * (host array of 6 int64, may be NULL), and resets the accumulators. */
hgsr_status hgsr_profile_enable(hgsr_ctx* ctx, int32_t enable);
hgsr_status hgsr_profile_read(hgsr_ctx* ctx, double* ms, int64_t* calls);

/* Thread-local description of the last error. */
const char* hgsr_last_error(void);

/* Library version string. */
const char* hgsr_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HGSR_H_ */
