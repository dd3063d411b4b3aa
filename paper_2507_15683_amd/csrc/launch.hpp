// Kernel argument blocks and host-side launchers (one per kernel family).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/hgsr.h"
#include "hgsr_device.hpp"

namespace hgsr {

// Sets the thread's hgsr_last_error() text; returns st.
hgsr_status report_error(hgsr_status st, const char* msg);

struct ProjectArgs {
  GaussArgs g;
  CamArgs c;
  const float* poses;        // P_total x 12
  int32_t P;                 // poses in this launch (<= kMaxPoses)
  int32_t pose_base;         // first pose of this launch
  Splat* recs;               // P_total x rec_cap
  uint2* rects;              // tile rectangle per record (tx0 | tx1 << 16, ty0 | ty1 << 16)
  uint32_t* pose_count;      // P x kSub sub-segment counters (may exceed rec_cap / kSub)
  uint32_t rec_cap;          // records per pose (a multiple of kSub)
  // tile counts taken here for few poses (else count_tiles_kernel): per
  // (pose, tile) for the bucket path, per record for the LSD path, or null
  uint32_t* tile_count;
  uint32_t* rec_keys;
  const uint64_t* part_vis;  // per pose: partitions that may be visible, or null
  // candidate (pose, Gaussian) pairs of the cull pass: per pose kSub
  // sub-segments of rec_cap / kSub Gaussian indices, with their counters
  uint32_t* cand;
  uint32_t* cand_count;
  int32_t* flags;            // [0]: overflow bits
};

struct BinArgs {
  CamArgs c;
  int32_t P;
  const Splat* recs;
  const uint2* rects;
  const uint32_t* pose_count;
  uint32_t rec_cap;
  uint32_t* tile_cursor;     // per (pose, tile) running slot
  const uint2* ranges;       // per (pose, tile) [begin, end)
  uint64_t* keys;            // (depth bits << 32 | gid) per entry
  uint32_t* vals;            // record index per entry
  uint64_t key_cap;
  int32_t* flags;
};

struct TileSortArgs {
  int32_t n_tiles;           // P x tiles
  const uint2* ranges;
  uint64_t* keys;
  uint32_t* vals;
  uint64_t* keys_alt;
  uint32_t* vals_alt;
  uint32_t* list;            // sorted record indices
  uint32_t* list_gid;        // Gaussian index of each sorted entry
  int32_t lds_cap;
  int32_t gid_bits;
  const int32_t* flags;
};

struct LsdArgs {
  const uint32_t* total;     // number of keys (device)
  uint64_t key_cap;
  int32_t n_blocks;          // blocks per pass (static, from capacity)
  uint64_t* keys[2];
  uint32_t* gids[2];
  uint32_t* vals[2];
  uint32_t* hist;            // 256 x n_blocks
  const int32_t* flags;
};

struct BlendArgs {
  CamArgs c;
  int32_t P;
  const uint2* ranges;
  const uint32_t* list;      // per-tile record indices in (depth, index) order
  const uint32_t* list_gid;  // Gaussian index of each list entry
  int32_t feat_mfma;         // accumulate 32 feature channels on the matrix cores
  const Splat* recs;
  const uint16_t* feat;      // n x D bf16
  float bg[3];
  float* rgb;
  float* depth;
  float* alpha;
  void* out_feat;
  float* final_T;
  uint32_t* n_used;
  int32_t schedule;
  int32_t n_items;
  uint32_t* queue;
  const int32_t* flags;
};

struct BackArgs {
  CamArgs c;
  int32_t P;
  int32_t feat_mfma;         // feature term of h on the matrix cores (D 32, one pixel per lane)
  const uint2* ranges;
  const uint32_t* list;
  const uint32_t* list_gid;  // Gaussian index of each list entry
  const Splat* recs;
  const uint16_t* feat;
  int32_t D;
  float bg[3];
  // residual loss and no per-Gaussian opacity gradient asked for: the
  // blend backward forms eight of the ten per-splat sums (no opacity or depth)
  int32_t pose_only;
  int32_t schedule;          // kSchedGrid, or a persistent queue of (pose, tile) items
  int32_t n_items;
  int32_t n_ctas;            // workgroups of the persistent launch
  uint32_t* queue;           // item counter (zero before the launch)
  const float* fwd_depth;
  const float* final_T;
  const uint32_t* n_used;
  const float* g_rgb;
  const float* g_depth;
  const float* g_alpha;
  const float* g_feat;
  float* g_rec;              // per record: du dv da db dc do dz dr dg db (+2 pad)
  float* g_featvec;          // n x D or null
  const int32_t* flags;
  // refinement residual formed per pixel in place of g_rgb / g_feat
  // (res_rgb_t != null): from the forward's rgb and feature outputs and the
  // targets; the per-(pose, tile) loss shares go to res_part
  const float* fwd_rgb;
  const void* fwd_feat;
  int32_t fwd_feat_bf16;
  const float* res_rgb_t;
  const float* res_feat_t;
  int32_t res_t_stride;      // 1: a target per pose; 0: one shared target
  float res_lam;
  float res_inv_hw;
  float* res_part;
};

struct ProjBackArgs {
  GaussArgs g;
  CamArgs c;
  const float* poses;
  int32_t P;
  const Splat* recs;
  const uint32_t* pose_count;
  uint32_t rec_cap;
  const float* g_rec;
  float* g_pose;
  float* g_means;
  float* g_opac;
  float* g_log_scales;
  float* g_quats;
  float* g_sh;
  const int32_t* flags;
};

constexpr int kGradRecStride = 12;

// Significance scoring: which Gaussians a view blends (vis: n rows of
// vis_stride bytes, one per view, vis_stride = P rounded up to 16; cleared
// before the walk), then per Gaussian the feature cosine at its projected
// mean summed over the views.
struct ContribArgs {
  CamArgs c;
  const uint2* ranges;
  const uint32_t* list;
  const Splat* recs;
  uint8_t* vis;
  int64_t vis_stride;
  const int32_t* flags;
};

struct ScoreArgs {
  CamArgs c;
  const float* poses;
  int32_t P;
  const float* means;
  const uint16_t* feat;
  int32_t D;
  int64_t n;
  const uint8_t* vis;
  int64_t vis_stride;
  const float* maps;
  int32_t map_w, map_h, map_layout;
  float* score_sum;
  uint32_t* vis_count;
  uint8_t* visible;
  const int32_t* flags;
  // planar maps, scored by map region (kScoreRegionW x kScoreRegionH cells
  // of one view): pairs binned per region, the region's planes staged in LDS
  int32_t n_rx, n_ry;        // regions per view along x and y
  uint32_t* rcount;          // pairs per region
  uint32_t* rcursor;         // placement cursor per region (zero before the scatter)
  const uint2* rranges;      // [begin, end) of each region's pairs
  uint2* pairs;              // (Gaussian, cell within its region) per pair
  float* cosb;               // per (Gaussian, view), Gaussian-major: the pair's cosine
};

constexpr int kScoreRegionW = 32;  // cells: a region row is one 128-byte line of a plane
constexpr int kScoreRegionH = 8;
constexpr int kScoreSegCells = 8;  // cells: a row segment is one 32-byte sector of a plane
static_assert(kScoreRegionW * kScoreRegionH / kScoreSegCells == 32, "one bit per row segment of a region");

// project.hip
void launch_partition_bounds(const GaussArgs& g, float* bounds, hipStream_t s);
void launch_partition_cull(const float* poses, int P, const float* bounds, int n_parts, const CamArgs& c,
                           uint64_t* vis, hipStream_t s);
// few poses: the fused pass per launch of up to kMaxPoses poses; many
// poses: the cull pass per launch of up to kMaxPoses poses, then the splat
// pass once for all
// group: Gaussians culled per thread of the fused pass (1 or 4)
void launch_project(const ProjectArgs& a, int group, hipStream_t s);
void launch_cull(const ProjectArgs& a, hipStream_t s);
void launch_splat(const ProjectArgs& a, int P_total, hipStream_t s);
void launch_validate(const GaussArgs& g, int32_t* bad, hipStream_t s);

// binning.hip
void launch_fill_u32(uint32_t* p, uint32_t value, int64_t n, hipStream_t s);
void launch_fill_f32(float* p, float value, int64_t n, hipStream_t s);
void launch_copy_u32(uint32_t* dst, const uint32_t* src, int64_t n, hipStream_t s);
void launch_clear4(uint32_t* p0, int64_t n0, uint32_t* p1, int64_t n1, uint32_t* p2, int64_t n2, uint32_t* p3,
                   int64_t n3, hipStream_t s);
int64_t scan_block_count(int64_t n);
void launch_scan(const uint32_t* in, int64_t n, uint32_t* out, uint2* ranges, uint32_t* block_sums,
                 uint32_t* total, uint64_t cap, int32_t* flags, int32_t flag_bit, hipStream_t s);
// tile_count (bucket) or rec_keys (LSD): the other may be null
void launch_count_tiles(const BinArgs& a, uint32_t* tile_count, uint32_t* rec_keys, hipStream_t s);
// lds: the per-workgroup LDS counters (many poses; the count kernel uses
// them whenever it runs on the bucket path)
void launch_emit_bucket(const BinArgs& a, bool lds, hipStream_t s);
void launch_tile_sort(const TileSortArgs& a, bool short_lists, hipStream_t s);
void launch_emit_lsd(const BinArgs& a, const uint32_t* rec_offsets, uint64_t* keys, uint32_t* gids,
                     uint32_t* vals, hipStream_t s);
void launch_lsd_sort(LsdArgs& a, int passes_gid, int passes_z, int passes_tile, int* out_buffer, hipStream_t s);
void launch_ranges_from_sorted(const uint64_t* keys, const uint32_t* total, uint64_t key_cap, uint2* ranges,
                               int32_t n_tiles, const int32_t* flags, hipStream_t s);

// blend.hip
void launch_loss_reduce(const float* part, int32_t tiles_per_pose, int32_t P, float* loss, hipStream_t s);
// probe.hip: wave64 FP32 FMA instructions per second the device issues
hipError_t probe_valu_rate(int n_cu, hipStream_t s, double* wave_fma_per_s);
void launch_blend_fwd(const BlendArgs& a, int D, bool bf16_out, int n_ctas, hipStream_t s);

// backward.hip
void launch_blend_bwd(const BackArgs& a, hipStream_t s);
void launch_project_bwd(const ProjBackArgs& a, hipStream_t s);
void launch_zero_grad_rec(float* g, const uint32_t* pose_count, uint32_t rec_cap, int P, hipStream_t s);

// match.hip: coarse-to-fine probabilistic mutual matching
struct MatchLaunch {
  const uint16_t* q_coarse;
  const uint16_t* r_coarse;
  const uint16_t* q_fine;   // null: coarse level only
  const uint16_t* r_fine;
  int32_t D, Hc, Wc, nq, nr;
  float tau_coarse, tau_fine;
  // workspace
  uint16_t* qvec;           // nq x D
  uint16_t* rvec;           // nr x D
  float* qnorm;
  float* rnorm;
  int32_t n_split;          // column ranges per row block (match_splits)
  float* row_part;          // n_split x nq
  int32_t* rowp_idx;        // n_split x nq
  float* col_part;          // row blocks x nr
  int32_t* colp_idx;        // row blocks x nr
  float* row_lse;           // nq
  float* col_lse;           // nr
  int32_t* row_arg;         // nq
  int32_t* col_arg;         // nr
  uint32_t* flag;           // nq
  uint32_t* offs;           // nq
  uint32_t* scan_tmp;
  // outputs
  uint32_t* n_coarse;
  int32_t* out_cq;
  int32_t* out_cr;
  float* out_cp;
  int32_t* out_fq;
  int32_t* out_fr;
  float* out_fp;
};
constexpr int kMatchRowBlock = 128;
int match_splits(int nq);
void launch_match(const MatchLaunch& L, hipStream_t s);

// pnp.hip: 2D-3D pose solve (RANSAC over given 3-point samples, refinement)
struct PnpArgs {
  const float* p2d;         // n x 2
  const float* x3d;         // n x 3
  int64_t n;
  const int32_t* samples;   // n_hyp x 3
  int32_t n_hyp;
  float tau;
  int32_t gn_iters, refine_iters;
  float fx, fy, cx, cy;
  const float* pose0;       // 12
  float* hyp;               // n_hyp x 12
  int32_t* counts;          // n_hyp (-1: invalid sample)
  int32_t* best;            // 1
  float* T;                 // 12: the pose being refined
  int32_t* state;           // 1: refinement running
  float* part;              // normal-equation partials, pnp_normal_blocks(n) x 28
  uint8_t* inliers;         // n or null
  int32_t* n_inliers;       // 1
  float* pose_out;          // 12
};
int pnp_normal_blocks(int64_t n);
void launch_pnp(const PnpArgs& a, hipStream_t s);
void launch_backproject(const float* depth, int W, int H, const float* pose, float fx, float fy, float cx, float cy,
                        const int32_t* pix, int n, float* x3d, hipStream_t s);
void launch_pose_consistency(const float* poses, int n, float tau_deg, int32_t* reliable, float* max_angle,
                             hipStream_t s);

// score.hip
void launch_contrib(const ContribArgs& a, int n_items, hipStream_t s);
void launch_score(const ScoreArgs& a, hipStream_t s);
// planar maps by region: count pairs per region (pass 0) or place them (pass 1)
void launch_score_bin(const ScoreArgs& a, int pass, hipStream_t s);
void launch_score_regions(const ScoreArgs& a, hipStream_t s);
void launch_score_reduce(const ScoreArgs& a, hipStream_t s);
void launch_score_final(const float* sum, const uint32_t* count, int64_t n, float* score, hipStream_t s);

// refine.hip
void launch_residual(const float* rgb, const void* feat, int feat_bf16, const float* rgb_t, const float* feat_t,
                     int P, int H, int W, int D, float lam_f, float* loss, float* g_rgb, float* g_feat,
                     hipStream_t s);
void launch_pose_retract(const float* poses, const float* xi, int P, float* out, hipStream_t s);
void launch_pose_tangent_grad(const float* xi, const float* g, int P, float* g_xi, hipStream_t s);
void launch_pose_adam(float* poses, const float* grad, float* m, float* v, int32_t* step, int P, float lr_rho,
                      float lr_phi, float b1, float b2, float eps, hipStream_t s);

}  // namespace hgsr
