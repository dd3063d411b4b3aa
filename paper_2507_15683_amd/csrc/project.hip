// Per-Gaussian stage: partition frustum cull, EWA projection, SH colour,
// support rectangle, per-pose compaction of visible splats and the per-tile
// entry counts of the tile binning.
#include "hgsr_device.hpp"
#include "launch.hpp"

namespace hgsr {

// ------------------------------------------------------------ partitions
// Box of partition k: every Gaussian's ball of radius 3.33 x its largest
// scale (the 1/255 support of an opaque Gaussian along its longest axis).
__global__ __launch_bounds__(256) void partition_bounds_kernel(GaussArgs g, float* bounds) {
  const int k = blockIdx.x;
  const int64_t b = g.part_offsets[k], e = g.part_offsets[k + 1];
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = b + threadIdx.x; i < e; i += blockDim.x) {
    const float s = __expf(fmaxf(g.log_scales[3 * i], fmaxf(g.log_scales[3 * i + 1], g.log_scales[3 * i + 2])));
    const float r = 3.33f * s;
    for (int a = 0; a < 3; ++a) {
      lo[a] = fminf(lo[a], g.means[3 * i + a] - r);
      hi[a] = fmaxf(hi[a], g.means[3 * i + a] + r);
    }
  }
  __shared__ float red[6][256];
  for (int a = 0; a < 3; ++a) {
    red[a][threadIdx.x] = lo[a];
    red[3 + a][threadIdx.x] = hi[a];
  }
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s)
      for (int a = 0; a < 3; ++a) {
        red[a][threadIdx.x] = fminf(red[a][threadIdx.x], red[a][threadIdx.x + s]);
        red[3 + a][threadIdx.x] = fmaxf(red[3 + a][threadIdx.x], red[3 + a][threadIdx.x + s]);
      }
    __syncthreads();
  }
  if (threadIdx.x < 6) bounds[6 * k + threadIdx.x] = red[threadIdx.x][0];
}

// Per (pose, partition): 1 when the partition's box may reach the image.
// The box is rejected only when all 8 corners lie behind the near plane or on
// the outer side of one of the four image-side planes (through the camera
// centre, pushed out by a margin of `margin` pixels).  One wave per pose, one
// lane per partition (at most 64), the mask assembled by a ballot.
__device__ __forceinline__ bool box_may_be_seen(const float* T, const float* B, const CamArgs& c, float margin) {
  if (!(B[0] <= B[3] && B[1] <= B[4] && B[2] <= B[5])) return false;  // empty (or NaN): nothing to draw
  const float l = (-margin - c.cx) / c.fx, r = (c.W + margin - c.cx) / c.fx;
  const float t = (-margin - c.cy) / c.fy, b = (c.H + margin - c.cy) / c.fy;
  bool all_near = true, all_l = true, all_r = true, all_t = true, all_b = true;
  for (int q = 0; q < 8; ++q) {
    const float w[3] = {(q & 1) ? B[3] : B[0], (q & 2) ? B[4] : B[1], (q & 4) ? B[5] : B[2]};
    float m[3];
    to_camera(T, w, m);
    all_near &= m[2] < c.near_z;
    all_l &= m[0] < l * m[2];
    all_r &= m[0] > r * m[2];
    all_t &= m[1] < t * m[2];
    all_b &= m[1] > b * m[2];
  }
  return !(all_near || all_l || all_r || all_t || all_b);
}

// The margin in pixels by which the image-side planes are pushed out.
__device__ __forceinline__ float box_margin(const CamArgs& c) {
  return 8.f + 0.05f * static_cast<float>(c.W > c.H ? c.W : c.H);
}

__global__ __launch_bounds__(64) void partition_cull_kernel(const float* poses, int P, const float* bounds,
                                                            int n_parts, CamArgs c, float margin, uint64_t* vis) {
  const int p = blockIdx.x;
  const int k = threadIdx.x;
  if (p >= P) return;  // uniform
  const bool seen = k < n_parts && box_may_be_seen(poses + 12 * p, bounds + 6 * k, c, margin);
  const uint64_t mask = __ballot(seen);
  if (k == 0) vis[p] = mask;
}

// True when no pose of the launch may see a partition overlapping the
// Gaussian range [i0, i1]: the workgroup covering it exits before reading
// anything (the same for all its threads).
__device__ __forceinline__ bool range_culled(const ProjectArgs& a, int64_t i0, int64_t i1) {
  if (a.g.n_parts <= 0) return false;
  int p0 = 0;
  while (p0 + 1 < a.g.n_parts && a.g.part_offsets[p0 + 1] <= i0) ++p0;
  int p1 = p0;
  while (p1 + 1 < a.g.n_parts && a.g.part_offsets[p1 + 1] <= i1) ++p1;
  uint64_t seen = 0;
  for (int p = 0; p < a.P; ++p) seen |= a.part_vis[a.pose_base + p];
  const int w = p1 - p0 + 1;
  const uint64_t span = (w >= 64 ? ~0ull : ((1ull << w) - 1ull)) << p0;
  return (seen & span) == 0;
}

// ------------------------------------------------------------ projection
// Few poses, compacted: a block culls G x 256 Gaussians with the
// cheap tests (opacity, partition, near plane, conservative footprint bound;
// all loads of a thread issued together), appends the candidates to an LDS
// list, and then runs the exact footprint, the record and the tile counts
// over that list with consecutive threads -- the ~7 % of Gaussians a view
// keeps fill whole waves instead of a few lanes of every wave.  Visible
// (pose, Gaussian) pairs are compacted per pose: phase B counts them per
// wave and then per block in LDS, one global atomic per (block, pose)
// reserves a range of one of the pose's kSub record sub-segments, and phase
// C writes the records at each lane's rank in its wave's share (with the
// footprint kept from phase B for one pose and one Gaussian per thread,
// else recomputed from the same inputs with the same arithmetic).  Every
// LDS counter is taken once per wave: LDS atomics from all lanes on one
// address are performed one lane after another.  G = 1 (the
// default) suits spatially ordered scenes (a workgroup keeps all or nothing,
// and small workgroups spread the kept ones over the chip); G = 4 suits
// scenes in arbitrary order (every workgroup keeps a few percent).  The
// autotuner picks.

// Tile-count histogram of one block's records when they fall in a small tile
// rectangle (a spatially ordered scene): counted in LDS, then one global
// atomic per non-empty tile instead of one per (record, tile).
constexpr int kProjHist = 2048;
struct BlockHist {
  uint32_t* bins;  // LDS, kProjHist, or null: count in global memory
  int tx0, ty0, w;
};

// SH colour (Sec. 3.1) of Gaussian i seen from the camera of pose T: the
// basis evaluated at the unit direction from the camera centre to the mean.
template <int DEG>
__device__ __forceinline__ void view_colour(const ProjectArgs& a, int64_t i, const float mu[3], const float* T,
                                            float rgb[3]) {
  const float Cx = -(T[0] * T[3] + T[4] * T[7] + T[8] * T[11]);
  const float Cy = -(T[1] * T[3] + T[5] * T[7] + T[9] * T[11]);
  const float Cz = -(T[2] * T[3] + T[6] * T[7] + T[10] * T[11]);
  float dx = mu[0] - Cx, dy = mu[1] - Cy, dz = mu[2] - Cz;
  const float inv = rsqrtf(dx * dx + dy * dy + dz * dz);
  dx *= inv; dy *= inv; dz *= inv;
  sh_colour_raw<DEG>(a.g.sh, i, dx, dy, dz, rgb);
}

template <int DEG>
__device__ __forceinline__ void write_record(const ProjectArgs& a, int64_t i, const float mu[3], float o, float k2,
                                             const float* T, int pg, const float mc[3], const Footprint& f,
                                             uint32_t slot, const BlockHist& hist, const float* rgb_in = nullptr) {
  float rgb[3];
  if (rgb_in) {
    rgb[0] = rgb_in[0]; rgb[1] = rgb_in[1]; rgb[2] = rgb_in[2];
  } else {
    view_colour<DEG>(a, i, mu, T, rgb);
  }
  const int64_t idx = static_cast<int64_t>(pg) * a.rec_cap + slot;
  Splat sp;
  sp.u = f.u; sp.v = f.v; sp.ca = f.ca; sp.cb = f.cb;
  sp.cc = f.cc; sp.o = o; sp.z = mc[2]; sp.gid = static_cast<uint32_t>(i);
  sp.r = fmaxf(rgb[0], 0.f); sp.g = fmaxf(rgb[1], 0.f); sp.b = fmaxf(rgb[2], 0.f);
  sp.pmin = -0.5f * k2;
  float4* dst = reinterpret_cast<float4*>(a.recs + idx);
  const float4* src = reinterpret_cast<const float4*>(&sp);
  dst[0] = src[0]; dst[1] = src[1]; dst[2] = src[2];
  const int tx0 = f.px0 >> a.c.tile_shift, tx1 = f.px1 >> a.c.tile_shift;
  const int ty0 = f.py0 >> a.c.tile_shift, ty1 = f.py1 >> a.c.tile_shift;
  a.rects[idx] = make_uint2(static_cast<uint32_t>(tx0) | (static_cast<uint32_t>(tx1) << 16),
                            static_cast<uint32_t>(ty0) | (static_cast<uint32_t>(ty1) << 16));
  if (a.tile_count || a.rec_keys) {
    const SplatShape shp = splat_shape(sp.u, sp.v, sp.ca, sp.cb, sp.cc, -2.f * sp.pmin);
    uint32_t ntiles = 0;
    uint32_t* tc = a.tile_count ? a.tile_count + static_cast<int64_t>(pg) * a.c.tiles_per_pose : nullptr;
    for (int ty = ty0; ty <= ty1; ++ty) {
      int ta, tb;
      row_span(shp, ty, a.c.tile, a.c.W, a.c.H, tx0, tx1, &ta, &tb);
      if (hist.bins && tc) {
        for (int tx = ta; tx <= tb; ++tx) atomicAdd(&hist.bins[(ty - hist.ty0) * hist.w + (tx - hist.tx0)], 1u);
        ntiles += tb >= ta ? static_cast<uint32_t>(tb - ta + 1) : 0u;
        continue;
      }
      for (int tx = ta; tx <= tb; ++tx) {
        ++ntiles;
        if (tc) atomicAdd(&tc[ty * a.c.ntx + tx], 1u);
      }
    }
    if (a.rec_keys) a.rec_keys[idx] = ntiles;
  }
}

template <int DEG, int G>
__global__ __launch_bounds__(256) void project_dense_kernel(ProjectArgs a) {
  constexpr int kProjPerThread = G;
  constexpr int kProjBlockItems = 256 * G;
  __shared__ uint32_t s_cnt[kMaxPoses];
  __shared__ uint32_t s_base[kMaxPoses];
  __shared__ uint32_t s_nc;
  __shared__ uint32_t s_idx[kProjBlockItems];  // candidate: offset from the block's first Gaussian
  __shared__ uint64_t s_mask[kProjBlockItems]; // poses that may see it
  __shared__ uint32_t s_hist[kProjHist];
  __shared__ int s_rect[4];                     // tile rectangle of the block's records (one pose)
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const uint64_t lanes_below = (uint64_t{1} << lane) - 1u;
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kProjBlockItems;
  if (range_culled(a, base, min(base + kProjBlockItems, a.g.n) - 1)) return;
  for (int p = tid; p < a.P; p += 256) s_cnt[p] = 0;
  if (tid == 0) {
    s_nc = 0;
    s_rect[0] = s_rect[1] = 0x7fffffff;
    s_rect[2] = s_rect[3] = -1;
  }
  // opacity, mean and largest log-scale in one round of loads (not gated on
  // the opacity test: a dependent round costs more than the few bytes of
  // the Gaussians that test drops)
  float o[kProjPerThread], mu[kProjPerThread][3], lsm[kProjPerThread];
#pragma unroll
  for (int q = 0; q < kProjPerThread; ++q) {
    const int64_t i = base + q * 256 + tid;
    o[q] = 0.f;
    mu[q][0] = mu[q][1] = mu[q][2] = lsm[q] = 0.f;
    if (i < a.g.n) {
      o[q] = a.g.opac[i];
      mu[q][0] = a.g.means[3 * i];
      mu[q][1] = a.g.means[3 * i + 1];
      mu[q][2] = a.g.means[3 * i + 2];
      lsm[q] = fmaxf(a.g.log_scales[3 * i], fmaxf(a.g.log_scales[3 * i + 1], a.g.log_scales[3 * i + 2]));
    }
  }

  // phase A: the cheap tests
  uint64_t pose_ok[kProjPerThread];
  bool live[kProjPerThread];
#pragma unroll
  for (int q = 0; q < kProjPerThread; ++q) {
    const int64_t i = base + q * 256 + tid;
    live[q] = o[q] >= kAlphaMin;  // also false for NaN and past the end
    pose_ok[q] = ~0ull;
    if (live[q] && a.g.n_parts > 0) {
      int part = 0;
      while (part + 1 < a.g.n_parts && a.g.part_offsets[part + 1] <= i) ++part;
      uint64_t ok = 0;
      for (int p = 0; p < a.P; ++p)
        if ((a.part_vis[a.pose_base + p] >> part) & 1ull) ok |= (1ull << p);
      pose_ok[q] = ok;
      live[q] = ok != 0;
    }
  }
  __syncthreads();  // s_nc and s_cnt cleared
#pragma unroll
  for (int q = 0; q < kProjPerThread; ++q) {
    uint64_t cand = 0;
    if (live[q]) {
      const float s2max = __expf(2.f * lsm[q]);
      const float k2 = 2.f * __logf(255.f * o[q]);
      for (int p = 0; p < a.P; ++p) {
        if (!((pose_ok[q] >> p) & 1ull)) continue;
        const float* T = a.poses + 12 * (a.pose_base + p);
        float mc[3];
        to_camera(T, mu[q], mc);
        if (!(mc[2] > a.c.near_z)) continue;
        if (maybe_visible(mc, s2max, k2, a.c)) cand |= 1ull << p;
      }
    }
    // appended per wave: one LDS atomic, each lane at its rank
    const uint64_t bal = __ballot(cand != 0);
    if (bal) {
      const int leader = __builtin_ctzll(bal);
      uint32_t wbase = 0;
      if (lane == leader) wbase = atomicAdd(&s_nc, static_cast<uint32_t>(__popcll(bal)));
      wbase = __shfl(wbase, leader, kWave);
      if (cand) {
        const uint32_t e = wbase + static_cast<uint32_t>(__popcll(bal & lanes_below));
        s_idx[e] = static_cast<uint32_t>(q * 256 + tid);
        s_mask[e] = cand;
      }
    }
  }
  __syncthreads();
  const uint32_t nc = s_nc;
  if (nc == 0) return;  // uniform: no candidate, nothing counted or written

  // phase B: exact footprints on the compacted candidates, counted per pose
  // (per wave first: an LDS atomic from every lane on one address would be
  // performed one lane after another)
  int rect[4] = {0x7fffffff, 0x7fffffff, -1, -1};  // one pose: tile rectangle of this lane's records
  uint64_t vis[kProjPerThread];
  // one Gaussian per thread and one pose: phase C reuses phase B's footprint
  constexpr bool kKeep = G == 1;
  float keep_m[3] = {0.f, 0.f, 0.f}, keep_mc[3] = {0.f, 0.f, 0.f}, keep_o = 0.f, keep_k2 = 0.f;
  Footprint keep_f{};
#pragma unroll
  for (int k = 0; k < kProjPerThread; ++k) {
    vis[k] = 0;
    const uint32_t e = static_cast<uint32_t>(k * 256 + tid);
    if (e >= nc) continue;
    const int64_t i = base + s_idx[e];
    const uint64_t cand = s_mask[e];
    const float m[3] = {a.g.means[3 * i], a.g.means[3 * i + 1], a.g.means[3 * i + 2]};
    const float ls[3] = {a.g.log_scales[3 * i], a.g.log_scales[3 * i + 1], a.g.log_scales[3 * i + 2]};
    const float oo = a.g.opac[i];
    const float k2 = 2.f * __logf(255.f * oo);
    float S[6];
    cov3_from(reinterpret_cast<const float4*>(a.g.quats)[i], ls, S);
    for (int p = 0; p < a.P; ++p) {
      if (!((cand >> p) & 1ull)) continue;
      const float* T = a.poses + 12 * (a.pose_base + p);
      float mc[3];
      to_camera(T, m, mc);
      Footprint f;
      if (footprint(T, mc, S, k2, a.c, f)) {
        vis[k] |= 1ull << p;
        if (kKeep && a.P == 1) {
          for (int c = 0; c < 3; ++c) {
            keep_m[c] = m[c];
            keep_mc[c] = mc[c];
          }
          keep_o = oo;
          keep_k2 = k2;
          keep_f = f;
        }
        if (a.P == 1) {
          rect[0] = min(rect[0], f.px0 >> a.c.tile_shift);
          rect[1] = min(rect[1], f.py0 >> a.c.tile_shift);
          rect[2] = max(rect[2], f.px1 >> a.c.tile_shift);
          rect[3] = max(rect[3], f.py1 >> a.c.tile_shift);
        }
      }
    }
  }
  for (int p = 0; p < a.P; ++p) {  // uniform: every lane of the wave
    uint32_t cnt = 0;
#pragma unroll
    for (int k = 0; k < kProjPerThread; ++k) cnt += static_cast<uint32_t>(__popcll(__ballot((vis[k] >> p) & 1ull)));
    if (lane == 0 && cnt) atomicAdd(&s_cnt[p], cnt);
  }
  if (a.P == 1) {
    for (int off = kWave / 2; off > 0; off >>= 1) {
      rect[0] = min(rect[0], __shfl_xor(rect[0], off, kWave));
      rect[1] = min(rect[1], __shfl_xor(rect[1], off, kWave));
      rect[2] = max(rect[2], __shfl_xor(rect[2], off, kWave));
      rect[3] = max(rect[3], __shfl_xor(rect[3], off, kWave));
    }
    if (lane == 0 && rect[2] >= 0) {
      atomicMin(&s_rect[0], rect[0]);
      atomicMin(&s_rect[1], rect[1]);
      atomicMax(&s_rect[2], rect[2]);
      atomicMax(&s_rect[3], rect[3]);
    }
  }
  __syncthreads();
  const int sub = static_cast<int>(blockIdx.x % kSub);
  const uint32_t sub_cap = a.rec_cap / kSub;
  for (int p = tid; p < a.P; p += 256) {
    const uint32_t cnt = s_cnt[p];
    s_base[p] = cnt ? atomicAdd(&a.pose_count[(a.pose_base + p) * kSub + sub], cnt) : 0u;
    s_cnt[p] = 0;
  }
  // one pose whose records span a small tile rectangle: count in LDS
  BlockHist hist;
  hist.bins = nullptr;
  hist.tx0 = s_rect[0];
  hist.ty0 = s_rect[1];
  hist.w = s_rect[2] - s_rect[0] + 1;
  const int hist_h = s_rect[3] - s_rect[1] + 1;
  const bool use_hist = a.P == 1 && a.tile_count && s_rect[2] >= 0 && hist.w * hist_h <= kProjHist;
  if (use_hist) {
    hist.bins = s_hist;
    for (int b = tid; b < hist.w * hist_h; b += 256) s_hist[b] = 0;
  }
  __syncthreads();

  // phase C: the records (footprints recomputed from the same inputs, or
  // kept from phase B), in slots the wave takes together: one LDS atomic per
  // wave and pose, each lane's slot at its rank among the wave's records
#pragma unroll
  for (int k = 0; k < kProjPerThread; ++k) {
    const uint32_t e = static_cast<uint32_t>(k * 256 + tid);
    int64_t i = 0;
    float m[3] = {0.f, 0.f, 0.f}, oo = 0.f, k2 = 0.f, S[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    const bool keep = kKeep && a.P == 1;
    if (vis[k]) {
      i = base + s_idx[e];
      if (!keep) {
        m[0] = a.g.means[3 * i]; m[1] = a.g.means[3 * i + 1]; m[2] = a.g.means[3 * i + 2];
        const float ls[3] = {a.g.log_scales[3 * i], a.g.log_scales[3 * i + 1], a.g.log_scales[3 * i + 2]};
        oo = a.g.opac[i];
        k2 = 2.f * __logf(255.f * oo);
        cov3_from(reinterpret_cast<const float4*>(a.g.quats)[i], ls, S);
      }
    }
    for (int p = 0; p < a.P; ++p) {  // uniform: every lane of the wave
      const bool has = (vis[k] >> p) & 1ull;
      const uint64_t bal = __ballot(has);
      if (bal == 0) continue;
      const int leader = __builtin_ctzll(bal);
      uint32_t wbase = 0;
      if (lane == leader) wbase = atomicAdd(&s_cnt[p], static_cast<uint32_t>(__popcll(bal)));
      wbase = __shfl(wbase, leader, kWave);
      if (!has) continue;
      const uint32_t local = s_base[p] + wbase + static_cast<uint32_t>(__popcll(bal & lanes_below));
      if (local >= sub_cap) {
        atomicOr(a.flags, 1);
        continue;
      }
      if (keep) {
        write_record<DEG>(a, i, keep_m, keep_o, keep_k2, a.poses + 12 * a.pose_base, a.pose_base, keep_mc, keep_f,
                          sub * sub_cap + local, hist);
        continue;
      }
      const int pg = a.pose_base + p;
      const float* T = a.poses + 12 * pg;
      float mc[3];
      to_camera(T, m, mc);
      Footprint f;
      footprint(T, mc, S, k2, a.c, f);
      write_record<DEG>(a, i, m, oo, k2, T, pg, mc, f, sub * sub_cap + local, hist);
    }
  }
  if (use_hist) {
    __syncthreads();
    uint32_t* tc = a.tile_count + static_cast<int64_t>(a.pose_base) * a.c.tiles_per_pose;
    for (int b = tid; b < hist.w * hist_h; b += 256) {
      const uint32_t v = s_hist[b];
      if (v) atomicAdd(&tc[(hist.ty0 + b / hist.w) * a.c.ntx + hist.tx0 + b % hist.w], v);
    }
  }
}

// Many poses: two passes, so that the expensive per-pair work runs on dense lanes.
//
// cull_kernel: one thread per Gaussian, looping over the launch's poses,
// applies the opacity, partition, near-plane and conservative footprint
// tests (maybe_visible: no covariance is formed) and appends the Gaussian's
// index to the candidate list of every pose that may see it.  Per block and
// pose the candidates are counted in LDS and one global atomic reserves a
// range of one of the pose's kSub candidate sub-segments.
//
// splat_kernel: one thread per candidate (pose, Gaussian): the EWA
// footprint with the exact support test, the SH colour, and the record;
// a block holds candidates of one pose sub-segment, so one LDS count and
// one global atomic per block reserve its records.
__global__ __launch_bounds__(256) void cull_kernel(ProjectArgs a) {
  __shared__ uint32_t s_cnt[kMaxPoses];
  __shared__ uint32_t s_base[kMaxPoses];
  const int tid = threadIdx.x;
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + tid;
  if (range_culled(a, static_cast<int64_t>(blockIdx.x) * 256, min(static_cast<int64_t>(blockIdx.x) * 256 + 256, a.g.n) - 1))
    return;
  for (int p = tid; p < a.P; p += 256) s_cnt[p] = 0;

  bool live = i < a.g.n;
  float mu[3] = {0.f, 0.f, 0.f}, o = 0.f, k2 = 0.f, s2max = 0.f;
  uint64_t pose_ok = ~0ull;
  if (live) {
    o = a.g.opac[i];
    live = o >= kAlphaMin;  // also false for NaN
    if (live && a.g.n_parts > 0) {
      int part = 0;
      while (part + 1 < a.g.n_parts && a.g.part_offsets[part + 1] <= i) ++part;
      pose_ok = 0;
      for (int p = 0; p < a.P; ++p)
        if ((a.part_vis[a.pose_base + p] >> part) & 1ull) pose_ok |= (1ull << p);
      live = pose_ok != 0;
    }
  }
  if (live) {
    mu[0] = a.g.means[3 * i];
    mu[1] = a.g.means[3 * i + 1];
    mu[2] = a.g.means[3 * i + 2];
    const float l0 = a.g.log_scales[3 * i], l1 = a.g.log_scales[3 * i + 1], l2 = a.g.log_scales[3 * i + 2];
    s2max = __expf(2.f * fmaxf(l0, fmaxf(l1, l2)));
    k2 = 2.f * __logf(255.f * o);
  }
  const int lane = tid & (kWave - 1), wave = tid >> 6;
  const uint64_t lanes_below = (uint64_t{1} << lane) - 1u;
  // The poses that may see any Gaussian of this block: the block's box (each
  // live Gaussian's ball of twice the 1/255 support radius of its largest
  // scale, 2 x 3.33 s: the linearised footprint the per-Gaussian test bounds
  // stays inside it) against each pose's frustum, the image-side planes
  // pushed out as for partitions.  The per-Gaussian tests then run only for
  // those poses (a view sees a few percent of the scene).
  __shared__ float s_box[256 / kWave][6];
  __shared__ uint64_t s_pmask;
  {
    float bx[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    if (live) {
      const float rr = 2.f * 3.33f * sqrtf(s2max);
      for (int d = 0; d < 3; ++d) {
        bx[d] = mu[d] - rr;
        bx[3 + d] = mu[d] + rr;
      }
    }
    for (int off = kWave / 2; off > 0; off >>= 1)
      for (int d = 0; d < 3; ++d) {
        bx[d] = fminf(bx[d], __shfl_xor(bx[d], off, kWave));
        bx[3 + d] = fmaxf(bx[3 + d], __shfl_xor(bx[3 + d], off, kWave));
      }
    if (lane == 0)
      for (int d = 0; d < 6; ++d) s_box[wave][d] = bx[d];
  }
  __syncthreads();  // s_box written, s_cnt cleared
  if (tid < kWave) {  // the first wave, one lane per pose (P <= 64)
    float B[6];
    for (int d = 0; d < 3; ++d) {
      B[d] = fminf(fminf(s_box[0][d], s_box[1][d]), fminf(s_box[2][d], s_box[3][d]));
      B[3 + d] = fmaxf(fmaxf(s_box[0][3 + d], s_box[1][3 + d]), fmaxf(s_box[2][3 + d], s_box[3][3 + d]));
    }
    const bool seen = tid < a.P && box_may_be_seen(a.poses + 12 * (a.pose_base + tid), B, a.c, box_margin(a.c));
    const uint64_t m = __ballot(seen);
    if (tid == 0) s_pmask = m;
  }
  __syncthreads();
  // counted per wave and pose (an LDS atomic from every lane on one address
  // would be performed one lane after another)
  uint64_t cand = 0;
  for (uint64_t pm = s_pmask; pm; pm &= pm - 1) {  // uniform: every lane of the wave
    const int p = __builtin_ctzll(pm);
    bool ok = false;
    if (live && ((pose_ok >> p) & 1ull)) {
      const float* T = a.poses + 12 * (a.pose_base + p);
      float mc[3];
      to_camera(T, mu, mc);
      ok = mc[2] > a.c.near_z && maybe_visible(mc, s2max, k2, a.c);
    }
    const uint64_t bal = __ballot(ok);
    if (lane == 0 && bal) atomicAdd(&s_cnt[p], static_cast<uint32_t>(__popcll(bal)));
    if (ok) cand |= 1ull << p;
  }
  __syncthreads();
  const int sub = static_cast<int>(blockIdx.x % kSub);
  const uint32_t sub_cap = a.rec_cap / kSub;
  for (int p = tid; p < a.P; p += 256) {
    const uint32_t cnt = s_cnt[p];
    s_base[p] = cnt ? atomicAdd(&a.cand_count[(a.pose_base + p) * kSub + sub], cnt) : 0u;
    s_cnt[p] = 0;
  }
  __syncthreads();
  // each pose's candidates take their slots per wave: one LDS atomic, each
  // lane at its rank
  uint64_t wave_cand = cand;  // OR over the wave (butterfly)
  for (int off = kWave / 2; off > 0; off >>= 1) {
    const uint64_t other =
        (static_cast<uint64_t>(__shfl_xor(static_cast<uint32_t>(wave_cand >> 32), off, kWave)) << 32) |
        __shfl_xor(static_cast<uint32_t>(wave_cand), off, kWave);
    wave_cand |= other;
  }
  while (wave_cand) {  // uniform: the poses any lane of the wave keeps
    const int p = __builtin_ctzll(wave_cand);
    wave_cand &= wave_cand - 1ull;
    const bool has = (cand >> p) & 1ull;
    const uint64_t bal = __ballot(has);
    const int leader = __builtin_ctzll(bal);
    uint32_t wbase = 0;
    if (lane == leader) wbase = atomicAdd(&s_cnt[p], static_cast<uint32_t>(__popcll(bal)));
    wbase = __shfl(wbase, leader, kWave);
    if (!has) continue;
    const uint32_t local = s_base[p] + wbase + static_cast<uint32_t>(__popcll(bal & lanes_below));
    if (local >= sub_cap) {
      atomicOr(a.flags, 1);
      continue;
    }
    a.cand[static_cast<int64_t>(a.pose_base + p) * a.rec_cap + sub * sub_cap + local] = static_cast<uint32_t>(i);
  }
}

// Candidates per splat block.
constexpr int kSplatBlock = 256;

template <int DEG>
__global__ __launch_bounds__(kSplatBlock) void splat_kernel(ProjectArgs a) {
  __shared__ uint32_t s_cnt, s_base;
  const int tid = threadIdx.x;
  const uint32_t sub_cap = a.rec_cap / kSub;
  const int chunks = static_cast<int>((sub_cap + kSplatBlock - 1) / kSplatBlock);
  // block -> (pose, candidate sub-segment, chunk of kSplatBlock candidates)
  const int chunk = static_cast<int>(blockIdx.x % chunks);
  const int csub = static_cast<int>((blockIdx.x / chunks) % kSub);
  const int pg = static_cast<int>(blockIdx.x / (chunks * kSub));
  const uint32_t n_cand = min(a.cand_count[pg * kSub + csub], sub_cap);
  const uint32_t first = static_cast<uint32_t>(chunk) * kSplatBlock;
  if (first >= n_cand) return;  // uniform: the whole block leaves
  if (tid == 0) s_cnt = 0;
  const uint32_t c = first + tid;
  bool vis = false;
  int64_t i = 0;
  float mu[3], mc[3], o = 0.f, k2 = 0.f;
  Footprint f;
  const float* T = a.poses + 12 * pg;
  if (c < n_cand) {
    i = a.cand[static_cast<int64_t>(pg) * a.rec_cap + csub * sub_cap + c];
    o = a.g.opac[i];
    mu[0] = a.g.means[3 * i];
    mu[1] = a.g.means[3 * i + 1];
    mu[2] = a.g.means[3 * i + 2];
    const float ls[3] = {a.g.log_scales[3 * i], a.g.log_scales[3 * i + 1], a.g.log_scales[3 * i + 2]};
    k2 = 2.f * __logf(255.f * o);
    float S[6];
    cov3_from(reinterpret_cast<const float4*>(a.g.quats)[i], ls, S);
    to_camera(T, mu, mc);
    vis = footprint(T, mc, S, k2, a.c, f);
  }
  // slots taken per wave (one LDS atomic, each lane at its rank)
  const int lane = tid & (kWave - 1);
  __syncthreads();  // s_cnt cleared
  const uint64_t bal = __ballot(vis);
  uint32_t local = 0;
  if (bal) {
    const int leader = __builtin_ctzll(bal);
    if (lane == leader) local = atomicAdd(&s_cnt, static_cast<uint32_t>(__popcll(bal)));
    local = __shfl(local, leader, kWave) + static_cast<uint32_t>(__popcll(bal & ((uint64_t{1} << lane) - 1u)));
  }
  __syncthreads();
  // records go to one of the pose's kSub record sub-segments, picked by
  // block index, so that the reservation atomics spread over kSub addresses
  const int sub = static_cast<int>(blockIdx.x % kSub);
  if (tid == 0) s_base = s_cnt ? atomicAdd(&a.pose_count[pg * kSub + sub], s_cnt) : 0u;
  __syncthreads();
  if (!vis) return;
  local += s_base;
  if (local >= sub_cap) {
    atomicOr(a.flags, 1);
    return;
  }
  const uint32_t slot = sub * sub_cap + local;
  // view direction from the camera centre C = -R^T t
  const float Cx = -(T[0] * T[3] + T[4] * T[7] + T[8] * T[11]);
  const float Cy = -(T[1] * T[3] + T[5] * T[7] + T[9] * T[11]);
  const float Cz = -(T[2] * T[3] + T[6] * T[7] + T[10] * T[11]);
  float dx = mu[0] - Cx, dy = mu[1] - Cy, dz = mu[2] - Cz;
  const float inv = rsqrtf(dx * dx + dy * dy + dz * dz);
  dx *= inv; dy *= inv; dz *= inv;
  float rgb[3];
  sh_colour_raw<DEG>(a.g.sh, i, dx, dy, dz, rgb);
  const int64_t idx = static_cast<int64_t>(pg) * a.rec_cap + slot;
  Splat sp;
  sp.u = f.u; sp.v = f.v; sp.ca = f.ca; sp.cb = f.cb;
  sp.cc = f.cc; sp.o = o; sp.z = mc[2]; sp.gid = static_cast<uint32_t>(i);
  sp.r = fmaxf(rgb[0], 0.f); sp.g = fmaxf(rgb[1], 0.f); sp.b = fmaxf(rgb[2], 0.f);
  sp.pmin = -0.5f * k2;
  float4* dst = reinterpret_cast<float4*>(a.recs + idx);
  const float4* src = reinterpret_cast<const float4*>(&sp);
  dst[0] = src[0]; dst[1] = src[1]; dst[2] = src[2];
  const int tx0 = f.px0 >> a.c.tile_shift, tx1 = f.px1 >> a.c.tile_shift;
  const int ty0 = f.py0 >> a.c.tile_shift, ty1 = f.py1 >> a.c.tile_shift;
  a.rects[idx] = make_uint2(static_cast<uint32_t>(tx0) | (static_cast<uint32_t>(tx1) << 16),
                            static_cast<uint32_t>(ty0) | (static_cast<uint32_t>(ty1) << 16));
  // few poses: the record's tiles are counted here (row spans of the same
  // stored values count_tiles_kernel would read); many poses: there
  if (a.tile_count || a.rec_keys) {
    const SplatShape shp = splat_shape(sp.u, sp.v, sp.ca, sp.cb, sp.cc, -2.f * sp.pmin);
    uint32_t ntiles = 0;
    uint32_t* tc = a.tile_count ? a.tile_count + static_cast<int64_t>(pg) * a.c.tiles_per_pose : nullptr;
    for (int ty = ty0; ty <= ty1; ++ty) {
      int ta, tb;
      row_span(shp, ty, a.c.tile, a.c.W, a.c.H, tx0, tx1, &ta, &tb);
      for (int tx = ta; tx <= tb; ++tx) {
        ++ntiles;
        if (tc) atomicAdd(&tc[ty * a.c.ntx + tx], 1u);
      }
    }
    if (a.rec_keys) a.rec_keys[idx] = ntiles;
  }
}

// ------------------------------------------------------------ validation
__global__ void validate_kernel(GaussArgs g, int32_t* bad) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= g.n) return;
  bool ok = true;
  for (int a = 0; a < 3; ++a) ok &= isfinite(g.means[3 * i + a]) && isfinite(g.log_scales[3 * i + a]);
  float qq = 0.f;
  for (int a = 0; a < 4; ++a) {
    const float q = g.quats[4 * i + a];
    ok &= isfinite(q);
    qq += q * q;
  }
  ok &= qq > 0.f;
  const float o = g.opac[i];
  ok &= (o >= 0.f && o <= 1.f);
  const int K = (g.sh_degree + 1) * (g.sh_degree + 1);
  for (int k = 0; k < 3 * K; ++k) ok &= isfinite(g.sh[static_cast<int64_t>(3 * K) * i + k]);
  // bfloat16 features: an all-ones exponent is Inf or NaN
  for (int k = 0; k < g.feat_dim; ++k) ok &= (g.feat[static_cast<int64_t>(g.feat_dim) * i + k] & 0x7f80u) != 0x7f80u;
  if (!ok) atomicOr(bad, 1);
}

// ------------------------------------------------------------ launchers
void launch_partition_bounds(const GaussArgs& g, float* bounds, hipStream_t s) {
  hipLaunchKernelGGL(partition_bounds_kernel, dim3(g.n_parts), dim3(256), 0, s, g, bounds);
}

void launch_partition_cull(const float* poses, int P, const float* bounds, int n_parts, const CamArgs& c,
                           uint64_t* vis, hipStream_t s) {
  const float margin = 8.f + 0.05f * static_cast<float>(c.W > c.H ? c.W : c.H);
  hipLaunchKernelGGL(partition_cull_kernel, dim3(P), dim3(64), 0, s, poses, P, bounds, n_parts, c, margin, vis);
}

template <int G>
static void launch_project_g(const ProjectArgs& a, hipStream_t s) {
  const dim3 grid(static_cast<unsigned>((a.g.n + 256 * G - 1) / (256 * G)));
  switch (a.g.sh_degree) {
    case 0: hipLaunchKernelGGL((project_dense_kernel<0, G>), grid, dim3(256), 0, s, a); break;
    case 1: hipLaunchKernelGGL((project_dense_kernel<1, G>), grid, dim3(256), 0, s, a); break;
    case 2: hipLaunchKernelGGL((project_dense_kernel<2, G>), grid, dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL((project_dense_kernel<3, G>), grid, dim3(256), 0, s, a); break;
  }
}

void launch_project(const ProjectArgs& a, int group, hipStream_t s) {
  if (group == 1) launch_project_g<1>(a, s);
  else launch_project_g<4>(a, s);
}

void launch_cull(const ProjectArgs& a, hipStream_t s) {
  const dim3 grid(static_cast<unsigned>((a.g.n + 255) / 256));
  hipLaunchKernelGGL(cull_kernel, grid, dim3(256), 0, s, a);
}

void launch_splat(const ProjectArgs& a, int P_total, hipStream_t s) {
  const int64_t chunks = (a.rec_cap / kSub + kSplatBlock - 1) / kSplatBlock;
  const dim3 grid(static_cast<unsigned>(static_cast<int64_t>(P_total) * kSub * chunks));
  const dim3 block(kSplatBlock);
  switch (a.g.sh_degree) {
    case 0: hipLaunchKernelGGL(splat_kernel<0>, grid, block, 0, s, a); break;
    case 1: hipLaunchKernelGGL(splat_kernel<1>, grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL(splat_kernel<2>, grid, block, 0, s, a); break;
    default: hipLaunchKernelGGL(splat_kernel<3>, grid, block, 0, s, a); break;
  }
}

void launch_validate(const GaussArgs& g, int32_t* bad, hipStream_t s) {
  hipLaunchKernelGGL(validate_kernel, dim3(static_cast<unsigned>((g.n + 255) / 256)), dim3(256), 0, s, g, bad);
}

}  // namespace hgsr
