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
// centre, pushed out by a margin of `margin` pixels).
__global__ void partition_cull_kernel(const float* poses, int P, const float* bounds, int n_parts, CamArgs c,
                                      float margin, uint64_t* vis) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const float* T = poses + 12 * p;
  const float l = (-margin - c.cx) / c.fx, r = (c.W + margin - c.cx) / c.fx;
  const float t = (-margin - c.cy) / c.fy, b = (c.H + margin - c.cy) / c.fy;
  uint64_t mask = 0;
  for (int k = 0; k < n_parts; ++k) {
    const float* B = bounds + 6 * k;
    if (!(B[0] <= B[3] && B[1] <= B[4] && B[2] <= B[5])) continue;  // empty box (or NaN): nothing to draw
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
    if (!(all_near || all_l || all_r || all_t || all_b)) mask |= (1ull << k);
  }
  vis[p] = mask;
}

// ------------------------------------------------------------ projection
// Few poses: one fused pass.  One thread per Gaussian, looping over the
// launch's poses (the Gaussian's parameters are read once for all poses).
// Visible (pose, Gaussian) pairs are compacted per pose: phase 1 counts them
// per block in LDS, one global atomic per (block, pose) reserves a range of
// that pose's record segment, phase 2 recomputes the footprint and writes the
// records.  With many poses the lanes of a wave rarely share a visible pose,
// so the expensive footprint runs on a few lanes per wave; the two passes
// below (cull, then one thread per candidate) keep those lanes dense.
template <int DEG>
__global__ __launch_bounds__(256) void project_kernel(ProjectArgs a) {
  __shared__ uint32_t s_cnt[kMaxPoses];
  __shared__ uint32_t s_base[kMaxPoses];
  const int tid = threadIdx.x;
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + tid;
  for (int p = tid; p < a.P; p += 256) s_cnt[p] = 0;

  bool live = i < a.g.n;
  float mu[3] = {0.f, 0.f, 0.f}, S[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, o = 0.f, k2 = 0.f;
  float ls[3] = {0.f, 0.f, 0.f}, s2max = 0.f;
  bool have_cov = false;  // the covariance is formed for the first pose that may see the Gaussian
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
    ls[0] = a.g.log_scales[3 * i];
    ls[1] = a.g.log_scales[3 * i + 1];
    ls[2] = a.g.log_scales[3 * i + 2];
    s2max = __expf(2.f * fmaxf(ls[0], fmaxf(ls[1], ls[2])));
    k2 = 2.f * __logf(255.f * o);
  }
  __syncthreads();

  // phase 1: count visible poses per block; vis_mask keeps the result for
  // phase 2
  uint64_t vis_mask = 0;
  if (live) {
    for (int p = 0; p < a.P; ++p) {
      if (!((pose_ok >> p) & 1ull)) continue;
      const float* T = a.poses + 12 * (a.pose_base + p);
      float mc[3];
      to_camera(T, mu, mc);
      if (!(mc[2] > a.c.near_z)) continue;
      if (!maybe_visible(mc, s2max, k2, a.c)) continue;
      if (!have_cov) {
        cov3_from(reinterpret_cast<const float4*>(a.g.quats)[i], ls, S);
        have_cov = true;
      }
      Footprint f;
      if (footprint(T, mc, S, k2, a.c, f)) {
        atomicAdd(&s_cnt[p], 1u);
        vis_mask |= 1ull << p;
      }
    }
  }
  __syncthreads();
  // each block reserves its slots from one of kSub counters per pose, so the
  // blocks' atomics spread over kSub addresses instead of one
  const int sub = static_cast<int>(blockIdx.x % kSub);
  const uint32_t sub_cap = a.rec_cap / kSub;
  for (int p = tid; p < a.P; p += 256) {
    const uint32_t cnt = s_cnt[p];
    s_base[p] = cnt ? atomicAdd(&a.pose_count[(a.pose_base + p) * kSub + sub], cnt) : 0u;
    s_cnt[p] = 0;
  }
  __syncthreads();

  // phase 2: write records (footprints recomputed, same inputs and
  // arithmetic as phase 1)
  if (!vis_mask) return;
  for (int p = 0; p < a.P; ++p) {
    if (!((vis_mask >> p) & 1ull)) continue;
    const int pg = a.pose_base + p;
    const float* T = a.poses + 12 * pg;
    float mc[3];
    to_camera(T, mu, mc);
    Footprint f;
    footprint(T, mc, S, k2, a.c, f);
    const uint32_t local = s_base[p] + atomicAdd(&s_cnt[p], 1u);
    if (local >= sub_cap) {
      atomicOr(a.flags, 1);
      continue;
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
  __syncthreads();
  uint64_t cand = 0;
  if (live) {
    for (int p = 0; p < a.P; ++p) {
      if (!((pose_ok >> p) & 1ull)) continue;
      const float* T = a.poses + 12 * (a.pose_base + p);
      float mc[3];
      to_camera(T, mu, mc);
      if (!(mc[2] > a.c.near_z)) continue;
      if (!maybe_visible(mc, s2max, k2, a.c)) continue;
      atomicAdd(&s_cnt[p], 1u);
      cand |= 1ull << p;
    }
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
  while (cand) {
    const int p = __builtin_ctzll(cand);
    cand &= cand - 1ull;
    const uint32_t local = s_base[p] + atomicAdd(&s_cnt[p], 1u);
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
  __syncthreads();
  uint32_t local = 0;
  if (vis) local = atomicAdd(&s_cnt, 1u);
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
  if (!ok) atomicOr(bad, 1);
}

// ------------------------------------------------------------ launchers
void launch_partition_bounds(const GaussArgs& g, float* bounds, hipStream_t s) {
  hipLaunchKernelGGL(partition_bounds_kernel, dim3(g.n_parts), dim3(256), 0, s, g, bounds);
}

void launch_partition_cull(const float* poses, int P, const float* bounds, int n_parts, const CamArgs& c,
                           uint64_t* vis, hipStream_t s) {
  const float margin = 8.f + 0.05f * static_cast<float>(c.W > c.H ? c.W : c.H);
  hipLaunchKernelGGL(partition_cull_kernel, dim3((P + 63) / 64), dim3(64), 0, s, poses, P, bounds, n_parts, c,
                     margin, vis);
}

void launch_project(const ProjectArgs& a, hipStream_t s) {
  const dim3 grid(static_cast<unsigned>((a.g.n + 255) / 256));
  switch (a.g.sh_degree) {
    case 0: hipLaunchKernelGGL(project_kernel<0>, grid, dim3(256), 0, s, a); break;
    case 1: hipLaunchKernelGGL(project_kernel<1>, grid, dim3(256), 0, s, a); break;
    case 2: hipLaunchKernelGGL(project_kernel<2>, grid, dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL(project_kernel<3>, grid, dim3(256), 0, s, a); break;
  }
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
