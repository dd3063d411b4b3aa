// Significance scoring of Gaussians against training views (Sec. 3.2).
//
// Visibility (the render-mask algorithm of Sec. 3.2): a Gaussian is visible
// in a view when the rendered RGB gives its mean a gradient, i.e. when it is
// blended with weight alpha T > 0 at one pixel at least, and its projected
// mean lies inside the image.  contrib_kernel walks the view's tile lists
// with the blend's own per-pixel decisions (the same pair arithmetic, gate,
// clamp and stop, in the same order) but accumulates nothing and writes no
// image: it marks vis[gid * vis_stride + view] for every Gaussian it blends
// (Gaussian-major, so that the scoring pass reads one Gaussian's flags for
// all views as a few 16-byte loads).
//
// Planar maps (D planes of the map per view) are scored by map region
// instead: each (view, Gaussian) pair reads one sector per channel, planes
// megabytes apart, so score_bin_kernel bins the pairs by (view, region of
// kScoreRegionW x kScoreRegionH cells), score_region_kernel stages in LDS the 32-byte row segments of a region's
// planes that its pairs read and scores the pairs from there, and
// score_reduce_kernel sums each Gaussian's cosines in view order -- the same
// per-pair arithmetic and the same order as score_kernel, so the results are
// bit for bit those of the interleaved path.
//
// Scoring (Eq. 4-6): score_kernel takes one Gaussian per thread and visits,
// in view order, only the views in which it was blended: it projects the mean,
// tests it against the image, reads the 2D feature map at the cell that
// contains it and adds the cosine with the Gaussian's feature to its sum
// (Eq. 5) and 1 to its count.  One thread owns each Gaussian, so the sums
// need no atomics and do not depend on scheduling.  score_final_kernel
// divides (Eq. 6).
#include "hgsr_device.hpp"
#include "launch.hpp"

namespace hgsr {

template <int TILE>
__global__ __launch_bounds__(BlendShape<TILE>::kThreads) void contrib_kernel(ContribArgs a) {
  using S = BlendShape<TILE>;
  constexpr int NT = S::kThreads, NB = S::kBatch, NW = S::kWaves, BW = S::kBlockW, PPT = S::kPPT;
  __shared__ float4 s_geo[NB];
  __shared__ float4 s_opz[NB];
  __shared__ float s_pmin[NB];
  __shared__ uint8_t s_mask[NB];
  __shared__ uint16_t s_list[NW][NB];
  if (a.flags[0] & 3) return;
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1), wave = tid >> 6;
  const int W = a.c.W, H = a.c.H;
  const int item = xcd_item(blockIdx.x, gridDim.x);
  const int pose = item / a.c.tiles_per_pose;
  const int tile = item - pose * a.c.tiles_per_pose;
  const int ty = tile / a.c.ntx, tx = tile - ty * a.c.ntx;
  const uint2 range = a.ranges[item];
  const int bx0 = tx * TILE + (wave % S::kBlocksX) * BW, by0 = ty * TILE + (wave / S::kBlocksX) * S::kBlockH;
  float pxf[PPT], pyf[PPT], T[PPT];
  bool done[PPT];
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int li = lane + k * kWave;
    const int px = bx0 + (li % BW), py = by0 + (li / BW);
    pxf[k] = static_cast<float>(px) + 0.5f;
    pyf[k] = static_cast<float>(py) + 0.5f;
    T[k] = 1.f;
    done[k] = !(px < W && py < H);
  }
  // flags are Gaussian-major: vis[gid * vis_stride + pose]
  uint8_t* vis = a.vis + pose;

  for (uint32_t b0 = range.x; b0 < range.y; b0 += NB) {
    bool all_mine = true;
#pragma unroll
    for (int k = 0; k < PPT; ++k) all_mine &= done[k];
    if (__syncthreads_and(all_mine)) break;
    if (tid < NB) {
      const uint32_t j = b0 + tid;
      if (j < range.y) {
        const uint32_t lv = a.list[j];
        const float4* sp = reinterpret_cast<const float4*>(a.recs + (lv & kRecMask));
        s_geo[tid] = sp[0];
        s_opz[tid] = sp[1];
        s_pmin[tid] = sp[2].w;
        s_mask[tid] = static_cast<uint8_t>(lv >> kRecBits);
      } else {
        s_mask[tid] = 0;
      }
    }
    __syncthreads();
    const int nb = static_cast<int>(min(static_cast<uint32_t>(NB), range.y - b0));
    int n_mine = 0;
    for (int c0 = 0; c0 < nb; c0 += kWave) {
      const int ce = c0 + lane;
      const bool hit = ce < nb && ((s_mask[ce] >> wave) & 1u);
      const uint64_t bal = __ballot(hit);
      if (hit) s_list[wave][n_mine + __popcll(bal & ((1ull << lane) - 1ull))] = static_cast<uint16_t>(ce);
      n_mine += __popcll(bal);
    }
    __builtin_amdgcn_wave_barrier();
    for (int ii = 0; ii < n_mine; ++ii) {
      bool mine = true;
#pragma unroll
      for (int k = 0; k < PPT; ++k) mine &= done[k];
      if (mine) break;
      const int jj = s_list[wave][ii];
      const float4 geo = s_geo[jj];
      const float4 opz = s_opz[jj];
      const float pmin = s_pmin[jj];
      bool blended = false;
#pragma unroll
      for (int k = 0; k < PPT; ++k) {
        if (done[k]) continue;
        const float dx = pxf[k] - geo.x, dy = pyf[k] - geo.y;
        const float power = pair_power(dx, dy, geo.z, geo.w, opz.x);
        if (power > 0.f || power < pmin - kPreReject) continue;
        const float alpha = pair_alpha(opz.y, power);
        if (alpha < kAlphaMin) continue;
        const float Tn = T[k] * (1.f - alpha);
        if (Tn < kTMin) {
          done[k] = true;
          continue;
        }
        T[k] = Tn;
        blended = true;
      }
      // every lane that blended the splat stores the same byte
      if (blended) vis[static_cast<int64_t>(__float_as_uint(opz.w)) * a.vis_stride] = 1;
    }
  }
}

// The map cell that the projected mean of a Gaussian falls in for view p:
// (U, V) = K (X / Z), placed as the renderer places it, scaled to the map's
// resolution.  False when the mean projects outside the image (no cosine).
__device__ __forceinline__ bool mean_cell(const ScoreArgs& a, const float* mu, int p, float sx, float sy, int& cx,
                                          int& cy) {
  const float* T = a.poses + 12 * p;
  float mc[3];
  to_camera(T, mu, mc);
  const float U = fmaf(a.c.fx, mc[0] / mc[2], a.c.cx);
  const float V = fmaf(a.c.fy, mc[1] / mc[2], a.c.cy);
  if (!(U >= 0.f && U < static_cast<float>(a.c.W) && V >= 0.f && V < static_cast<float>(a.c.H))) return false;
  cx = min(static_cast<int>(floorf(U * sx)), a.map_w - 1);
  cy = min(static_cast<int>(floorf(V * sy)), a.map_h - 1);
  return true;
}

template <int D, bool INTERLEAVED>
__global__ __launch_bounds__(256) void score_kernel(ScoreArgs a) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (a.flags[0] & 3) return;
  if (j >= a.n) return;
  const float mu[3] = {a.means[3 * j], a.means[3 * j + 1], a.means[3 * j + 2]};
  float f[D];
  {
    const uint4* fv = reinterpret_cast<const uint4*>(a.feat + j * D);
#pragma unroll
    for (int q = 0; q < D / 8; ++q) {
      const uint4 w = fv[q];
      f[8 * q + 0] = bf16_lo(w.x); f[8 * q + 1] = bf16_hi(w.x);
      f[8 * q + 2] = bf16_lo(w.y); f[8 * q + 3] = bf16_hi(w.y);
      f[8 * q + 4] = bf16_lo(w.z); f[8 * q + 5] = bf16_hi(w.z);
      f[8 * q + 6] = bf16_lo(w.w); f[8 * q + 7] = bf16_hi(w.w);
    }
  }
  float ff = 0.f;
#pragma unroll
  for (int d = 0; d < D; ++d) ff = fmaf(f[d], f[d], ff);
  const float nf = sqrtf(ff);
  float sum = a.score_sum[j];
  uint32_t cnt = a.vis_count[j];
  const float sx = static_cast<float>(a.map_w) / static_cast<float>(a.c.W);
  const float sy = static_cast<float>(a.map_h) / static_cast<float>(a.c.H);
  const int64_t cells = static_cast<int64_t>(a.map_w) * a.map_h;
  const uint8_t* vrow = a.vis + j * a.vis_stride;
  for (int p0 = 0; p0 < a.P; p0 += 16) {
    // blended flags (0 or 1 per byte) of views p0 .. p0 + 15 as a bit mask
    const uint4 w = *reinterpret_cast<const uint4*>(vrow + p0);
    uint32_t todo = 0;
    const uint32_t wd[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint32_t x = wd[q];
      todo |= ((x & 1u) | ((x >> 7) & 2u) | ((x >> 14) & 4u) | ((x >> 21) & 8u)) << (4 * q);
    }
    uint32_t inside_mask = 0;
    while (todo) {
      const int k = __builtin_ctz(todo);
      todo &= todo - 1u;
      const int p = p0 + k;
      int cx, cy;
      if (!mean_cell(a, mu, p, sx, sy, cx, cy)) continue;
      inside_mask |= 1u << k;
      const int64_t cell = static_cast<int64_t>(cy) * a.map_w + cx;
      float dot = 0.f, tt = 0.f;
      if constexpr (INTERLEAVED) {
        const float4* m = reinterpret_cast<const float4*>(a.maps + (static_cast<int64_t>(p) * cells + cell) * D);
#pragma unroll
        for (int q = 0; q < D / 4; ++q) {
          const float4 t = m[q];
          dot = fmaf(f[4 * q + 0], t.x, dot); tt = fmaf(t.x, t.x, tt);
          dot = fmaf(f[4 * q + 1], t.y, dot); tt = fmaf(t.y, t.y, tt);
          dot = fmaf(f[4 * q + 2], t.z, dot); tt = fmaf(t.z, t.z, tt);
          dot = fmaf(f[4 * q + 3], t.w, dot); tt = fmaf(t.w, t.w, tt);
        }
      } else {
        const float* m = a.maps + static_cast<int64_t>(p) * D * cells + cell;
#pragma unroll
        for (int d = 0; d < D; ++d) {
          const float t = m[d * cells];
          dot = fmaf(f[d], t, dot);
          tt = fmaf(t, t, tt);
        }
      }
      sum += dot / fmaf(nf, sqrtf(tt), kCosEps);
      ++cnt;
    }
    if (a.visible) {
      const int np = min(16, a.P - p0);
      for (int k = 0; k < np; ++k)
        a.visible[static_cast<int64_t>(p0 + k) * a.n + j] = static_cast<uint8_t>((inside_mask >> k) & 1u);
    }
  }
  a.score_sum[j] = sum;
  a.vis_count[j] = cnt;
}

// A visible pair whose projected mean lies outside the image: no cosine.
constexpr uint32_t kNoCosine = 0xffffffffu;

// Binning of the (view, Gaussian) pairs that score_kernel visits by map
// region, one Gaussian per thread, in view order.  Pass 0 counts the pairs of
// each region and marks the pairs whose mean projects outside the image; pass
// 1 writes (Gaussian, cell in region) into the region's range.  (A visible
// Gaussian is blended in about two of the views on average, so the lanes of a
// wave rarely share a view and region: one atomic per pair, all lanes' in
// flight together, is the fast form.)
template <int PASS>
__global__ __launch_bounds__(256) void score_bin_kernel(ScoreArgs a) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (a.flags[0] & 3) return;
  if (j >= a.n) return;
  const float mu[3] = {a.means[3 * j], a.means[3 * j + 1], a.means[3 * j + 2]};
  const float sx = static_cast<float>(a.map_w) / static_cast<float>(a.c.W);
  const float sy = static_cast<float>(a.map_h) / static_cast<float>(a.c.H);
  const uint32_t regions = static_cast<uint32_t>(a.n_rx) * static_cast<uint32_t>(a.n_ry);
  const uint8_t* vrow = a.vis + j * a.vis_stride;
  for (int p0 = 0; p0 < a.P; p0 += 16) {
    const uint4 w = *reinterpret_cast<const uint4*>(vrow + p0);
    uint32_t todo = 0;
    const uint32_t wd[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint32_t x = wd[q];
      todo |= ((x & 1u) | ((x >> 7) & 2u) | ((x >> 14) & 4u) | ((x >> 21) & 8u)) << (4 * q);
    }
    while (todo) {
      const int k = __builtin_ctz(todo);
      todo &= todo - 1u;
      const int p = p0 + k;
      int cx, cy;
      if (!mean_cell(a, mu, p, sx, sy, cx, cy)) {
        if constexpr (PASS == 0) a.cosb[j * a.vis_stride + p] = __uint_as_float(kNoCosine);
        continue;
      }
      const uint32_t r = static_cast<uint32_t>(p) * regions +
                         static_cast<uint32_t>(cy / kScoreRegionH) * a.n_rx + static_cast<uint32_t>(cx / kScoreRegionW);
      const uint32_t cell = static_cast<uint32_t>((cy % kScoreRegionH) * kScoreRegionW + cx % kScoreRegionW);
      if constexpr (PASS == 0) {
        atomicAdd(&a.rcount[r], 1u);
      } else {
        const uint32_t pos = a.rranges[r].x + atomicAdd(&a.rcursor[r], 1u);
        a.pairs[pos] = make_uint2(static_cast<uint32_t>(j), cell);
      }
    }
  }
}

// Eq. 4 for one pair: the cosine of the Gaussian's feature vector (packed
// bf16 pairs, norm nf) with the map vector at `cell` of the staged planes
// (plane stride RC floats), summed in channel order as score_kernel does.
template <int D, int RC>
__device__ __forceinline__ float region_cosine(const uint4 (&fw)[D / 8], const float* s_m, uint32_t cell) {
  float f[D];
#pragma unroll
  for (int qq = 0; qq < D / 8; ++qq) {
    const uint4 w = fw[qq];
    f[8 * qq + 0] = bf16_lo(w.x); f[8 * qq + 1] = bf16_hi(w.x);
    f[8 * qq + 2] = bf16_lo(w.y); f[8 * qq + 3] = bf16_hi(w.y);
    f[8 * qq + 4] = bf16_lo(w.z); f[8 * qq + 5] = bf16_hi(w.z);
    f[8 * qq + 6] = bf16_lo(w.w); f[8 * qq + 7] = bf16_hi(w.w);
  }
  float ff = 0.f;
#pragma unroll
  for (int d = 0; d < D; ++d) ff = fmaf(f[d], f[d], ff);
  const float nf = sqrtf(ff);
  float dot = 0.f, tt = 0.f;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const float t = s_m[d * RC + cell];
    dot = fmaf(f[d], t, dot);
    tt = fmaf(t, t, tt);
  }
  return dot / fmaf(nf, sqrtf(tt), kCosEps);
}

template <int D>
__global__ __launch_bounds__(256) void score_region_kernel(ScoreArgs a) {
  constexpr int RC = kScoreRegionW * kScoreRegionH;  // cells per region
  __shared__ float4 s_m4[D * RC / 4];
  float* s_m = reinterpret_cast<float*>(s_m4);
  if (a.flags[0] & 3) return;
  const int64_t r = blockIdx.x;
  const uint2 range = a.rranges[r];
  if (range.x == range.y) return;  // no pair: the region's planes are never read
  const int64_t regions = static_cast<int64_t>(a.n_rx) * a.n_ry;
  const int p = static_cast<int>(r / regions);
  const int rr = static_cast<int>(r - static_cast<int64_t>(p) * regions);
  const int y0 = (rr / a.n_rx) * kScoreRegionH, x0 = (rr % a.n_rx) * kScoreRegionW;
  const int64_t cells = static_cast<int64_t>(a.map_w) * a.map_h;
  const float* mp = a.maps + static_cast<int64_t>(p) * D * cells;
  // The thread's first pair and its feature vector, in flight while the
  // planes are staged (a region holds a few pairs on average, rarely more than
  // one per thread).
  const uint32_t q0 = range.x + threadIdx.x;
  const bool first = q0 < range.y;
  uint2 pr0 = make_uint2(0u, 0u);
  uint4 fw0[D / 8];
  if (first) {
    pr0 = a.pairs[q0];
    const uint4* fv = reinterpret_cast<const uint4*>(a.feat + static_cast<int64_t>(pr0.x) * D);
#pragma unroll
    for (int qq = 0; qq < D / 8; ++qq) fw0[qq] = fv[qq];
  }
  // The row segments that some pair of the region reads, bit (row *
  // kScoreRegionW + col) / kScoreSegCells, gathered in the first word of the
  // staging buffer (overwritten by the planes once every thread has read it:
  // a sixth of LDS per workgroup keeps five workgroups on a CU).
  uint32_t* s_seg = reinterpret_cast<uint32_t*>(s_m4);
  if (threadIdx.x == 0) *s_seg = 0u;
  __syncthreads();
  {
    uint32_t used = first ? 1u << (pr0.y / kScoreSegCells) : 0u;
    for (uint32_t q = q0 + 256; q < range.y; q += 256) used |= 1u << (a.pairs[q].y / kScoreSegCells);
    // OR over the wave first: one LDS atomic per wave, not one per lane on
    // the same word (those are performed one lane after another)
    for (int off = kWave / 2; off > 0; off >>= 1) used |= __shfl_xor(used, off, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0 && used) atomicOr(s_seg, used);
  }
  __syncthreads();
  const uint32_t seg = *s_seg;
  // D planes x kScoreRegionH rows of kScoreRegionW cells, as 16-byte pieces of
  // the used segments: consecutive threads read consecutive pieces of a row,
  // all of a thread's pieces in flight at once; pieces that are not 16-byte
  // aligned or run past the map's edge are read cell by cell.  Cells of unused
  // segments and past the edge are not read: no pair refers to them.
  constexpr int RW4 = kScoreRegionW / 4;
  constexpr int NPIECE = D * RC / 4;
  constexpr int PER = (NPIECE + 255) / 256;
  const bool vec_rows = (a.map_w & 3) == 0;
  float4 v[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int e4 = threadIdx.x + k * 256;
    v[k] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (e4 < NPIECE) {
      const int d = e4 / (RC / 4), rc4 = e4 - d * (RC / 4);
      const int gy = y0 + rc4 / RW4, gx = x0 + 4 * (rc4 % RW4);
      const float* src = mp + d * cells + static_cast<int64_t>(gy) * a.map_w + gx;
      if (((seg >> (4 * rc4 / kScoreSegCells)) & 1u) && gy < a.map_h) {
        if (vec_rows && gx + 3 < a.map_w) {
          v[k] = *reinterpret_cast<const float4*>(src);
        } else {
          if (gx < a.map_w) v[k].x = src[0];
          if (gx + 1 < a.map_w) v[k].y = src[1];
          if (gx + 2 < a.map_w) v[k].z = src[2];
          if (gx + 3 < a.map_w) v[k].w = src[3];
        }
      }
    }
  }
  __syncthreads();  // every thread holds seg before the planes overwrite it
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int e4 = threadIdx.x + k * 256;
    if (e4 < NPIECE) s_m4[e4] = v[k];
  }
  __syncthreads();
  if (!first) return;
  a.cosb[static_cast<int64_t>(pr0.x) * a.vis_stride + p] = region_cosine<D, RC>(fw0, s_m, pr0.y);
  for (uint32_t q = q0 + 256; q < range.y; q += 256) {
    const uint2 pr = a.pairs[q];
    uint4 fw[D / 8];
    const uint4* fv = reinterpret_cast<const uint4*>(a.feat + static_cast<int64_t>(pr.x) * D);
#pragma unroll
    for (int qq = 0; qq < D / 8; ++qq) fw[qq] = fv[qq];
    a.cosb[static_cast<int64_t>(pr.x) * a.vis_stride + p] = region_cosine<D, RC>(fw, s_m, pr.y);
  }
}

__global__ __launch_bounds__(256) void score_reduce_kernel(ScoreArgs a) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (a.flags[0] & 3) return;
  if (j >= a.n) return;
  float sum = a.score_sum[j];
  uint32_t cnt = a.vis_count[j];
  const uint8_t* vrow = a.vis + j * a.vis_stride;
  const float* crow = a.cosb + j * a.vis_stride;
  for (int p0 = 0; p0 < a.P; p0 += 16) {
    const uint4 w = *reinterpret_cast<const uint4*>(vrow + p0);
    uint32_t todo = 0;
    const uint32_t wd[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint32_t x = wd[q];
      todo |= ((x & 1u) | ((x >> 7) & 2u) | ((x >> 14) & 4u) | ((x >> 21) & 8u)) << (4 * q);
    }
    uint32_t inside_mask = 0;
    while (todo) {
      const int k = __builtin_ctz(todo);
      todo &= todo - 1u;
      const float v = crow[p0 + k];
      if (__float_as_uint(v) == kNoCosine) continue;
      inside_mask |= 1u << k;
      sum += v;
      ++cnt;
    }
    if (a.visible) {
      const int np = min(16, a.P - p0);
      for (int k = 0; k < np; ++k)
        a.visible[static_cast<int64_t>(p0 + k) * a.n + j] = static_cast<uint8_t>((inside_mask >> k) & 1u);
    }
  }
  a.score_sum[j] = sum;
  a.vis_count[j] = cnt;
}

__global__ void score_final_kernel(const float* sum, const uint32_t* count, int64_t n, float* score) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const uint32_t c = count[i];
    score[i] = c ? sum[i] / static_cast<float>(c) : 0.f;
  }
}

void launch_contrib(const ContribArgs& a, int n_items, hipStream_t s) {
  if (n_items <= 0) return;
  switch (a.c.tile) {
    case 8: hipLaunchKernelGGL(contrib_kernel<8>, dim3(n_items), dim3(BlendShape<8>::kThreads), 0, s, a); break;
    case 32: hipLaunchKernelGGL(contrib_kernel<32>, dim3(n_items), dim3(BlendShape<32>::kThreads), 0, s, a); break;
    default: hipLaunchKernelGGL(contrib_kernel<16>, dim3(n_items), dim3(BlendShape<16>::kThreads), 0, s, a); break;
  }
}

template <int D>
static void launch_score_d(const ScoreArgs& a, hipStream_t s) {
  const dim3 grid(static_cast<unsigned>((a.n + 255) / 256));
  if (a.map_layout == 1) hipLaunchKernelGGL((score_kernel<D, true>), grid, dim3(256), 0, s, a);
  else hipLaunchKernelGGL((score_kernel<D, false>), grid, dim3(256), 0, s, a);
}

void launch_score(const ScoreArgs& a, hipStream_t s) {
  if (a.n <= 0) return;
  switch (a.D) {
    case 8: launch_score_d<8>(a, s); break;
    case 16: launch_score_d<16>(a, s); break;
    case 32: launch_score_d<32>(a, s); break;
    default: launch_score_d<64>(a, s); break;
  }
}

void launch_score_bin(const ScoreArgs& a, int pass, hipStream_t s) {
  if (a.n <= 0) return;
  const dim3 grid(static_cast<unsigned>((a.n + 255) / 256));
  if (pass == 0) hipLaunchKernelGGL(score_bin_kernel<0>, grid, dim3(256), 0, s, a);
  else hipLaunchKernelGGL(score_bin_kernel<1>, grid, dim3(256), 0, s, a);
}

void launch_score_regions(const ScoreArgs& a, hipStream_t s) {
  const int64_t nreg = static_cast<int64_t>(a.P) * a.n_rx * a.n_ry;
  if (nreg <= 0 || a.n <= 0) return;
  const dim3 grid(static_cast<unsigned>(nreg));
  switch (a.D) {
    case 8: hipLaunchKernelGGL(score_region_kernel<8>, grid, dim3(256), 0, s, a); break;
    case 16: hipLaunchKernelGGL(score_region_kernel<16>, grid, dim3(256), 0, s, a); break;
    case 32: hipLaunchKernelGGL(score_region_kernel<32>, grid, dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL(score_region_kernel<64>, grid, dim3(256), 0, s, a); break;
  }
}

void launch_score_reduce(const ScoreArgs& a, hipStream_t s) {
  if (a.n <= 0) return;
  hipLaunchKernelGGL(score_reduce_kernel, dim3(static_cast<unsigned>((a.n + 255) / 256)), dim3(256), 0, s, a);
}

void launch_score_final(const float* sum, const uint32_t* count, int64_t n, float* score, hipStream_t s) {
  if (n <= 0) return;
  int64_t b = (n + 255) / 256;
  if (b > 8192) b = 8192;
  hipLaunchKernelGGL(score_final_kernel, dim3(static_cast<unsigned>(b)), dim3(256), 0, s, sum, count, n, score);
}

}  // namespace hgsr
