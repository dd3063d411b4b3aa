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
      const float* T = a.poses + 12 * p;
      float mc[3];
      to_camera(T, mu, mc);
      // (U, V) = K (X / Z): the projected mean, as the renderer places it
      const float U = fmaf(a.c.fx, mc[0] / mc[2], a.c.cx);
      const float V = fmaf(a.c.fy, mc[1] / mc[2], a.c.cy);
      const bool inside =
          U >= 0.f && U < static_cast<float>(a.c.W) && V >= 0.f && V < static_cast<float>(a.c.H);
      if (!inside) continue;
      inside_mask |= 1u << k;
      const int cx = min(static_cast<int>(floorf(U * sx)), a.map_w - 1);
      const int cy = min(static_cast<int>(floorf(V * sy)), a.map_h - 1);
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

void launch_score_final(const float* sum, const uint32_t* count, int64_t n, float* score, hipStream_t s) {
  if (n <= 0) return;
  int64_t b = (n + 255) / 256;
  if (b > 8192) b = 8192;
  hipLaunchKernelGGL(score_final_kernel, dim3(static_cast<unsigned>(b)), dim3(256), 0, s, sum, count, n, score);
}

}  // namespace hgsr
