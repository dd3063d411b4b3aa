// Front-to-back alpha blend, one workgroup per (pose, tile).
//
// Each workgroup walks its tile's depth-ordered list in batches: every thread
// stages one splat (geometry, colour and bf16 feature vector) into LDS, then
// every thread runs its pixel(s) through the whole batch, reading each splat
// as an LDS broadcast.  A pixel stops at the first splat that would take its
// transmittance below 1e-4; the batch loop ends as soon as every pixel of the
// tile has stopped (__syncthreads_and).  Colour, depth and the D feature
// channels accumulate in FP32 registers.  Outputs are planar per pose, so a
// wave's stores of one channel are contiguous row segments.
#include "hgsr_device.hpp"
#include "launch.hpp"

namespace hgsr {

template <int TILE>
struct BlendShape {
  static constexpr int kThreads = TILE == 8 ? 64 : 256;
  static constexpr int kPPT = TILE * TILE / kThreads;  // pixels per thread
};

template <int TILE, int D, bool BF16>
__global__ __launch_bounds__(BlendShape<TILE>::kThreads) void blend_fwd_kernel(BlendArgs a) {
  constexpr int NT = BlendShape<TILE>::kThreads;
  constexpr int PPT = BlendShape<TILE>::kPPT;
  constexpr int DV = D / 8;  // 16-byte vectors per feature
  __shared__ float4 s_geo[NT];
  __shared__ float4 s_opz[NT];
  __shared__ float4 s_col[NT];
  __shared__ uint4 s_feat[DV > 0 ? NT * DV : 1];
  __shared__ int s_item;
  if (a.flags[0] & 3) return;
  const int tid = threadIdx.x;
  const int W = a.c.W, H = a.c.H;
  const int64_t HW = static_cast<int64_t>(W) * H;
  const bool persistent = a.schedule != kSchedGrid;

  for (int iter = 0;; ++iter) {
    int item;
    if (persistent) {
      if (tid == 0) s_item = static_cast<int>(atomicAdd(a.queue, 1u));
      __syncthreads();
      item = s_item;
      __syncthreads();
      if (item >= a.n_items) break;
    } else {
      if (iter > 0) break;
      item = blockIdx.x;
    }
    int pose, tile;
    if (a.schedule == kSchedTileMajor) {
      tile = item / a.P;
      pose = item - tile * a.P;
    } else {
      pose = item / a.c.tiles_per_pose;
      tile = item - pose * a.c.tiles_per_pose;
    }
    const int ty = tile / a.c.ntx, tx = tile - ty * a.c.ntx;
    const uint2 range = a.ranges[static_cast<int64_t>(pose) * a.c.tiles_per_pose + tile];

    float pxf[PPT], pyf[PPT], T[PPT], C[PPT][3], Z[PPT];
    float F[PPT][D > 0 ? D : 1];
    uint32_t used[PPT];
    bool done[PPT], inside[PPT];
    int pix[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      const int li = tid + k * NT;
      const int px = tx * TILE + (li % TILE), py = ty * TILE + (li / TILE);
      inside[k] = px < W && py < H;
      pix[k] = py * W + px;
      pxf[k] = static_cast<float>(px) + 0.5f;
      pyf[k] = static_cast<float>(py) + 0.5f;
      T[k] = 1.f;
      C[k][0] = C[k][1] = C[k][2] = 0.f;
      Z[k] = 0.f;
#pragma unroll
      for (int d = 0; d < (D > 0 ? D : 1); ++d) F[k][d] = 0.f;
      used[k] = 0;
      done[k] = !inside[k];
    }

    for (uint32_t b0 = range.x; b0 < range.y; b0 += NT) {
      bool all_mine = true;
#pragma unroll
      for (int k = 0; k < PPT; ++k) all_mine &= done[k];
      if (__syncthreads_and(all_mine)) break;
      const uint32_t j = b0 + tid;
      if (j < range.y) {
        const uint32_t r = a.list[j];
        const float4* sp = reinterpret_cast<const float4*>(a.recs + r);
        const float4 g0 = sp[0], g1 = sp[1], g2 = sp[2];
        s_geo[tid] = g0;
        s_opz[tid] = g1;
        s_col[tid] = g2;
        if constexpr (DV > 0) {
          const uint4* fv = reinterpret_cast<const uint4*>(a.feat) + static_cast<int64_t>(__float_as_uint(g1.w)) * DV;
#pragma unroll
          for (int q = 0; q < DV; ++q) s_feat[tid * DV + q] = fv[q];
        }
      }
      __syncthreads();
      const int nb = static_cast<int>(min(static_cast<uint32_t>(NT), range.y - b0));
      for (int jj = 0; jj < nb; ++jj) {
        bool mine = true;
#pragma unroll
        for (int k = 0; k < PPT; ++k) mine &= done[k];
        if (mine) break;
        const float4 geo = s_geo[jj];
        const float4 opz = s_opz[jj];
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
          if (done[k]) continue;
          const float dx = pxf[k] - geo.x, dy = pyf[k] - geo.y;
          const float power = pair_power(dx, dy, geo.z, geo.w, opz.x);
          if (power > 0.f) continue;
          const float alpha = pair_alpha(opz.y, power);
          if (alpha < kAlphaMin) continue;
          const float Tn = T[k] * (1.f - alpha);
          if (Tn < kTMin) {
            done[k] = true;
            continue;
          }
          const float w = alpha * T[k];
          const float4 col = s_col[jj];
          C[k][0] = fmaf(w, col.x, C[k][0]);
          C[k][1] = fmaf(w, col.y, C[k][1]);
          C[k][2] = fmaf(w, col.z, C[k][2]);
          Z[k] = fmaf(w, opz.z, Z[k]);
          if constexpr (DV > 0) {
#pragma unroll
            for (int q = 0; q < DV; ++q) {
              const uint4 fq = s_feat[jj * DV + q];
              F[k][8 * q + 0] = fmaf(w, bf16_lo(fq.x), F[k][8 * q + 0]);
              F[k][8 * q + 1] = fmaf(w, bf16_hi(fq.x), F[k][8 * q + 1]);
              F[k][8 * q + 2] = fmaf(w, bf16_lo(fq.y), F[k][8 * q + 2]);
              F[k][8 * q + 3] = fmaf(w, bf16_hi(fq.y), F[k][8 * q + 3]);
              F[k][8 * q + 4] = fmaf(w, bf16_lo(fq.z), F[k][8 * q + 4]);
              F[k][8 * q + 5] = fmaf(w, bf16_hi(fq.z), F[k][8 * q + 5]);
              F[k][8 * q + 6] = fmaf(w, bf16_lo(fq.w), F[k][8 * q + 6]);
              F[k][8 * q + 7] = fmaf(w, bf16_hi(fq.w), F[k][8 * q + 7]);
            }
          }
          T[k] = Tn;
          used[k] = b0 + jj - range.x + 1;
        }
      }
    }

    const int64_t pbase = static_cast<int64_t>(pose) * HW;
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      if (!inside[k]) continue;
      const int64_t o = pbase + pix[k];
      const int64_t o3 = static_cast<int64_t>(pose) * 3 * HW + pix[k];
      a.rgb[o3] = fmaf(T[k], a.bg[0], C[k][0]);
      a.rgb[o3 + HW] = fmaf(T[k], a.bg[1], C[k][1]);
      a.rgb[o3 + 2 * HW] = fmaf(T[k], a.bg[2], C[k][2]);
      const float A = 1.f - T[k];
      a.alpha[o] = A;
      a.depth[o] = A > 0.f ? Z[k] / A : 0.f;
      a.final_T[o] = T[k];
      a.n_used[o] = used[k];
      if constexpr (D > 0) {
        if (a.out_feat) {
          const int64_t of = static_cast<int64_t>(pose) * D * HW + pix[k];
          if constexpr (BF16) {
            uint16_t* fo = static_cast<uint16_t*>(a.out_feat);
#pragma unroll
            for (int d = 0; d < D; ++d) fo[of + d * HW] = f32_to_bf16_rne(F[k][d]);
          } else {
            float* fo = static_cast<float*>(a.out_feat);
#pragma unroll
            for (int d = 0; d < D; ++d) fo[of + d * HW] = F[k][d];
          }
        }
      }
    }
    if (persistent) __syncthreads();
  }
}

template <int TILE, int D, bool BF16>
static void launch_t(const BlendArgs& a, int n_ctas, hipStream_t s) {
  constexpr int NT = BlendShape<TILE>::kThreads;
  hipLaunchKernelGGL((blend_fwd_kernel<TILE, D, BF16>), dim3(n_ctas), dim3(NT), 0, s, a);
}

template <int TILE, int D>
static void launch_td(const BlendArgs& a, bool bf16, int n_ctas, hipStream_t s) {
  if (bf16) launch_t<TILE, D, true>(a, n_ctas, s);
  else launch_t<TILE, D, false>(a, n_ctas, s);
}

template <int TILE>
static void launch_tile(const BlendArgs& a, int D, bool bf16, int n_ctas, hipStream_t s) {
  switch (D) {
    case 0: launch_t<TILE, 0, false>(a, n_ctas, s); break;
    case 8: launch_td<TILE, 8>(a, bf16, n_ctas, s); break;
    case 16: launch_td<TILE, 16>(a, bf16, n_ctas, s); break;
    case 32: launch_td<TILE, 32>(a, bf16, n_ctas, s); break;
    default: launch_td<TILE, 64>(a, bf16, n_ctas, s); break;
  }
}

void launch_blend_fwd(const BlendArgs& a, int D, bool bf16_out, int n_ctas, hipStream_t s) {
  switch (a.c.tile) {
    case 8: launch_tile<8>(a, D, bf16_out, n_ctas, s); break;
    case 32: launch_tile<32>(a, D, bf16_out, n_ctas, s); break;
    default: launch_tile<16>(a, D, bf16_out, n_ctas, s); break;
  }
}

}  // namespace hgsr
