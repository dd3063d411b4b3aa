// Front-to-back alpha blend, one workgroup per (pose, tile).
//
// Each wave owns a square block of the tile (8x8 pixels at tile 8 and 16,
// 16x16 at tile 32 with 4 pixels per lane).  The workgroup walks the tile's
// depth-ordered list in batches: every thread stages one splat (geometry,
// colour, FP32 feature vector) into LDS and marks which waves' blocks its
// support rectangle touches; each wave then compacts the batch to the entries
// that touch its block and runs its pixels through them, reading each splat
// as an LDS broadcast.  Pairs whose exponent is clearly below the 1/255 gate
// are rejected before the exponential; the exact gate, clamp and stop tests
// follow.  A pixel stops at the first splat that would take its transmittance
// below 1e-4; the batch loop ends when every pixel of the tile has stopped.
// Outputs are planar per pose.
#include "hgsr_device.hpp"
#include "launch.hpp"

namespace hgsr {

template <int TILE>
struct BlendShape {
  static constexpr int kThreads = TILE == 8 ? 64 : 256;
  static constexpr int kWaves = kThreads / kWave;
  static constexpr int kBlock = TILE == 32 ? 16 : 8;       // side of a wave's pixel block
  static constexpr int kPPT = kBlock * kBlock / kWave;     // pixels per lane
  static constexpr int kBlocksX = TILE / kBlock;
};

// Pixel-centre rectangle of a splat's support, padded; shared by the wave
// culling of the forward and backward blends.
__device__ __forceinline__ void splat_rect(const float4 geo, const float4 opz, float pmin, float& x0, float& x1,
                                           float& y0, float& y1) {
  const float det = geo.z * opz.x - geo.w * geo.w;
  const float k2 = -2.f * pmin;
  const float rx = 1.001f * sqrtf(fmaxf(k2 * opz.x / det, 0.f)) + 0.05f;
  const float ry = 1.001f * sqrtf(fmaxf(k2 * geo.z / det, 0.f)) + 0.05f;
  x0 = geo.x - rx - 0.5f;
  x1 = geo.x + rx - 0.5f;
  y0 = geo.y - ry - 0.5f;
  y1 = geo.y + ry - 0.5f;
}

template <int TILE, int D, bool BF16>
__global__ __launch_bounds__(BlendShape<TILE>::kThreads) void blend_fwd_kernel(BlendArgs a) {
  using S = BlendShape<TILE>;
  constexpr int NT = S::kThreads, NW = S::kWaves, B = S::kBlock, PPT = S::kPPT;
  constexpr bool LDS_F32 = D > 0 && D <= 32;            // features as FP32 in LDS
  constexpr int FW = D == 0 ? 1 : (LDS_F32 ? D : D / 2);  // 32-bit words per feature vector
  __shared__ float4 s_geo[NT];
  __shared__ float4 s_opz[NT];
  __shared__ float4 s_col[NT];
  __shared__ uint32_t s_fw[NT * FW];
  __shared__ uint8_t s_mask[NT];
  __shared__ uint16_t s_list[NW][NT];
  __shared__ int s_item;
  if (a.flags[0] & 3) return;
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1), wave = tid >> 6;
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
    // this wave's pixel block
    const int bx0 = tx * TILE + (wave % S::kBlocksX) * B, by0 = ty * TILE + (wave / S::kBlocksX) * B;

    float pxf[PPT], pyf[PPT], T[PPT], C[PPT][3], Z[PPT];
    float F[PPT][D > 0 ? D : 1];
    uint32_t used[PPT];
    bool done[PPT], inside[PPT];
    int pix[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      const int li = lane + k * kWave;
      const int px = bx0 + (li % B), py = by0 + (li / B);
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
        float x0, x1, y0, y1;
        splat_rect(g0, g1, g2.w, x0, x1, y0, y1);
        uint8_t m = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
          const float wx0 = static_cast<float>(tx * TILE + (w % S::kBlocksX) * B);
          const float wy0 = static_cast<float>(ty * TILE + (w / S::kBlocksX) * B);
          if (x1 >= wx0 && x0 <= wx0 + (B - 1) && y1 >= wy0 && y0 <= wy0 + (B - 1)) m |= 1u << w;
        }
        s_mask[tid] = m;
        if constexpr (D > 0) {
          const uint4* fv = reinterpret_cast<const uint4*>(a.feat) + static_cast<int64_t>(__float_as_uint(g1.w)) * (D / 8);
          if constexpr (LDS_F32) {
#pragma unroll
            for (int q = 0; q < D / 8; ++q) {
              const uint4 f = fv[q];
              uint4* dst = reinterpret_cast<uint4*>(&s_fw[tid * FW + 8 * q]);
              dst[0] = make_uint4(f.x << 16, f.x & 0xffff0000u, f.y << 16, f.y & 0xffff0000u);
              dst[1] = make_uint4(f.z << 16, f.z & 0xffff0000u, f.w << 16, f.w & 0xffff0000u);
            }
          } else {
#pragma unroll
            for (int q = 0; q < D / 8; ++q) reinterpret_cast<uint4*>(&s_fw[tid * FW])[q] = fv[q];
          }
        }
      } else {
        s_mask[tid] = 0;
      }
      __syncthreads();
      const int nb = static_cast<int>(min(static_cast<uint32_t>(NT), range.y - b0));
      // compact the batch to the entries touching this wave's block (in order)
      int n_mine = 0;
      for (int c0 = 0; c0 < nb; c0 += kWave) {
        const int e = c0 + lane;
        const bool hit = e < nb && ((s_mask[e] >> wave) & 1u);
        const uint64_t bal = __ballot(hit);
        if (hit) s_list[wave][n_mine + __popcll(bal & ((1ull << lane) - 1ull))] = static_cast<uint16_t>(e);
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
        const float pmin = s_col[jj].w;
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
          const float w = alpha * T[k];
          const float4 col = s_col[jj];
          C[k][0] = fmaf(w, col.x, C[k][0]);
          C[k][1] = fmaf(w, col.y, C[k][1]);
          C[k][2] = fmaf(w, col.z, C[k][2]);
          Z[k] = fmaf(w, opz.z, Z[k]);
          if constexpr (D > 0) {
            if constexpr (LDS_F32) {
              const float4* fq = reinterpret_cast<const float4*>(&s_fw[jj * FW]);
#pragma unroll
              for (int q = 0; q < D / 4; ++q) {
                const float4 f = fq[q];
                F[k][4 * q + 0] = fmaf(w, f.x, F[k][4 * q + 0]);
                F[k][4 * q + 1] = fmaf(w, f.y, F[k][4 * q + 1]);
                F[k][4 * q + 2] = fmaf(w, f.z, F[k][4 * q + 2]);
                F[k][4 * q + 3] = fmaf(w, f.w, F[k][4 * q + 3]);
              }
            } else {
              const uint4* fq = reinterpret_cast<const uint4*>(&s_fw[jj * FW]);
#pragma unroll
              for (int q = 0; q < D / 8; ++q) {
                const uint4 f = fq[q];
                F[k][8 * q + 0] = fmaf(w, bf16_lo(f.x), F[k][8 * q + 0]);
                F[k][8 * q + 1] = fmaf(w, bf16_hi(f.x), F[k][8 * q + 1]);
                F[k][8 * q + 2] = fmaf(w, bf16_lo(f.y), F[k][8 * q + 2]);
                F[k][8 * q + 3] = fmaf(w, bf16_hi(f.y), F[k][8 * q + 3]);
                F[k][8 * q + 4] = fmaf(w, bf16_lo(f.z), F[k][8 * q + 4]);
                F[k][8 * q + 5] = fmaf(w, bf16_hi(f.z), F[k][8 * q + 5]);
                F[k][8 * q + 6] = fmaf(w, bf16_lo(f.w), F[k][8 * q + 6]);
                F[k][8 * q + 7] = fmaf(w, bf16_hi(f.w), F[k][8 * q + 7]);
              }
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
