// Front-to-back alpha blend, one workgroup per (pose, tile).
//
// Each wave owns a square block of the tile (8x8 pixels at tile 8 and 16,
// 16x16 with 4 pixels per lane at tile 32); compact blocks keep the lanes'
// blend decisions coherent.  The workgroup walks the tile's
// depth-ordered list in batches: every thread stages one splat (geometry,
// colour, FP32 feature vector) into LDS and marks which waves' blocks its
// support rectangle touches; each wave then compacts the batch to the entries
// that touch its block and runs its pixels through them, reading each splat
// as an LDS broadcast.  Each splat's tile-list entry carries its Gaussian
// index beside its record index, so the staging loads of record and feature
// vector go out together.  Pairs whose exponent is clearly below the 1/255 gate
// are rejected before the exponential; the exact gate, clamp and stop tests
// follow.  A pixel stops at the first splat that would take its transmittance
// below 1e-4; the batch loop ends when every pixel of the tile has stopped.
// Outputs are planar per pose.
#include "hgsr_device.hpp"
#include "launch.hpp"

namespace hgsr {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short shortx4 __attribute__((ext_vector_type(4)));

// Splats per matrix-core step of the feature sum (16 or 8).
#ifndef HGSR_MF_GROUP
#define HGSR_MF_GROUP 8
#endif
constexpr int kMfGroup = HGSR_MF_GROUP;
#ifndef HGSR_FEAT_ROUND
#define HGSR_FEAT_ROUND 4
#endif
constexpr int kFeatRound = HGSR_FEAT_ROUND;

template <int TILE, int D, bool BF16, bool MFK>
__global__ __launch_bounds__(BlendShape<TILE>::kThreads) void blend_fwd_kernel(BlendArgs a) {
  using S = BlendShape<TILE>;
  constexpr int NT = S::kThreads, NB = S::kBatch, NW = S::kWaves, BW = S::kBlockW, BH = S::kBlockH, PPT = S::kPPT;
  // 32 feature channels, one pixel per lane: the feature sum can run on the
  // matrix cores, per 16 splats F^T[32 ch x 64 px] += Feat^T[32 x 16] W[16 x 64]
  // with the FP32 weights split exactly into three bfloat16 parts
  constexpr bool MF = MFK && D == 32 && PPT == 1;
  constexpr bool LDS_F32 = D > 0 && D <= 32 && !MF;     // features as FP32 in LDS (else raw bf16)
  constexpr int FW = D == 0 ? 1 : (LDS_F32 ? D : D / 2);  // 32-bit words per feature vector
  // slot stride in words: padded by 4 so that the staging threads' 16-byte
  // writes (one slot each) fall in different banks
  constexpr int FS = D == 0 ? 1 : FW + 4;
  constexpr int DV = D / 8;                              // 16-byte bf16 vectors per feature
  constexpr int PARTS = (DV >= NT / NB) ? NT / NB : 1;   // threads sharing one splat's feature load
  __shared__ float4 s_geo[NB];
  __shared__ float4 s_opz[NB];
  __shared__ float4 s_col[NB];
  __shared__ uint32_t s_fw[NB * FS];
  __shared__ uint8_t s_mask[NB];
  __shared__ uint16_t s_list[NW][NB];
  __shared__ int s_item;
  if (a.flags[0] & 3) return;
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1), wave = tid >> 6;
  const int W = a.c.W, H = a.c.H;
  const int64_t HW = static_cast<int64_t>(W) * H;
  const bool persistent = a.schedule != kSchedGrid;
  int chunk_next = 0, chunk_left = 0;  // persistent: the claimed run of items

  for (int iter = 0;; ++iter) {
    int item;
    if (persistent) {
      if (chunk_left == 0) {
        if (tid == 0) s_item = static_cast<int>(atomicAdd(a.queue, static_cast<uint32_t>(kQueueChunk)));
        __syncthreads();
        chunk_next = s_item;
        chunk_left = kQueueChunk;
        __syncthreads();
      }
      item = chunk_next++;
      --chunk_left;
      if (item >= a.n_items) break;
    } else {
      if (iter > 0) break;
      item = xcd_item(blockIdx.x, gridDim.x);
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
    const int bx0 = tx * TILE + (wave % S::kBlocksX) * BW, by0 = ty * TILE + (wave / S::kBlocksX) * BH;
    float pxf[PPT], pyf[PPT], T[PPT], C[PPT][3], Z[PPT];
    float F[PPT][(D > 0 && !MF) ? D : 1];
    floatx16 acc0 = {}, acc1 = {};
    uint32_t used[PPT];
    bool done[PPT], inside[PPT];
    int pix[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      const int li = lane + k * kWave;
      const int px = bx0 + (li % BW), py = by0 + (li / BW);
      inside[k] = px < W && py < H;
      pix[k] = py * W + px;
      pxf[k] = static_cast<float>(px) + 0.5f;
      pyf[k] = static_cast<float>(py) + 0.5f;
      T[k] = 1.f;
      C[k][0] = C[k][1] = C[k][2] = 0.f;
      Z[k] = 0.f;
#pragma unroll
      for (int d = 0; d < ((D > 0 && !MF) ? D : 1); ++d) F[k][d] = 0.f;
      used[k] = 0;
      done[k] = !inside[k];
    }

    for (uint32_t b0 = range.x; b0 < range.y; b0 += NB) {
      bool all_mine = true;
#pragma unroll
      for (int k = 0; k < PPT; ++k) all_mine &= done[k];
      if (__syncthreads_and(all_mine)) break;
      const int e = tid % NB, part = tid / NB;
      const uint32_t j = b0 + e;
      if (j < range.y) {
        const uint32_t lv = a.list[j];
        const uint32_t gid = a.list_gid[j];
        const float4* sp = reinterpret_cast<const float4*>(a.recs + (lv & kRecMask));
        const float4 g1 = sp[1];
        if (part == 0) {
          s_geo[e] = sp[0];
          s_opz[e] = g1;
          s_col[e] = sp[2];
          s_mask[e] = static_cast<uint8_t>(lv >> kRecBits);  // waves whose block the support meets
        }
        if constexpr (D > 0) {
          if (part < PARTS) {
            constexpr int QV = DV / PARTS;
            const uint4* fv = reinterpret_cast<const uint4*>(a.feat) + static_cast<int64_t>(gid) * DV + part * QV;
            if constexpr (LDS_F32) {
#pragma unroll
              for (int q = 0; q < QV; ++q) {
                const uint4 f = fv[q];
                uint4* dst = reinterpret_cast<uint4*>(&s_fw[e * FS + 8 * (part * QV + q)]);
                dst[0] = make_uint4(f.x << 16, f.x & 0xffff0000u, f.y << 16, f.y & 0xffff0000u);
                dst[1] = make_uint4(f.z << 16, f.z & 0xffff0000u, f.w << 16, f.w & 0xffff0000u);
              }
            } else {
#pragma unroll
              for (int q = 0; q < QV; ++q) reinterpret_cast<uint4*>(&s_fw[e * FS])[part * QV + q] = fv[q];
            }
          }
        }
      } else if (part == 0) {
        s_mask[e] = 0;
      }
      __syncthreads();
      const int nb = static_cast<int>(min(static_cast<uint32_t>(NB), range.y - b0));
      // compact the batch to the entries touching this wave's block (in order)
      int n_mine = 0;
      for (int c0 = 0; c0 < nb; c0 += kWave) {
        const int ce = c0 + lane;
        const bool hit = ce < nb && ((s_mask[ce] >> wave) & 1u);
        const uint64_t bal = __ballot(hit);
        if (hit) s_list[wave][n_mine + __popcll(bal & ((1ull << lane) - 1ull))] = static_cast<uint16_t>(ce);
        n_mine += __popcll(bal);
      }
      __builtin_amdgcn_wave_barrier();
      if constexpr (MF) {
        // MG splats per matrix step: 16 (32x32x16 bf16) or 8 (32x32x8 bf16)
        constexpr int MG = kMfGroup, HG = MG / 2;
        const int ch = lane & 31, half = lane >> 5;
        for (int ii = 0; ii < n_mine; ii += MG) {
          if (__all(done[0] ? 1 : 0)) break;  // every lane of the wave has stopped (uniform)
          // colour, depth and transmittance on the VALU, in list order; wq[q]
          // is this pixel's weight for the group's q-th splat (0 if not blended)
          float wq[MG];
          int jq[MG];
          bool any_w = false;
#pragma unroll
          for (int q = 0; q < MG; ++q) {
            const int i = ii + q;
            const int jj = i < n_mine ? __builtin_amdgcn_readfirstlane(static_cast<int>(s_list[wave][i])) : -1;
            jq[q] = jj;
            float w = 0.f;
            if (jj >= 0 && !done[0]) {
              const float4 geo = s_geo[jj];
              const float4 opz = s_opz[jj];
              const float dx = pxf[0] - geo.x, dy = pyf[0] - geo.y;
              const float power = pair_power(dx, dy, geo.z, geo.w, opz.x);
              if (power <= 0.f && power >= s_col[jj].w - kPreReject) {
                const float alpha = pair_alpha(opz.y, power);
                if (alpha >= kAlphaMin) {
                  const float Tn = T[0] * (1.f - alpha);
                  if (Tn < kTMin) {
                    done[0] = true;
                  } else {
                    w = alpha * T[0];
                    const float4 col = s_col[jj];
                    C[0][0] = fmaf(w, col.x, C[0][0]);
                    C[0][1] = fmaf(w, col.y, C[0][1]);
                    C[0][2] = fmaf(w, col.z, C[0][2]);
                    Z[0] = fmaf(w, opz.z, Z[0]);
                    T[0] = Tn;
                    used[0] = b0 + jj - range.x + 1;
                    any_w = true;
                  }
                }
              }
            }
            wq[q] = w;
          }
          if (!__any(any_w ? 1 : 0)) continue;
          // A: channel ch of splats HG*half + 0..HG-1 (raw bf16; a missing
          // splat reads slot 0 and meets zero weights)
          uint32_t ap[HG / 2];
#pragma unroll
          for (int t = 0; t < HG; t += 2) {
            const int j0 = max(half ? jq[HG + t] : jq[t], 0), j1 = max(half ? jq[HG + 1 + t] : jq[t + 1], 0);
            const uint32_t f0 = reinterpret_cast<const uint16_t*>(s_fw)[j0 * 2 * FS + ch];
            const uint32_t f1 = reinterpret_cast<const uint16_t*>(s_fw)[j1 * 2 * FS + ch];
            ap[t / 2] = f0 | (f1 << 16);
          }
          // B: weights of splats HG*half + t for pixel ch (acc0) or 32 + ch
          // (acc1); one lane-half exchange gives both.  The FP32 weights go
          // in as three exact bfloat16 parts (hi, mid, lo): each step feeds
          // the top 8 significant bits and keeps the exact remainder.
          float r0[HG], r1[HG];
#pragma unroll
          for (int t = 0; t < HG; ++t) {
            const auto sw = __builtin_amdgcn_permlane32_swap(__float_as_uint(wq[t]), __float_as_uint(wq[HG + t]),
                                                             false, false);
            r0[t] = __uint_as_float(sw[0]);
            r1[t] = __uint_as_float(sw[1]);
          }
#pragma unroll
          for (int part = 0; part < 3; ++part) {
#pragma unroll
            for (int side = 0; side < 2; ++side) {
              float* r = side ? r1 : r0;
              uint32_t bp[HG / 2];
#pragma unroll
              for (int t = 0; t < HG / 2; ++t) {
                const uint32_t x = __float_as_uint(r[2 * t]) & 0xffff0000u;
                const uint32_t y = __float_as_uint(r[2 * t + 1]) & 0xffff0000u;
                bp[t] = (x >> 16) | y;
                if (part < 2) {
                  r[2 * t] -= __uint_as_float(x);
                  r[2 * t + 1] -= __uint_as_float(y);
                }
              }
              floatx16& acc = side ? acc1 : acc0;
              if constexpr (MG == 16) {
                bf16x8 av, bv;
                __builtin_memcpy(&av, ap, 16);
                __builtin_memcpy(&bv, bp, 16);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
              } else {
                shortx4 av, bv;
                __builtin_memcpy(&av, ap, 8);
                __builtin_memcpy(&bv, bp, 8);
                acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(av, bv, acc, 0, 0, 0);
              }
            }
          }
        }
      } else {
        // the next entry's index is read one step ahead, and a splat's
        // geometry, colour and feature vector each in one round of LDS reads,
        // so that a step waits on LDS latency twice instead of seven times
        int jn = n_mine > 0 ? static_cast<int>(s_list[wave][0]) : 0;
        for (int ii = 0; ii < n_mine; ++ii) {
          bool mine = true;
#pragma unroll
          for (int k = 0; k < PPT; ++k) mine &= done[k];
          if (mine) break;
          const int jj = __builtin_amdgcn_readfirstlane(jn);
          jn = ii + 1 < n_mine ? static_cast<int>(s_list[wave][ii + 1]) : 0;
          const float4 geo = s_geo[jj];
          const float4 opz = s_opz[jj];
          const float4 col = s_col[jj];
          const float pmin = col.w;
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
            C[k][0] = fmaf(w, col.x, C[k][0]);
            C[k][1] = fmaf(w, col.y, C[k][1]);
            C[k][2] = fmaf(w, col.z, C[k][2]);
            Z[k] = fmaf(w, opz.z, Z[k]);
            if constexpr (D > 0) {
              if constexpr (LDS_F32) {
                const float4* fsrc = reinterpret_cast<const float4*>(&s_fw[jj * FS]);
                constexpr int FR = (D / 4 > kFeatRound) ? kFeatRound : D / 4;  // float4 reads per round
#pragma unroll
                for (int q0 = 0; q0 < D / 4; q0 += FR) {
                  float4 fq[FR];
#pragma unroll
                  for (int q = 0; q < FR; ++q) fq[q] = fsrc[q0 + q];
                  __builtin_amdgcn_sched_barrier(0);  // the round's reads issued before its FMAs
#pragma unroll
                  for (int q = 0; q < FR; ++q) {
                    const float4 f = fq[q];
                    F[k][4 * (q0 + q) + 0] = fmaf(w, f.x, F[k][4 * (q0 + q) + 0]);
                    F[k][4 * (q0 + q) + 1] = fmaf(w, f.y, F[k][4 * (q0 + q) + 1]);
                    F[k][4 * (q0 + q) + 2] = fmaf(w, f.z, F[k][4 * (q0 + q) + 2]);
                    F[k][4 * (q0 + q) + 3] = fmaf(w, f.w, F[k][4 * (q0 + q) + 3]);
                  }
                }
              } else {
                const uint4* fq = reinterpret_cast<const uint4*>(&s_fw[jj * FS]);
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
      if constexpr (D > 0 && !MF) {
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
    if constexpr (MF) {
      // accumulator layout (32x32 MFMA): lane l, register r holds channel
      // 8 (r/4) + 4 (l/32) + r%4 of pixel l%32 (acc0) or 32 + l%32 (acc1)
      if (a.out_feat) {
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
          const int li = (lane & 31) + 32 * nb;
          const int px = bx0 + (li % BW), py = by0 + (li / BW);
          if (px < W && py < H) {
            // 32-bit offsets within this pose's feature planes
            const uint32_t pofs = static_cast<uint32_t>(py * W + px) +
                                  static_cast<uint32_t>(4 * (lane >> 5)) * static_cast<uint32_t>(HW);
            const int64_t pbase_f = static_cast<int64_t>(pose) * D * HW;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
              const uint32_t o = pofs + static_cast<uint32_t>(8 * (r / 4) + (r % 4)) * static_cast<uint32_t>(HW);
              const float v = nb == 0 ? acc0[r] : acc1[r];
              if constexpr (BF16) (static_cast<uint16_t*>(a.out_feat) + pbase_f)[o] = f32_to_bf16_rne(v);
              else (static_cast<float*>(a.out_feat) + pbase_f)[o] = v;
            }
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
  if (D == 32 && TILE != 32 && a.feat_mfma)
    hipLaunchKernelGGL((blend_fwd_kernel<TILE, D, BF16, true>), dim3(n_ctas), dim3(NT), 0, s, a);
  else
    hipLaunchKernelGGL((blend_fwd_kernel<TILE, D, BF16, false>), dim3(n_ctas), dim3(NT), 0, s, a);
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
