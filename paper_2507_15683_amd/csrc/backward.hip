// Backward of the splat rasterizer.
//
// blend_bwd: one workgroup per (pose, tile).  Each pixel starts from its
// saved final transmittance and list length and walks its tile list back to
// front, recovering T_j = T_{j+1} / (1 - alpha_j) instead of storing
// per-pixel lists.  With h_j = gC.c_j + gZ z_j + gF.f_j and the suffix sum
// S_j = sum_{k>j} w_k h_k,
//   dL/dalpha_j = T_j h_j - (S_j + gT T_final) / (1 - alpha_j),
// where gT collects the outputs' direct dependence on T_final (background,
// depth normalisation, alpha).  Per-splat gradients are summed across the
// 64 lanes of a wave before one atomic per value.
//
// project_bwd: one thread per visible (pose, Gaussian): chains the splat
// gradients through the conic inverse, the EWA covariance, the clamped
// pinhole Jacobian, the camera transform and the SH view direction, into
// dL/d(mean, opacity, scales, rotation, SH) and the pose's left-perturbation
// tangent (rho, phi), block-reduced per pose.
#include "hgsr_device.hpp"
#include "launch.hpp"

namespace hgsr {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef short shortx4 __attribute__((ext_vector_type(4)));

// Splats per matrix-core group of the feature term (MFH).
constexpr int kHGroup = 32;

// MFH: the feature part of h_j = gF . f_j for a group of 32 splats and the
// wave's 64 pixels is one matrix product H[32 x 64] = F[32 x 32] gF[32 x 64],
// run as v_mfma_f32_32x32x8_bf16 (channels in four steps of 8, pixels in two
// blocks of 32).  F is the splats' stored bf16 features (exact); the FP32
// pixel gradient gF enters as three bf16 parts (top, middle and last 8
// significant bits), so the products are exact and only the summation order
// differs from the FP32 dot product.  H goes to LDS, where the walk reads its
// pixel's value of each splat.
// PO (pose only, residual loss): the opacity and depth sums are not formed
// (the residual has no depth term and no opacity gradient was asked for),
// eight sums per splat instead of ten.
template <int TILE, int D, bool FEATGRAD, bool RES, bool MFH, bool PO>
__device__ __forceinline__ void blend_bwd_item(const BackArgs& a, const int item) {
  using Sh = BlendShape<TILE>;
  constexpr int NT = Sh::kThreads, NB = Sh::kBatch, NW = Sh::kWaves, BW = Sh::kBlockW, BH = Sh::kBlockH;
  constexpr int PPT = Sh::kPPT;
  constexpr int DV = D / 8;                             // 16-byte bf16 vectors per feature
  constexpr int DD = D > 0 ? D : 1;
  constexpr int PARTS = (DV >= NT / NB) ? NT / NB : 1;  // threads sharing one splat's feature load
  constexpr bool MF = MFH && D == 32 && PPT == 1 && !FEATGRAD;
  __shared__ float4 s_geo[NB];
  __shared__ float4 s_opz[NB];
  __shared__ float4 s_col[NB];
  __shared__ uint32_t s_rec[NB];
  constexpr int FS = D + 4;  // padded slot stride (words): staging writes spread over banks
  __shared__ float s_f[(D > 0 && !MF) ? NB * FS : 1];  // features as FP32
  constexpr int FBS = 20;    // MF: raw bf16 feature slot (16 words + 4 of padding)
  __shared__ uint32_t s_fb[MF ? NB * FBS : 1];
  __shared__ float s_h[MF ? NW : 1][MF ? kHGroup : 1][MF ? kWave : 1];  // MF: H per wave
  __shared__ uint8_t s_mask[NB];
  __shared__ uint16_t s_list[NW][NB];
  __shared__ float s_g[NB][10];  // per staged splat: the workgroup's gradient sums
  __shared__ uint32_t s_max;
  __shared__ float s_lw[NW];
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1), wave = tid >> 6;
  const int W = a.c.W, H = a.c.H;
  const int64_t HW = static_cast<int64_t>(W) * H;
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
  const int bx0 = tx * TILE + (wave % Sh::kBlocksX) * BW, by0 = ty * TILE + (wave / Sh::kBlocksX) * BH;

  float pxf[PPT], pyf[PPT], T[PPT], Tf[PPT], S[PPT], gC[PPT][3], GZ[PPT], gT[PPT];
  float gF[PPT][DD];
  uint32_t last[PPT];
  if (tid == 0) s_max = 0;
  for (int e = tid; e < NB * 10; e += NT) (&s_g[0][0])[e] = 0.f;
  __syncthreads();
  uint32_t my_max = 0;
  float lsum = 0.f;  // this lane's residual terms (RES)
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int li = lane + k * kWave;
    const int px = bx0 + (li % BW), py = by0 + (li / BW);
    const bool inside = px < W && py < H;
    pxf[k] = static_cast<float>(px) + 0.5f;
    pyf[k] = static_cast<float>(py) + 0.5f;
    last[k] = 0;
    T[k] = Tf[k] = 1.f;
    S[k] = 0.f;
    gC[k][0] = gC[k][1] = gC[k][2] = 0.f;
    GZ[k] = gT[k] = 0.f;
#pragma unroll
    for (int d = 0; d < DD; ++d) gF[k][d] = 0.f;
    if (!inside) continue;
    const int64_t pix = static_cast<int64_t>(py) * W + px;
    const int64_t o = static_cast<int64_t>(pose) * HW + pix;
    last[k] = a.n_used[o];
    Tf[k] = T[k] = a.final_T[o];
    const float A = 1.f - Tf[k];
    float gtv = 0.f;
    if constexpr (RES) {
      // the residual's gradient at this pixel (the definition the residual
      // kernel evaluates), from the forward's outputs and the target
      const float inv = a.res_inv_hw;
      const int64_t o3 = static_cast<int64_t>(pose) * 3 * HW + pix;
      const int64_t tp = static_cast<int64_t>(pose) * a.res_t_stride;
      float l = 0.f;
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        const float d = a.fwd_rgb[o3 + ch * HW] - a.res_rgb_t[tp * 3 * HW + pix + ch * HW];
        l += fabsf(d);
        gC[k][ch] = d > 0.f ? inv : (d < 0.f ? -inv : 0.f);
      }
      gtv = gC[k][0] * a.bg[0] + gC[k][1] * a.bg[1] + gC[k][2] * a.bg[2];
      if constexpr (D > 0) {
        const int64_t of = static_cast<int64_t>(pose) * D * HW + pix;
        const int64_t tf = tp * D * HW + pix;
        float t[D];
        float dot = 0.f, na = 0.f, nb = 0.f;
#pragma unroll
        for (int d = 0; d < D; ++d) {
          gF[k][d] = a.fwd_feat_bf16 ? bf16_lo(static_cast<const uint16_t*>(a.fwd_feat)[of + d * HW])
                                     : static_cast<const float*>(a.fwd_feat)[of + d * HW];
          t[d] = a.res_feat_t[tf + d * HW];
          dot = fmaf(gF[k][d], t[d], dot);
          na = fmaf(gF[k][d], gF[k][d], na);
          nb = fmaf(t[d], t[d], nb);
        }
        na = sqrtf(na);
        nb = sqrtf(nb);
        const float n = na * nb + kCosEps;
        const float cosv = dot / n;
        l += a.res_lam * (1.f - cosv);
        const float s1 = -a.res_lam * inv / n;
        const float s2 = na > 0.f ? a.res_lam * inv * dot * nb / (n * n * na) : 0.f;
#pragma unroll
        for (int d = 0; d < D; ++d) gF[k][d] = s1 * t[d] + s2 * gF[k][d];
      }
      lsum += l * inv;
    } else if (a.g_rgb) {
      const int64_t o3 = static_cast<int64_t>(pose) * 3 * HW + pix;
      gC[k][0] = a.g_rgb[o3];
      gC[k][1] = a.g_rgb[o3 + HW];
      gC[k][2] = a.g_rgb[o3 + 2 * HW];
      gtv = gC[k][0] * a.bg[0] + gC[k][1] * a.bg[1] + gC[k][2] * a.bg[2];
    }
    if (a.g_depth && A > 0.f) {
      const float gd = a.g_depth[o];
      GZ[k] = gd / A;
      gtv += gd * a.fwd_depth[o] / A;
    }
    if (a.g_alpha) gtv -= a.g_alpha[o];
    gT[k] = gtv;
    if constexpr (D > 0 && !RES) {
      if (a.g_feat) {
        const int64_t of = static_cast<int64_t>(pose) * D * HW + pix;
#pragma unroll
        for (int d = 0; d < D; ++d) gF[k][d] = a.g_feat[of + d * HW];
      }
    }
    my_max = max(my_max, last[k]);
  }
  // list positions this wave must visit: below the largest saved length
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) my_max = max(my_max, static_cast<uint32_t>(__shfl_xor(my_max, off, kWave)));
  const uint32_t wave_max = my_max;
  if (lane == 0) atomicMax(&s_max, wave_max);
  if constexpr (RES) {
    // this tile's loss share, summed in a fixed order (lanes, then waves)
    lsum = wave_sum(lsum);
    if (lane == 0) s_lw[wave] = lsum;
  }
  __syncthreads();
  if constexpr (RES) {
    if (tid == 0) {
      float t = 0.f;
#pragma unroll
      for (int w = 0; w < NW; ++w) t += s_lw[w];
      a.res_part[static_cast<int64_t>(pose) * a.c.tiles_per_pose + tile] = t;
    }
  }
  const uint32_t n_max = s_max;
  if (n_max == 0) return;

  // batches back to front; positions are relative to range.x
  const int n_batches = static_cast<int>((n_max + NB - 1) / NB);
  for (int bi = n_batches - 1; bi >= 0; --bi) {
    const uint32_t b0 = static_cast<uint32_t>(bi) * NB;
    const int nb = static_cast<int>(min(static_cast<uint32_t>(NB), n_max - b0));
    {
      const int e = tid % NB, part = tid / NB;
      if (e < nb) {
        const uint32_t lv = a.list[range.x + b0 + e];
        const uint32_t gid = a.list_gid[range.x + b0 + e];
        const uint32_t r = lv & kRecMask;
        const float4* sp = reinterpret_cast<const float4*>(a.recs + r);
        const float4 g1 = sp[1];
        if (part == 0) {
          s_geo[e] = sp[0];
          s_opz[e] = g1;
          s_col[e] = sp[2];
          s_rec[e] = r;
          s_mask[e] = static_cast<uint8_t>(lv >> kRecBits);  // waves whose block the support meets
        }
        if constexpr (DV > 0) {
          if (part < PARTS) {
            constexpr int QV = DV / PARTS;
            const uint4* fv = reinterpret_cast<const uint4*>(a.feat) + static_cast<int64_t>(gid) * DV + part * QV;
#pragma unroll
            for (int q = 0; q < QV; ++q) {
              const uint4 f = fv[q];
              if constexpr (MF) {
                reinterpret_cast<uint4*>(&s_fb[e * FBS])[part * QV + q] = f;
              } else {
                float4* dst = reinterpret_cast<float4*>(&s_f[e * FS + 8 * (part * QV + q)]);
                dst[0] = make_float4(bf16_lo(f.x), bf16_hi(f.x), bf16_lo(f.y), bf16_hi(f.y));
                dst[1] = make_float4(bf16_lo(f.z), bf16_hi(f.z), bf16_lo(f.w), bf16_hi(f.w));
              }
            }
          }
        }
      }
    }
    __syncthreads();
    // compact the batch to the entries touching this wave's block and below
    // its largest saved length (in list order)
    int n_mine = 0;
    for (int c0 = 0; c0 < nb; c0 += kWave) {
      const int ce = c0 + lane;
      const bool hit = ce < nb && b0 + ce < wave_max && ((s_mask[ce] >> wave) & 1u);
      const uint64_t bal = __ballot(hit);
      if (hit) s_list[wave][n_mine + __popcll(bal & ((1ull << lane) - 1ull))] = static_cast<uint16_t>(ce);
      n_mine += __popcll(bal);
    }
    __builtin_amdgcn_wave_barrier();
    // the next entry's index is read one step ahead
    int jn = n_mine > 0 ? static_cast<int>(s_list[wave][n_mine - 1]) : 0;
    for (int ii = n_mine - 1; ii >= 0; --ii) {
      if constexpr (MF) {
        if (ii == n_mine - 1 || (ii + 1) % kHGroup == 0) {
          // H for the group of compacted entries [g0, g0 + 32) holding ii
          const int g0 = ii / kHGroup * kHGroup;
          const int row = lane & 31, half = lane >> 5;
          const int e = g0 + row;
          const int js = e < n_mine ? static_cast<int>(s_list[wave][e]) : -1;
          floatx16 acc0 = {}, acc1 = {};
#pragma unroll
          for (int ks = 0; ks < 4; ++ks) {
            uint2 av = make_uint2(0u, 0u);
            if (js >= 0) av = *reinterpret_cast<const uint2*>(&s_fb[js * FBS + 4 * ks + 2 * half]);
            shortx4 A;
            __builtin_memcpy(&A, &av, 8);
            // B: this lane's pixel gradient, channels 8 ks .. 8 ks + 7, split
            // into three exact bf16 parts; lane l supplies channels
            // 8 ks + 4 (l / 32) + 0..3 of pixel l % 32 (block 0) and of pixel
            // 32 + l % 32 (block 1): its own half of the channels for its own
            // block, the partner lane's (l ^ 32) for the other, exchanged with
            // one lane-half swap per word
            float r[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) {
              r[c] = gF[0][8 * ks + c];
              // keeps the split inside the group loop (recomputed per group)
              // instead of hoisted into 48 live registers for the whole walk
              asm volatile("" : "+v"(r[c]));
            }
#pragma unroll
            for (int part = 0; part < 3; ++part) {
              uint32_t hw[4];  // bf16 pairs: channels (0,1) (2,3) (4,5) (6,7)
#pragma unroll
              for (int c = 0; c < 4; ++c) {
                const uint32_t x = __float_as_uint(r[2 * c]) & 0xffff0000u;
                const uint32_t y = __float_as_uint(r[2 * c + 1]) & 0xffff0000u;
                hw[c] = (x >> 16) | y;
                if (part < 2) {
                  r[2 * c] -= __uint_as_float(x);
                  r[2 * c + 1] -= __uint_as_float(y);
                }
              }
              uint32_t b0w[2], b1w[2];
#pragma unroll
              for (int w = 0; w < 2; ++w) {
                const auto sw = __builtin_amdgcn_permlane32_swap(hw[w], hw[2 + w], false, false);
                b0w[w] = sw[0];
                b1w[w] = sw[1];
              }
              shortx4 B0, B1;
              __builtin_memcpy(&B0, b0w, 8);
              __builtin_memcpy(&B1, b1w, 8);
              acc0 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(A, B0, acc0, 0, 0, 0);
              acc1 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(A, B1, acc1, 0, 0, 0);
            }
          }
          // accumulator layout: lane l, register r holds row 8 (r/4) + 4 (l/32)
          // + r%4 (group entry) of column l % 32 (pixel, + 32 for acc1)
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int hr = 8 * (r / 4) + 4 * half + (r % 4);
            s_h[MF ? wave : 0][hr][row] = acc0[r];
            s_h[MF ? wave : 0][hr][32 + row] = acc1[r];
          }
          __builtin_amdgcn_wave_barrier();
        }
      }
      const int jj = __builtin_amdgcn_readfirstlane(jn);
      jn = ii > 0 ? static_cast<int>(s_list[wave][ii - 1]) : 0;
      const uint32_t pos = b0 + jj;
      const float4 geo = s_geo[jj];
      const float4 opz = s_opz[jj];
      const float4 col = s_col[jj];
      float g[10];
#pragma unroll
      for (int q = 0; q < 10; ++q) g[q] = 0.f;
      float gfe[FEATGRAD ? DD : 1];
      if constexpr (FEATGRAD) {
#pragma unroll
        for (int d = 0; d < DD; ++d) gfe[d] = 0.f;
      }
      bool any = false;
#pragma unroll
      for (int k = 0; k < PPT; ++k) {
        if (pos >= last[k]) continue;
        const float dx = pxf[k] - geo.x, dy = pyf[k] - geo.y;
        const float power = pair_power(dx, dy, geo.z, geo.w, opz.x);
        if (power > 0.f) continue;
        const float G = __expf(power);
        const float alpha = fminf(kAlphaMax, opz.y * G);
        if (alpha < kAlphaMin) continue;
        any = true;
        const float om = 1.f - alpha;
        const float iom = __builtin_amdgcn_rcpf(om);  // 1/(1 - alpha), alpha <= 0.99
        const float Tj = T[k] * iom;
        const float w = alpha * Tj;
        // gradient arithmetic (not a blend decision): fused multiply-adds
        float h = fmaf(gC[k][0], col.x, fmaf(gC[k][1], col.y, fmaf(gC[k][2], col.z, GZ[k] * opz.z)));
        if constexpr (MF) {
          h += s_h[MF ? wave : 0][ii % kHGroup][lane];
        } else if constexpr (D > 0) {
          const float4* fq = reinterpret_cast<const float4*>(&s_f[jj * FS]);
#pragma unroll
          for (int q = 0; q < D / 4; ++q) {
            const float4 f = fq[q];
            h = fmaf(gF[k][4 * q + 0], f.x, h);
            h = fmaf(gF[k][4 * q + 1], f.y, h);
            h = fmaf(gF[k][4 * q + 2], f.z, h);
            h = fmaf(gF[k][4 * q + 3], f.w, h);
          }
        }
        const float dA = fmaf(Tj, h, -(fmaf(gT[k], Tf[k], S[k]) * iom));
        S[k] = fmaf(w, h, S[k]);
        T[k] = Tj;
        g[7] = fmaf(w, gC[k][0], g[7]);
        g[8] = fmaf(w, gC[k][1], g[8]);
        g[9] = fmaf(w, gC[k][2], g[9]);
        if constexpr (!PO) g[6] = fmaf(w, GZ[k], g[6]);
        if (opz.y * G <= kAlphaMax) {
          const float dpow = dA * alpha;
          const float hx = -0.5f * dpow * dx, hy = -0.5f * dpow * dy;
          if constexpr (!PO) g[5] = fmaf(dA, G, g[5]);
          g[0] = fmaf(dpow, fmaf(geo.z, dx, geo.w * dy), g[0]);
          g[1] = fmaf(dpow, fmaf(geo.w, dx, opz.x * dy), g[1]);
          g[2] = fmaf(hx, dx, g[2]);
          g[3] = fmaf(2.f * hx, dy, g[3]);
          g[4] = fmaf(hy, dy, g[4]);
        }
        if constexpr (FEATGRAD) {
#pragma unroll
          for (int d = 0; d < DD; ++d) gfe[d] = fmaf(w, gF[k][d], gfe[d]);
        }
      }
      if (!__any(any)) continue;
      if constexpr (PO) wave_add8(g, s_g[jj]);
      else wave_add10(g, s_g[jj]);
      if constexpr (FEATGRAD) {
#pragma unroll
        for (int d = 0; d < DD; ++d) gfe[d] = wave_sum(gfe[d]);
        if (lane == 0) {
          float* fd = a.g_featvec + static_cast<int64_t>(__float_as_uint(opz.w)) * D;
#pragma unroll
          for (int d = 0; d < DD; ++d) atomicAdd(fd + d, gfe[d]);
        }
      }
    }
    __syncthreads();
    // one global atomic per nonzero sum of the batch; clear for the next
    for (int e = tid; e < nb * 10; e += NT) {
      const int slot = e / 10, q = e - slot * 10;
      const float v = s_g[slot][q];
      if (v != 0.f) {
        atomicAdd(a.g_rec + static_cast<int64_t>(s_rec[slot]) * kGradRecStride + q, v);
        s_g[slot][q] = 0.f;
      }
    }
  }
}

// One workgroup per (pose, tile) item, or (PERSIST) a grid of workgroups
// claiming runs of kQueueChunk items from a device counter until it passes
// the item count.
template <int TILE, int D, bool FEATGRAD, bool RES, bool MFH, bool PERSIST, bool PO = false>
__global__ __launch_bounds__(BlendShape<TILE>::kThreads) void blend_bwd_kernel(BackArgs a) {
  if (a.flags[0] & 3) return;
  if constexpr (PERSIST) {
    __shared__ int s_item;
    for (;;) {
      if (threadIdx.x == 0) s_item = static_cast<int>(atomicAdd(a.queue, static_cast<uint32_t>(kQueueChunk)));
      __syncthreads();
      const int first = s_item;
      __syncthreads();
      if (first >= a.n_items) break;
      const int last = min(first + kQueueChunk, a.n_items);
      for (int item = first; item < last; ++item) {
        blend_bwd_item<TILE, D, FEATGRAD, RES, MFH, PO>(a, item);
        __syncthreads();  // the item's LDS is reused by the next one
      }
    }
  } else {
    blend_bwd_item<TILE, D, FEATGRAD, RES, MFH, PO>(a, xcd_item(blockIdx.x, gridDim.x));
  }
}

// Per-pose loss from the per-tile shares, in a fixed order (deterministic).
__global__ __launch_bounds__(256) void loss_reduce_kernel(const float* part, int32_t tiles_per_pose, float* loss) {
  __shared__ float s_r[256];
  const int pose = blockIdx.x;
  const float* p = part + static_cast<int64_t>(pose) * tiles_per_pose;
  float v = 0.f;
  for (int t = threadIdx.x; t < tiles_per_pose; t += 256) v += p[t];
  s_r[threadIdx.x] = v;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) s_r[threadIdx.x] += s_r[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[pose] = s_r[0];
}

void launch_loss_reduce(const float* part, int32_t tiles_per_pose, int32_t P, float* loss, hipStream_t s) {
  hipLaunchKernelGGL(loss_reduce_kernel, dim3(P), dim3(256), 0, s, part, tiles_per_pose, loss);
}

template <int TILE, int D, bool PERSIST>
static void launch_bwd_tdp(const BackArgs& a, int items, hipStream_t s) {
  constexpr int NT = BlendShape<TILE>::kThreads;
  // the feature term on the matrix cores: 32 channels, one pixel per lane,
  // no per-Gaussian feature gradient
  constexpr bool MFOK = D == 32 && BlendShape<TILE>::kPPT == 1;
  const bool mf = MFOK && a.feat_mfma && !a.g_featvec;
  if (a.res_rgb_t) {
    if (a.g_featvec)
      hipLaunchKernelGGL((blend_bwd_kernel<TILE, D, true, true, false, PERSIST>), dim3(items), dim3(NT), 0, s, a);
    else if (mf)
      hipLaunchKernelGGL((blend_bwd_kernel<TILE, D, false, true, MFOK, PERSIST>), dim3(items), dim3(NT), 0, s, a);
    else if (a.pose_only)
      hipLaunchKernelGGL((blend_bwd_kernel<TILE, D, false, true, false, PERSIST, true>), dim3(items), dim3(NT), 0, s,
                         a);
    else
      hipLaunchKernelGGL((blend_bwd_kernel<TILE, D, false, true, false, PERSIST>), dim3(items), dim3(NT), 0, s, a);
  } else {
    if (a.g_featvec)
      hipLaunchKernelGGL((blend_bwd_kernel<TILE, D, true, false, false, PERSIST>), dim3(items), dim3(NT), 0, s, a);
    else if (mf)
      hipLaunchKernelGGL((blend_bwd_kernel<TILE, D, false, false, MFOK, PERSIST>), dim3(items), dim3(NT), 0, s, a);
    else
      hipLaunchKernelGGL((blend_bwd_kernel<TILE, D, false, false, false, PERSIST>), dim3(items), dim3(NT), 0, s, a);
  }
}

template <int TILE, int D>
static void launch_bwd_td(const BackArgs& a, int items, hipStream_t s) {
  if (a.schedule != kSchedGrid) launch_bwd_tdp<TILE, D, true>(a, a.n_ctas, s);
  else launch_bwd_tdp<TILE, D, false>(a, items, s);
}

template <int TILE>
static void launch_bwd_t(const BackArgs& a, int items, hipStream_t s) {
  switch (a.D) {
    case 0: launch_bwd_td<TILE, 0>(a, items, s); break;
    case 8: launch_bwd_td<TILE, 8>(a, items, s); break;
    case 16: launch_bwd_td<TILE, 16>(a, items, s); break;
    case 32: launch_bwd_td<TILE, 32>(a, items, s); break;
    default: launch_bwd_td<TILE, 64>(a, items, s); break;
  }
}

void launch_blend_bwd(const BackArgs& a, hipStream_t s) {
  const int items = a.P * a.c.tiles_per_pose;
  switch (a.c.tile) {
    case 8: launch_bwd_t<8>(a, items, s); break;
    case 32: launch_bwd_t<32>(a, items, s); break;
    default: launch_bwd_t<16>(a, items, s); break;
  }
}

// ------------------------------------------------------------ projection backward
// Gradient of the real SH basis polynomials (as functions on R^3) contracted
// with per-basis weights c[k] (one colour channel): returns sum_k c_k grad Y_k.
template <int DEG>
__device__ __forceinline__ void sh_grad_dir(const float* c, float x, float y, float z, float g[3]) {
  g[0] = g[1] = g[2] = 0.f;
  if constexpr (DEG >= 1) {
    const float C1 = 0.48860251190291987f;
    g[1] += -C1 * c[1];
    g[2] += C1 * c[2];
    g[0] += -C1 * c[3];
  }
  if constexpr (DEG >= 2) {
    const float A = 1.0925484305920792f, B = 0.31539156525252005f, Cc = 0.5462742152960396f;
    g[0] += c[4] * A * y;
    g[1] += c[4] * A * x;
    g[1] += -c[5] * A * z;
    g[2] += -c[5] * A * y;
    g[0] += -2.f * c[6] * B * x;
    g[1] += -2.f * c[6] * B * y;
    g[2] += 4.f * c[6] * B * z;
    g[0] += -c[7] * A * z;
    g[2] += -c[7] * A * x;
    g[0] += 2.f * c[8] * Cc * x;
    g[1] += -2.f * c[8] * Cc * y;
  }
  if constexpr (DEG >= 3) {
    const float a3 = 0.5900435899266435f, b3 = 2.890611442640554f, c3 = 0.4570457994644658f,
                d3 = 0.3731763325901154f, e3 = 1.445305721320277f;
    const float xx = x * x, yy = y * y, zz = z * z;
    g[0] += c[9] * (-6.f * a3 * x * y);
    g[1] += c[9] * (-a3 * (3.f * xx - 3.f * yy));
    g[0] += c[10] * b3 * y * z;
    g[1] += c[10] * b3 * x * z;
    g[2] += c[10] * b3 * x * y;
    g[0] += c[11] * (2.f * c3 * x * y);
    g[1] += c[11] * (-c3 * (4.f * zz - xx - 3.f * yy));
    g[2] += c[11] * (-8.f * c3 * y * z);
    g[0] += c[12] * (-6.f * d3 * x * z);
    g[1] += c[12] * (-6.f * d3 * y * z);
    g[2] += c[12] * (d3 * (6.f * zz - 3.f * xx - 3.f * yy));
    g[0] += c[13] * (-c3 * (4.f * zz - 3.f * xx - yy));
    g[1] += c[13] * (2.f * c3 * x * y);
    g[2] += c[13] * (-8.f * c3 * x * z);
    g[0] += c[14] * (2.f * e3 * x * z);
    g[1] += c[14] * (-2.f * e3 * y * z);
    g[2] += c[14] * (e3 * (xx - yy));
    g[0] += c[15] * (-a3 * (3.f * xx - 3.f * yy));
    g[1] += c[15] * (6.f * a3 * x * y);
  }
}

// The Gaussian's SH coefficients (3 (DEG+1)^2 floats), read once for the
// colour and its direction gradient (16-byte loads when the array allows).
template <int DEG>
__device__ __forceinline__ void load_sh(const float* sh, int64_t i, float* v) {
  constexpr int N = 3 * (DEG + 1) * (DEG + 1);
  const float* c = sh + static_cast<int64_t>(N) * i;
  if constexpr (N % 4 == 0) {
    if ((reinterpret_cast<uintptr_t>(sh) & 15) == 0) {
#pragma unroll
      for (int q = 0; q < N / 4; ++q) {
        const float4 f = reinterpret_cast<const float4*>(c)[q];
        v[4 * q] = f.x; v[4 * q + 1] = f.y; v[4 * q + 2] = f.z; v[4 * q + 3] = f.w;
      }
      return;
    }
  }
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] = c[k];
}

// One record's gradients: the pose tangent's six components are added to gp;
// GAUSS: the Gaussian's own gradients (means, opacity, scales, rotation, SH)
// where their arrays are given.
template <int DEG, bool GAUSS>
__device__ __forceinline__ void record_grad(const ProjBackArgs& a, const int pose, const uint32_t slot, float gp[6]) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  {
    const int64_t idx = static_cast<int64_t>(pose) * a.rec_cap + slot;
    const float* gr = a.g_rec + idx * kGradRecStride;
    const float g_u = gr[0], g_v = gr[1], g_ca = gr[2], g_cb = gr[3], g_cc = gr[4], g_o = gr[5], g_z = gr[6];
    const float gcol[3] = {gr[7], gr[8], gr[9]};
    const Splat sp = a.recs[idx];
    const int64_t i = sp.gid;
    const float* Pm = a.poses + 12 * pose;
    const float mu[3] = {a.g.means[3 * i], a.g.means[3 * i + 1], a.g.means[3 * i + 2]};
    const float4 q4 = reinterpret_cast<const float4*>(a.g.quats)[i];
    const float ls[3] = {a.g.log_scales[3 * i], a.g.log_scales[3 * i + 1], a.g.log_scales[3 * i + 2]};
    float Sw[6];
    cov3_from(q4, ls, Sw);
    float mc[3];
    to_camera(Pm, mu, mc);
    const float x = mc[0], y = mc[1], z = mc[2];
    const float iz = 1.f / z;
    const float xz = x / z, yz = y / z;
    const bool clx = fabsf(xz) > a.c.limx, cly = fabsf(yz) > a.c.limy;
    const float xh = fminf(fmaxf(xz, -a.c.limx), a.c.limx);
    const float yh = fminf(fmaxf(yz, -a.c.limy), a.c.limy);
    const float fx = a.c.fx, fy = a.c.fy;
    const float J00 = fx * iz, J02 = -fx * xh * iz, J11 = fy * iz, J12 = -fy * yh * iz;
    // M = J R (rows m0, m1)
    const float m0[3] = {J00 * Pm[0] + J02 * Pm[8], J00 * Pm[1] + J02 * Pm[9], J00 * Pm[2] + J02 * Pm[10]};
    const float m1[3] = {J11 * Pm[4] + J12 * Pm[8], J11 * Pm[5] + J12 * Pm[9], J11 * Pm[6] + J12 * Pm[10]};
    // dL/dSigma' = -C G C with G = [[g_ca, g_cb/2], [g_cb/2, g_cc]]
    const float ca = sp.ca, cb = sp.cb, cc = sp.cc;
    const float h01 = 0.5f * g_cb;
    // C G
    const float t00 = ca * g_ca + cb * h01, t01 = ca * h01 + cb * g_cc;
    const float t10 = cb * g_ca + cc * h01, t11 = cb * h01 + cc * g_cc;
    const float Gs00 = -(t00 * ca + t01 * cb);
    const float Gs01 = -(t00 * cb + t01 * cc);
    const float Gs11 = -(t10 * cb + t11 * cc);
    // dL/dM = 2 Gs M Sw (2x3)
    float SM0[3], SM1[3];  // Sw m0, Sw m1
    SM0[0] = Sw[0] * m0[0] + Sw[1] * m0[1] + Sw[2] * m0[2];
    SM0[1] = Sw[1] * m0[0] + Sw[3] * m0[1] + Sw[4] * m0[2];
    SM0[2] = Sw[2] * m0[0] + Sw[4] * m0[1] + Sw[5] * m0[2];
    SM1[0] = Sw[0] * m1[0] + Sw[1] * m1[1] + Sw[2] * m1[2];
    SM1[1] = Sw[1] * m1[0] + Sw[3] * m1[1] + Sw[4] * m1[2];
    SM1[2] = Sw[2] * m1[0] + Sw[4] * m1[1] + Sw[5] * m1[2];
    float gM0[3], gM1[3];
    for (int k = 0; k < 3; ++k) {
      gM0[k] = 2.f * (Gs00 * SM0[k] + Gs01 * SM1[k]);
      gM1[k] = 2.f * (Gs01 * SM0[k] + Gs11 * SM1[k]);
    }
    // dL/dJ = dL/dM R^T (only the structurally non-zero entries)
    const float gJ00 = gM0[0] * Pm[0] + gM0[1] * Pm[1] + gM0[2] * Pm[2];
    const float gJ02 = gM0[0] * Pm[8] + gM0[1] * Pm[9] + gM0[2] * Pm[10];
    const float gJ11 = gM1[0] * Pm[4] + gM1[1] * Pm[5] + gM1[2] * Pm[6];
    const float gJ12 = gM1[0] * Pm[8] + gM1[1] * Pm[9] + gM1[2] * Pm[10];
    // dL/dmc
    const float iz2 = iz * iz;
    float gmc[3];
    gmc[0] = g_u * fx * iz;
    gmc[1] = g_v * fy * iz;
    gmc[2] = -g_u * fx * x * iz2 - g_v * fy * y * iz2 + g_z;
    gmc[2] += -gJ00 * fx * iz2 - gJ11 * fy * iz2;
    if (!clx) {
      gmc[0] += -gJ02 * fx * iz2;
      gmc[2] += 2.f * gJ02 * fx * x * iz2 * iz;
    } else {
      gmc[2] += gJ02 * fx * xh * iz2;
    }
    if (!cly) {
      gmc[1] += -gJ12 * fy * iz2;
      gmc[2] += 2.f * gJ12 * fy * y * iz2 * iz;
    } else {
      gmc[2] += gJ12 * fy * yh * iz2;
    }
    // dL/dR through the covariance: Jcol^T dL/dM, i.e. GRc[r][c] = sum_a J[a][r] gM[a][c]
    float GRc[3][3];
    for (int c2 = 0; c2 < 3; ++c2) {
      GRc[0][c2] = J00 * gM0[c2];
      GRc[1][c2] = J11 * gM1[c2];
      GRc[2][c2] = J02 * gM0[c2] + J12 * gM1[c2];
    }
    // B = R GRc^T ; dL/dphi (covariance part) = (B12 - B21, B20 - B02, B01 - B10)
    float B[3][3];
    for (int r = 0; r < 3; ++r)
      for (int c2 = 0; c2 < 3; ++c2)
        B[r][c2] = Pm[4 * r + 0] * GRc[c2][0] + Pm[4 * r + 1] * GRc[c2][1] + Pm[4 * r + 2] * GRc[c2][2];
    // SH view direction
    const float Cx = -(Pm[0] * Pm[3] + Pm[4] * Pm[7] + Pm[8] * Pm[11]);
    const float Cy = -(Pm[1] * Pm[3] + Pm[5] * Pm[7] + Pm[9] * Pm[11]);
    const float Cz = -(Pm[2] * Pm[3] + Pm[6] * Pm[7] + Pm[10] * Pm[11]);
    float dir[3] = {mu[0] - Cx, mu[1] - Cy, mu[2] - Cz};
    const float inv = rsqrtf(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
    const float n0 = dir[0] * inv, n1 = dir[1] * inv, n2 = dir[2] * inv;
    // the forward's unclamped colour (the sums of sh_colour_raw, in its
    // order), from coefficients read once
    float shv[3 * K];
    load_sh<DEG>(a.g.sh, i, shv);
    float Y[K];
    sh_basis<DEG>(n0, n1, n2, Y);
    float raw[3] = {0.5f, 0.5f, 0.5f};
#pragma unroll
    for (int k = 0; k < K; ++k) {
      raw[0] = fmaf(shv[3 * k + 0], Y[k], raw[0]);
      raw[1] = fmaf(shv[3 * k + 1], Y[k], raw[1]);
      raw[2] = fmaf(shv[3 * k + 2], Y[k], raw[2]);
    }
    float graw[3];
    for (int c2 = 0; c2 < 3; ++c2) graw[c2] = raw[c2] > 0.f ? gcol[c2] : 0.f;
    float gdir[3] = {0.f, 0.f, 0.f};
    if constexpr (DEG >= 1) {
      for (int c2 = 0; c2 < 3; ++c2) {
        if (graw[c2] == 0.f) continue;
        float cch[K];
        for (int k = 0; k < K; ++k) cch[k] = shv[3 * k + c2];
        float gg[3];
        sh_grad_dir<DEG>(cch, n0, n1, n2, gg);
        const float nd = gg[0] * n0 + gg[1] * n1 + gg[2] * n2;
        gdir[0] += graw[c2] * (gg[0] - n0 * nd) * inv;
        gdir[1] += graw[c2] * (gg[1] - n1 * nd) * inv;
        gdir[2] += graw[c2] * (gg[2] - n2 * nd) * inv;
      }
    }
    if (GAUSS && a.g_sh) {
      float* gs = a.g_sh + static_cast<int64_t>(K) * 3 * i;
      for (int k = 0; k < K; ++k)
        for (int c2 = 0; c2 < 3; ++c2)
          if (graw[c2] != 0.f) atomicAdd(gs + 3 * k + c2, graw[c2] * Y[k]);
    }
    // Gaussian gradients
    if (GAUSS && a.g_means) {
      for (int c2 = 0; c2 < 3; ++c2) {
        const float gm = Pm[c2] * gmc[0] + Pm[4 + c2] * gmc[1] + Pm[8 + c2] * gmc[2] + gdir[c2];
        atomicAdd(a.g_means + 3 * i + c2, gm);
      }
    }
    if (GAUSS && a.g_opac) atomicAdd(a.g_opac + i, g_o);
    if (GAUSS && (a.g_log_scales || a.g_quats)) {
      // dL/dSigma_w = M^T Gs M
      float Gw[3][3];
      for (int r = 0; r < 3; ++r)
        for (int c2 = 0; c2 < 3; ++c2)
          Gw[r][c2] = m0[r] * (Gs00 * m0[c2] + Gs01 * m1[c2]) + m1[r] * (Gs01 * m0[c2] + Gs11 * m1[c2]);
      const float qn = rsqrtf(q4.x * q4.x + q4.y * q4.y + q4.z * q4.z + q4.w * q4.w);
      const float w = q4.x * qn, qx = q4.y * qn, qy = q4.z * qn, qz = q4.w * qn;
      const float Rq[3][3] = {{1.f - 2.f * (qy * qy + qz * qz), 2.f * (qx * qy - w * qz), 2.f * (qx * qz + w * qy)},
                              {2.f * (qx * qy + w * qz), 1.f - 2.f * (qx * qx + qz * qz), 2.f * (qy * qz - w * qx)},
                              {2.f * (qx * qz - w * qy), 2.f * (qy * qz + w * qx), 1.f - 2.f * (qx * qx + qy * qy)}};
      const float s2[3] = {__expf(2.f * ls[0]), __expf(2.f * ls[1]), __expf(2.f * ls[2])};
      if (a.g_log_scales) {
        for (int k = 0; k < 3; ++k) {
          float acc = 0.f;
          for (int r = 0; r < 3; ++r)
            for (int c2 = 0; c2 < 3; ++c2) acc += Rq[r][k] * Gw[r][c2] * Rq[c2][k];
          atomicAdd(a.g_log_scales + 3 * i + k, 2.f * s2[k] * acc);
        }
      }
      if (a.g_quats) {
        // dL/dRq = 2 Gw Rq S^2
        float G[3][3];
        for (int r = 0; r < 3; ++r)
          for (int c2 = 0; c2 < 3; ++c2)
            G[r][c2] = 2.f * (Gw[r][0] * Rq[0][c2] + Gw[r][1] * Rq[1][c2] + Gw[r][2] * Rq[2][c2]) * s2[c2];
        const float gw = 2.f * (-qz * G[0][1] + qy * G[0][2] + qz * G[1][0] - qx * G[1][2] - qy * G[2][0] + qx * G[2][1]);
        const float gx = 2.f * (qy * G[0][1] + qz * G[0][2] + qy * G[1][0] - 2.f * qx * G[1][1] - w * G[1][2] +
                                qz * G[2][0] + w * G[2][1] - 2.f * qx * G[2][2]);
        const float gy = 2.f * (-2.f * qy * G[0][0] + qx * G[0][1] + w * G[0][2] + qx * G[1][0] + qz * G[1][2] -
                                w * G[2][0] + qz * G[2][1] - 2.f * qy * G[2][2]);
        const float gz = 2.f * (-2.f * qz * G[0][0] - w * G[0][1] + qx * G[0][2] + w * G[1][0] - 2.f * qz * G[1][1] +
                                qy * G[1][2] + qx * G[2][0] + qy * G[2][1]);
        const float dq = gw * w + gx * qx + gy * qy + gz * qz;
        atomicAdd(a.g_quats + 4 * i + 0, (gw - w * dq) * qn);
        atomicAdd(a.g_quats + 4 * i + 1, (gx - qx * dq) * qn);
        atomicAdd(a.g_quats + 4 * i + 2, (gy - qy * dq) * qn);
        atomicAdd(a.g_quats + 4 * i + 3, (gz - qz * dq) * qn);
      }
    }
    // pose tangent (rho, phi)
    gp[0] += gmc[0] + Pm[0] * gdir[0] + Pm[1] * gdir[1] + Pm[2] * gdir[2];
    gp[1] += gmc[1] + Pm[4] * gdir[0] + Pm[5] * gdir[1] + Pm[6] * gdir[2];
    gp[2] += gmc[2] + Pm[8] * gdir[0] + Pm[9] * gdir[1] + Pm[10] * gdir[2];
    gp[3] += (y * gmc[2] - z * gmc[1]) + (B[1][2] - B[2][1]);
    gp[4] += (z * gmc[0] - x * gmc[2]) + (B[2][0] - B[0][2]);
    gp[5] += (x * gmc[1] - y * gmc[0]) + (B[0][1] - B[1][0]);
  }
}

// Records of one pose per blockIdx.y, walked compacted (the in-use slots of
// the kSub sub-segments, through the prefix of their counters) by a grid of
// workgroups; each thread sums its records' pose tangents, the workgroup
// reduces them (wave sums, then four waves) and adds them once per pose.
template <int DEG, bool GAUSS>
__global__ __launch_bounds__(256) void project_bwd_kernel(ProjBackArgs a) {
  __shared__ uint32_t s_pre[kSub + 1];
  __shared__ float s_red[4][6];
  if (a.flags[0] & 3) return;
  const int pose = blockIdx.y;
  const uint32_t sub_cap = a.rec_cap / kSub;
  if (threadIdx.x < kWave) {
    const int l = threadIdx.x;
    uint32_t v = l < kSub ? min(a.pose_count[pose * kSub + l], sub_cap) : 0u;
#pragma unroll
    for (int off = 1; off < kSub; off <<= 1) {
      const uint32_t u = __shfl_up(v, off, kWave);
      if (l >= off) v += u;
    }
    if (l < kSub) s_pre[l + 1] = v;
    if (l == 0) s_pre[0] = 0;
  }
  __syncthreads();
  const uint32_t total = s_pre[kSub];
  float gp[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (uint32_t c = blockIdx.x * 256 + threadIdx.x; c < total; c += gridDim.x * 256) {
    int lo = 0, hi = kSub;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (s_pre[mid] <= c) lo = mid;
      else hi = mid;
    }
    record_grad<DEG, GAUSS>(a, pose, static_cast<uint32_t>(lo) * sub_cap + (c - s_pre[lo]), gp);
  }
  if (!a.g_pose) return;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    float v = gp[k];
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    if (lane == 0) s_red[wave][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    const int k = threadIdx.x;
    const float v = (s_red[0][k] + s_red[1][k]) + (s_red[2][k] + s_red[3][k]);
    if (v != 0.f) atomicAdd(a.g_pose + 6 * pose + k, v);
  }
}

// The gradient sums of the in-use records, cleared before the blend backward
// adds into them: a grid per pose walking the compacted slots.
__global__ __launch_bounds__(256) void zero_grad_rec_kernel(float* g, const uint32_t* pose_count, uint32_t rec_cap) {
  __shared__ uint32_t s_pre[kSub + 1];
  const int pose = blockIdx.y;
  const uint32_t sub_cap = rec_cap / kSub;
  if (threadIdx.x < kWave) {
    const int l = threadIdx.x;
    uint32_t v = l < kSub ? min(pose_count[pose * kSub + l], sub_cap) : 0u;
#pragma unroll
    for (int off = 1; off < kSub; off <<= 1) {
      const uint32_t u = __shfl_up(v, off, kWave);
      if (l >= off) v += u;
    }
    if (l < kSub) s_pre[l + 1] = v;
    if (l == 0) s_pre[0] = 0;
  }
  __syncthreads();
  const uint32_t total = s_pre[kSub];
  const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
  for (uint32_t c = blockIdx.x * 256 + threadIdx.x; c < total; c += gridDim.x * 256) {
    int lo = 0, hi = kSub;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (s_pre[mid] <= c) lo = mid;
      else hi = mid;
    }
    const uint32_t slot = static_cast<uint32_t>(lo) * sub_cap + (c - s_pre[lo]);
    float4* d = reinterpret_cast<float4*>(g + (static_cast<int64_t>(pose) * rec_cap + slot) * kGradRecStride);
    d[0] = z; d[1] = z; d[2] = z;
  }
}

void launch_zero_grad_rec(float* g, const uint32_t* pose_count, uint32_t rec_cap, int P, hipStream_t s) {
  const dim3 grid(std::min<uint32_t>((rec_cap + 255) / 256, 512), P);
  hipLaunchKernelGGL(zero_grad_rec_kernel, grid, dim3(256), 0, s, g, pose_count, rec_cap);
}

template <bool GAUSS>
static void launch_project_bwd_g(const ProjBackArgs& a, hipStream_t s) {
  // enough workgroups per pose for its slots at one record per thread, at
  // most kProjBwdBlocks (the walk strides over the rest)
  constexpr uint32_t kProjBwdBlocks = 512;
  const dim3 grid(std::min<uint32_t>((a.rec_cap + 255) / 256, kProjBwdBlocks), a.P);
  switch (a.g.sh_degree) {
    case 0: hipLaunchKernelGGL((project_bwd_kernel<0, GAUSS>), grid, dim3(256), 0, s, a); break;
    case 1: hipLaunchKernelGGL((project_bwd_kernel<1, GAUSS>), grid, dim3(256), 0, s, a); break;
    case 2: hipLaunchKernelGGL((project_bwd_kernel<2, GAUSS>), grid, dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL((project_bwd_kernel<3, GAUSS>), grid, dim3(256), 0, s, a); break;
  }
}

void launch_project_bwd(const ProjBackArgs& a, hipStream_t s) {
  // without per-Gaussian gradients the kernel carries none of their code
  if (a.g_means || a.g_opac || a.g_log_scales || a.g_quats || a.g_sh) launch_project_bwd_g<true>(a, s);
  else launch_project_bwd_g<false>(a, s);
}

}  // namespace hgsr
