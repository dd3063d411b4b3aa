// Device-side definitions shared by the HIP kernels of the splat rasterizer
// (gfx950, wave64).  Everything here is FP32; the exact per-pair expressions
// used by the forward blend and by its reverse replay live in one place so
// that both take bit-identical decisions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hgsr {

constexpr float kAlphaMin = 1.0f / 255.0f;  // blend gate
constexpr float kAlphaMax = 0.99f;          // opacity clamp
constexpr float kTMin = 1e-4f;              // transmittance stop
constexpr float kDilation = 0.3f;           // screen-space low-pass, px^2
constexpr float kGuard = 1.3f;              // Jacobian guard band, x field of view
constexpr float kRectPad = 5e-4f;           // support rectangle padding, px
constexpr float kPreReject = 1e-3f;         // exponent margin below the gate for the early reject
constexpr float kCosEps = 1e-8f;     // added to |F| |F*| in the feature cosine
constexpr int kMaxPoses = 64;               // poses per projection launch
constexpr int kSub = 32;                    // record sub-segments (and counters) per pose
constexpr int kWave = 64;

// blend launch shapes: one workgroup per (pose, tile), or a persistent grid
// pulling (pose, tile) items pose-major or tile-major from a device counter
enum { kSchedGrid = 0, kSchedPoseMajor = 1, kSchedTileMajor = 2 };
// Items a persistent workgroup claims per queue atomic: the counter is one
// device-scope address, whose atomics are performed one after another at the
// memory side, so one atomic per (pose, tile) item would serialise the launch.
constexpr int kQueueChunk = 16;

// One visible (pose, Gaussian): what the blend reads per list entry.
struct alignas(16) Splat {
  float u, v, ca, cb;   // projected mean (px), conic a, b
  float cc, o, z;       // conic c, opacity, camera z
  uint32_t gid;         // Gaussian index
  float r, g, b;        // colour
  float pmin;           // -ln(255 o): exponent at which o e^power = 1/255
};

struct GaussArgs {
  const float* means;
  const float* log_scales;
  const float* quats;
  const float* opac;
  const float* sh;
  const uint16_t* feat;
  int64_t n;
  int32_t sh_degree;
  int32_t feat_dim;
  int32_t n_parts;
  const int64_t* part_offsets;
  const float* part_bounds;
};

struct CamArgs {
  float fx, fy, cx, cy;
  int32_t W, H;
  float near_z;
  float limx, limy;      // guard band on x/z and y/z
  int32_t tile, tile_shift;
  int32_t ntx, nty, tiles_per_pose;
};

// ---------------------------------------------------------------- helpers
__device__ __forceinline__ float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  uint32_t b = __float_as_uint(f);
  if ((b & 0x7fffffffu) > 0x7f800000u) return static_cast<uint16_t>((b >> 16) | 0x40);  // quiet NaN
  b += 0x7fffu + ((b >> 16) & 1u);
  return static_cast<uint16_t>(b >> 16);
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Rotate a value by n lanes within each row of 16 lanes (DPP row_ror).
template <int N>
__device__ __forceinline__ float row_ror(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x120 | N, 0xf, 0xf, false));
}

// Sum over the row of 16 lanes, in every lane of the row.
__device__ __forceinline__ float row_sum16(float v) {
  v += row_ror<8>(v);
  v += row_ror<4>(v);
  v += row_ror<2>(v);
  v += row_ror<1>(v);
  return v;
}

// Sums ten per-lane values over the wave and atomically adds total v to
// dst[v] (dst in LDS or global memory).  A reduce-scatter: the lane-half
// exchange (v_permlane32_swap) pairs value i with value 5 + i, so lanes 0-31
// carry values 0-4 and lanes 32-63 values 5-9; the row exchange
// (v_permlane16_swap) pairs them again, leaving three partial sums per lane
// that a 16-lane DPP row sum completes.  Totals end in lanes 0, 16, 32, 48:
// row r = lane / 16 holds values 5 (r / 2) + (r % 2), 5 (r / 2) + 2 + (r % 2)
// and, for even rows, 5 (r / 2) + 4.
__device__ __forceinline__ void wave_add10(const float g[10], float* dst) {
  float b[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    const auto s = __builtin_amdgcn_permlane32_swap(__float_as_uint(g[i]), __float_as_uint(g[5 + i]), false, false);
    b[i] = __uint_as_float(s[0]) + __uint_as_float(s[1]);
  }
  const auto s0 = __builtin_amdgcn_permlane16_swap(__float_as_uint(b[0]), __float_as_uint(b[1]), false, false);
  const auto s1 = __builtin_amdgcn_permlane16_swap(__float_as_uint(b[2]), __float_as_uint(b[3]), false, false);
  const auto s2 = __builtin_amdgcn_permlane16_swap(__float_as_uint(b[4]), __float_as_uint(b[4]), false, false);
  const float c0 = row_sum16(__uint_as_float(s0[0]) + __uint_as_float(s0[1]));
  const float c1 = row_sum16(__uint_as_float(s1[0]) + __uint_as_float(s1[1]));
  const float c2 = row_sum16(__uint_as_float(s2[0]) + __uint_as_float(s2[1]));
  const int lane = threadIdx.x & (kWave - 1);
  if ((lane & 15) == 0) {
    const int base = 5 * (lane >> 5), odd = (lane >> 4) & 1;
    atomicAdd(dst + base + odd, c0);
    atomicAdd(dst + base + 2 + odd, c1);
    if (!odd) atomicAdd(dst + base + 4, c2);
  }
}

// The same for eight of the ten sums (0-4 and 7-9; 5 and 6 are left alone):
// each value meets the same reduction tree as in wave_add10 (lane pairs 32
// apart, then 16 apart, then a row sum), so the eight results have the same
// bits.
__device__ __forceinline__ void wave_add8(const float g[10], float* dst) {
  const float lo[4] = {g[0], g[1], g[2], g[3]}, hi[4] = {g[4], g[7], g[8], g[9]};
  float b[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const auto s = __builtin_amdgcn_permlane32_swap(__float_as_uint(lo[i]), __float_as_uint(hi[i]), false, false);
    b[i] = __uint_as_float(s[0]) + __uint_as_float(s[1]);
  }
  const auto s0 = __builtin_amdgcn_permlane16_swap(__float_as_uint(b[0]), __float_as_uint(b[1]), false, false);
  const auto s1 = __builtin_amdgcn_permlane16_swap(__float_as_uint(b[2]), __float_as_uint(b[3]), false, false);
  const float c0 = row_sum16(__uint_as_float(s0[0]) + __uint_as_float(s0[1]));
  const float c1 = row_sum16(__uint_as_float(s1[0]) + __uint_as_float(s1[1]));
  const int lane = threadIdx.x & (kWave - 1);
  if ((lane & 15) == 0) {
    const int half = lane >> 5, odd = (lane >> 4) & 1;
    atomicAdd(dst + (half ? (odd ? 7 : 4) : odd), c0);       // g0, g1 | g4, g7
    atomicAdd(dst + (half ? (odd ? 9 : 8) : 2 + odd), c1);   // g2, g3 | g8, g9
  }
}

// World covariance Sigma_w = R_q diag(exp(2 ls)) R_q^T, (w,x,y,z) quaternion
// normalised here.  Returns xx, xy, xz, yy, yz, zz.
__device__ __forceinline__ void cov3_from(const float4 q4, const float ls[3], float S[6]) {
  const float qn = rsqrtf(q4.x * q4.x + q4.y * q4.y + q4.z * q4.z + q4.w * q4.w);
  const float w = q4.x * qn, x = q4.y * qn, y = q4.z * qn, z = q4.w * qn;
  const float R[9] = {1.f - 2.f * (y * y + z * z), 2.f * (x * y - w * z), 2.f * (x * z + w * y),
                      2.f * (x * y + w * z), 1.f - 2.f * (x * x + z * z), 2.f * (y * z - w * x),
                      2.f * (x * z - w * y), 2.f * (y * z + w * x), 1.f - 2.f * (x * x + y * y)};
  const float s0 = __expf(2.f * ls[0]), s1 = __expf(2.f * ls[1]), s2 = __expf(2.f * ls[2]);
  S[0] = R[0] * R[0] * s0 + R[1] * R[1] * s1 + R[2] * R[2] * s2;
  S[1] = R[0] * R[3] * s0 + R[1] * R[4] * s1 + R[2] * R[5] * s2;
  S[2] = R[0] * R[6] * s0 + R[1] * R[7] * s1 + R[2] * R[8] * s2;
  S[3] = R[3] * R[3] * s0 + R[4] * R[4] * s1 + R[5] * R[5] * s2;
  S[4] = R[3] * R[6] * s0 + R[4] * R[7] * s1 + R[5] * R[8] * s2;
  S[5] = R[6] * R[6] * s0 + R[7] * R[7] * s1 + R[8] * R[8] * s2;
}

// Camera-space mean m_c = R mu + t.
__device__ __forceinline__ void to_camera(const float* P, const float mu[3], float mc[3]) {
  mc[0] = fmaf(P[0], mu[0], fmaf(P[1], mu[1], fmaf(P[2], mu[2], P[3])));
  mc[1] = fmaf(P[4], mu[0], fmaf(P[5], mu[1], fmaf(P[6], mu[2], P[7])));
  mc[2] = fmaf(P[8], mu[0], fmaf(P[9], mu[1], fmaf(P[10], mu[2], P[11])));
}

struct Footprint {
  float u, v;           // projected mean
  float sxx, sxy, syy;  // Sigma' with dilation
  float ca, cb, cc;     // conic
  int px0, px1, py0, py1;
};

// EWA footprint of a Gaussian with camera-space mean mc and world covariance
// S (pose P = [R|t] row-major).  k2 = 2 ln(255 o).  Returns false when the
// support rectangle misses the image (or the covariance degenerates).
__device__ __forceinline__ bool footprint(const float* P, const float mc[3], const float S[6], float k2,
                                          const CamArgs& c, Footprint& f) {
  const float z = mc[2];
  const float iz = 1.0f / z;
  const float xz = mc[0] / z, yz = mc[1] / z;
  const float xh = fminf(fmaxf(xz, -c.limx), c.limx);
  const float yh = fminf(fmaxf(yz, -c.limy), c.limy);
  const float j00 = c.fx * iz, j02 = -c.fx * xh * iz;
  const float j11 = c.fy * iz, j12 = -c.fy * yh * iz;
  // rows of M = J R
  const float a0 = j00 * P[0] + j02 * P[8], a1 = j00 * P[1] + j02 * P[9], a2 = j00 * P[2] + j02 * P[10];
  const float b0 = j11 * P[4] + j12 * P[8], b1 = j11 * P[5] + j12 * P[9], b2 = j11 * P[6] + j12 * P[10];
  // S a, S b
  const float sa0 = S[0] * a0 + S[1] * a1 + S[2] * a2;
  const float sa1 = S[1] * a0 + S[3] * a1 + S[4] * a2;
  const float sa2 = S[2] * a0 + S[4] * a1 + S[5] * a2;
  const float sb0 = S[0] * b0 + S[1] * b1 + S[2] * b2;
  const float sb1 = S[1] * b0 + S[3] * b1 + S[4] * b2;
  const float sb2 = S[2] * b0 + S[4] * b1 + S[5] * b2;
  f.sxx = a0 * sa0 + a1 * sa1 + a2 * sa2 + kDilation;
  f.sxy = b0 * sa0 + b1 * sa1 + b2 * sa2;
  f.syy = b0 * sb0 + b1 * sb1 + b2 * sb2 + kDilation;
  const float det = f.sxx * f.syy - f.sxy * f.sxy;
  if (!(det > 0.f)) return false;
  const float idet = 1.0f / det;
  f.ca = f.syy * idet;
  f.cb = -f.sxy * idet;
  f.cc = f.sxx * idet;
  f.u = fmaf(c.fx, xz, c.cx);
  f.v = fmaf(c.fy, yz, c.cy);
  const float rx = sqrtf(k2 * f.sxx), ry = sqrtf(k2 * f.syy);
  const float bx0 = f.u - rx - 0.5f - kRectPad, bx1 = f.u + rx - 0.5f + kRectPad;
  const float by0 = f.v - ry - 0.5f - kRectPad, by1 = f.v + ry - 0.5f + kRectPad;
  const float wm1 = static_cast<float>(c.W - 1), hm1 = static_cast<float>(c.H - 1);
  if (!(bx1 >= 0.f && by1 >= 0.f && bx0 <= wm1 && by0 <= hm1)) return false;
  const float x0 = ceilf(fmaxf(bx0, 0.f)), x1 = floorf(fminf(bx1, wm1));
  const float y0 = ceilf(fmaxf(by0, 0.f)), y1 = floorf(fminf(by1, hm1));
  if (!(x0 <= x1 && y0 <= y1)) return false;
  f.px0 = static_cast<int>(x0); f.px1 = static_cast<int>(x1);
  f.py0 = static_cast<int>(y0); f.py1 = static_cast<int>(y1);
  return true;
}

// Conservative early test before the covariance is formed: the support
// half-width footprint() finds, sqrt(k2 (a^T Sigma a + dilation)) with
// a = row 0 of J R, is at most sqrt(k2 (|a|^2 s_max^2 + dilation)) where
// |a|^2 = (fx/z)^2 (1 + xh^2) for a rotation R and s_max is the largest
// scale (likewise for y).  Returns false only when that larger rectangle,
// widened by 0.1% and one pixel for rounding, misses the image; such a
// Gaussian fails footprint() too.
__device__ __forceinline__ bool maybe_visible(const float mc[3], float s2max, float k2, const CamArgs& c) {
  // hardware reciprocal and square root (about 1 ulp): the widening below
  // covers their error many times over
  const float iz = __builtin_amdgcn_rcpf(mc[2]);
  const float xz = mc[0] * iz, yz = mc[1] * iz;
  const float xh = fminf(fmaxf(xz, -c.limx), c.limx);
  const float yh = fminf(fmaxf(yz, -c.limy), c.limy);
  const float gx = c.fx * iz, gy = c.fy * iz;
  const float rx = 1.001f * __builtin_amdgcn_sqrtf(k2 * fmaf(gx * gx * fmaf(xh, xh, 1.f), s2max, kDilation)) + 1.f;
  const float ry = 1.001f * __builtin_amdgcn_sqrtf(k2 * fmaf(gy * gy * fmaf(yh, yh, 1.f), s2max, kDilation)) + 1.f;
  const float u = fmaf(c.fx, xz, c.cx), v = fmaf(c.fy, yz, c.cy);
  return u + rx >= 0.f && v + ry >= 0.f && u - rx <= static_cast<float>(c.W) && v - ry <= static_cast<float>(c.H);
}

// Real spherical harmonics up to degree 3 (Condon-Shortley phase, index
// l^2 + l + m) at unit direction (x, y, z), with the standard normalisation
// sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!) (x sqrt 2 for m != 0).
template <int DEG>
__device__ __forceinline__ void sh_basis(float x, float y, float z, float Y[(DEG + 1) * (DEG + 1)]) {
  Y[0] = 0.28209479177387814f;
  if constexpr (DEG >= 1) {
    Y[1] = -0.48860251190291987f * y;
    Y[2] = 0.48860251190291987f * z;
    Y[3] = -0.48860251190291987f * x;
  }
  if constexpr (DEG >= 2) {
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = 1.0925484305920792f * x * y;
    Y[5] = -1.0925484305920792f * y * z;
    Y[6] = 0.31539156525252005f * (2.f * zz - xx - yy);
    Y[7] = -1.0925484305920792f * x * z;
    Y[8] = 0.5462742152960396f * (xx - yy);
    if constexpr (DEG >= 3) {
      Y[9] = -0.5900435899266435f * y * (3.f * xx - yy);
      Y[10] = 2.890611442640554f * x * y * z;
      Y[11] = -0.4570457994644658f * y * (4.f * zz - xx - yy);
      Y[12] = 0.3731763325901154f * z * (2.f * zz - 3.f * xx - 3.f * yy);
      Y[13] = -0.4570457994644658f * x * (4.f * zz - xx - yy);
      Y[14] = 1.445305721320277f * z * (xx - yy);
      Y[15] = -0.5900435899266435f * x * (xx - 3.f * yy);
    }
  }
}

// Unclamped SH colour (before max(0, .)) of Gaussian `i` seen along dir.
template <int DEG>
__device__ __forceinline__ void sh_colour_raw(const float* sh, int64_t i, float dx, float dy, float dz,
                                              float rgb[3]) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  float Y[K];
  sh_basis<DEG>(dx, dy, dz, Y);
  const float* c = sh + static_cast<int64_t>(K) * 3 * i;
  float r = 0.5f, g = 0.5f, b = 0.5f;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    r = fmaf(c[3 * k + 0], Y[k], r);
    g = fmaf(c[3 * k + 1], Y[k], g);
    b = fmaf(c[3 * k + 2], Y[k], b);
  }
  rgb[0] = r; rgb[1] = g; rgb[2] = b;
}

// The per-pair exponent -q/2 of the blend, shared bit for bit by the forward
// and the reverse replay.
__device__ __forceinline__ float pair_power(float dx, float dy, float ca, float cb, float cc) {
  const float quad = fmaf(ca, dx * dx, cc * (dy * dy));
  return fmaf(-0.5f, quad, -cb * (dx * dy));
}

__device__ __forceinline__ float pair_alpha(float o, float power) { return fminf(kAlphaMax, o * __expf(power)); }

// Records of pose p live in kSub sub-segments of rec_cap / kSub slots; slot
// `slot` is in use when its offset within its sub-segment is below that
// sub-segment's counter.
__device__ __forceinline__ bool rec_in_use(const uint32_t* sub_count, uint32_t rec_cap, int pose, uint32_t slot) {
  const uint32_t sub_cap = rec_cap / kSub;
  const uint32_t s = slot / sub_cap;
  return slot - s * sub_cap < min(sub_count[pose * kSub + s], sub_cap);
}

// Bitonic sort of n <= 256 (key, value) pairs by one wave, 4 per lane in
// registers: partners across lanes by shuffle, across a lane's registers by
// swap.  Keys are unique except the ~0 padding.  Every lane of the wave must
// call it; on return lane l holds sorted elements q*64 + l in key[q], val[q].
__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m) {
  const uint32_t lo = __shfl_xor(static_cast<uint32_t>(v), m, kWave);
  const uint32_t hi = __shfl_xor(static_cast<uint32_t>(v >> 32), m, kWave);
  return (static_cast<uint64_t>(hi) << 32) | lo;
}

__device__ __forceinline__ int wave_sort256(const uint64_t* keys, const uint32_t* vals, uint32_t n, uint64_t key[4],
                                            uint32_t val[4]) {
  const int lane = threadIdx.x & (kWave - 1);
  int R = 1;
  while (R * kWave < static_cast<int>(n)) R <<= 1;  // 1, 2 or 4 registers
  const uint32_t m = static_cast<uint32_t>(R) * kWave;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint32_t e = q * kWave + lane;
    key[q] = ~0ull;
    val[q] = 0;
    if (q < R && e < n) {
      key[q] = keys[e];
      val[q] = vals[e];
    }
  }
  for (uint32_t k = 2; k <= m; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      if (j >= kWave) {
        const int rj = static_cast<int>(j / kWave);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int q2 = q ^ rj;
          if (q >= R || q2 <= q) continue;
          const uint32_t e = q * kWave + lane;
          const bool up = (e & k) == 0;
          if ((key[q] > key[q2]) == up) {
            const uint64_t tk = key[q]; key[q] = key[q2]; key[q2] = tk;
            const uint32_t tv = val[q]; val[q] = val[q2]; val[q2] = tv;
          }
        }
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (q >= R) continue;
          const uint64_t ok = shfl_xor_u64(key[q], static_cast<int>(j));
          const uint32_t ov = __shfl_xor(val[q], static_cast<int>(j), kWave);
          const uint32_t e = q * kWave + lane;
          const bool up = (e & k) == 0;
          const bool lower = (e & j) == 0;
          const bool take = lower == up ? (ok < key[q]) : (ok > key[q]);
          if (take) {
            key[q] = ok;
            val[q] = ov;
          }
        }
      }
    }
  }
  return R;
}

template <int TILE>
struct BlendShape {
  static constexpr int kThreads = TILE == 8 ? 64 : 256;
  static constexpr int kBatch = kThreads < 128 ? kThreads : 128;  // splats staged per round
  static constexpr int kWaves = kThreads / kWave;
  // a wave's pixel block: 8x8 (16x16 with 4 pixels per lane at tile 32)
  static constexpr int kBlockW = TILE == 32 ? 16 : 8;
  static constexpr int kBlockH = TILE * TILE / kWaves / kBlockW;
  static constexpr int kPPT = kBlockW * kBlockH / kWave;  // pixels per lane
  static constexpr int kBlocksX = TILE / kBlockW;
};

// Smallest conic distance q(p - mean) = a dx^2 + 2 b dx dy + c dy^2 over the
// rectangle [x0, x1] x [y0, y1] (ia = 1/a, ic = 1/c).  q is convex: 0 when
// the mean is inside, otherwise the smallest of the four edge minima, each a
// one-variable quadratic minimised at its clamped stationary point.
__device__ __forceinline__ float min_q_box(float a, float b, float c, float ia, float ic, float u, float v, float x0,
                                           float x1, float y0, float y1) {
  if (u >= x0 && u <= x1 && v >= y0 && v <= y1) return 0.f;
  float best = 3.4e38f;
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const float dx = (e ? x1 : x0) - u;
    const float dy = fminf(fmaxf(-b * dx * ic, y0 - v), y1 - v);
    best = fminf(best, fmaf(a * dx, dx, fmaf(2.f * b * dx, dy, c * dy * dy)));
  }
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const float dy = (e ? y1 : y0) - v;
    const float dx = fminf(fmaxf(-b * dy * ia, x0 - u), x1 - u);
    best = fminf(best, fmaf(a * dx, dx, fmaf(2.f * b * dx, dy, c * dy * dy)));
  }
  return best;
}

// Listing margins, wider than FP32 rounding of the mean (1e-4 px at 2000 px)
// and of q: rectangles grow by kListGrow px, the threshold k^2 by a relative
// kListSlack plus 10 kListSlack.
constexpr float kListGrow = 5e-4f;
constexpr float kListSlack = 1e-5f;

// Whether a splat (mean u, v; conic a, b, c; k2 = 2 ln(255 o)) meets the
// rectangle of pixel centres [x0 + 0.5, x1 - 0.5] x [y0 + 0.5, y1 - 0.5]
// (pixel-edge coordinates x0..x1, y0..y1), with the listing margins.
struct SplatShape {
  float u, v, a, b, c, ia, ic, thr;
};
__device__ __forceinline__ SplatShape splat_shape(float u, float v, float a, float b, float c, float k2) {
  return SplatShape{u, v, a, b, c, 1.f / a, 1.f / c, fmaf(k2, kListSlack, k2) + 10.f * kListSlack};
}
__device__ __forceinline__ bool meets_centres(const SplatShape& s, float x0, float x1, float y0, float y1) {
  return min_q_box(s.a, s.b, s.c, s.ia, s.ic, s.u, s.v, x0 + (0.5f - kListGrow), x1 - (0.5f - kListGrow),
                   y0 + (0.5f - kListGrow), y1 - (0.5f - kListGrow)) <= s.thr;
}
// Tiles of row ty whose pixel-centre rectangles meet the support ellipse:
// [*ta, *tb] within [tx0, tx1] (empty when *ta > *tb).  Equivalent to
// tile_meets on each tile of the row, at two square roots per row: within
// the row's band of pixel-centre y the ellipse's x-extent is an interval,
// whose right end x_r(dy) = (-b dy + sqrt(a thr - det dy^2)) / a is concave
// in dy with its maximum at dy = -b sqrt(thr / (c det)) (and the left end
// mirrors it), so both ends are evaluated at that point clamped to the band.
__device__ __forceinline__ void row_span(const SplatShape& s, int ty, int tile, int W, int H, int tx0, int tx1,
                                         int* ta, int* tb) {
  const float det = s.a * s.c - s.b * s.b;
  const float ymax = sqrtf(s.a * s.thr / det);
  const float lo = fmaxf(static_cast<float>(ty * tile) + (0.5f - kListGrow) - s.v, -ymax);
  const float hi = fminf(static_cast<float>(min((ty + 1) * tile, H)) - (0.5f - kListGrow) - s.v, ymax);
  if (!(lo <= hi)) {
    *ta = 1;
    *tb = 0;
    return;
  }
  const float dyr = -s.b * sqrtf(s.thr / (s.c * det));
  const float dr = fminf(fmaxf(dyr, lo), hi), dl = fminf(fmaxf(-dyr, lo), hi);
  const float xr = s.u + (-s.b * dr + sqrtf(fmaxf(s.a * s.thr - det * dr * dr, 0.f))) * s.ia;
  const float xl = s.u + (-s.b * dl - sqrtf(fmaxf(s.a * s.thr - det * dl * dl, 0.f))) * s.ia;
  const float inv = 1.f / static_cast<float>(tile);
  int a = static_cast<int>(ceilf((xl + (0.5f - kListGrow)) * inv - 1.f));
  int b = static_cast<int>(floorf((xr - (0.5f - kListGrow)) * inv));
  if (xl > static_cast<float>(W) - (0.5f - kListGrow)) b = -1;  // right of the last pixel centre
  *ta = max(a, tx0);
  *tb = min(b, tx1);
}

// Tile-list entries carry the record index in the low kRecBits bits and, in
// the top four, which of the tile's blend blocks (the waves' pixel blocks:
// one 8x8 block at tile 8, 2 x 2 blocks of tile/2 otherwise) the splat's
// support meets, so the blend stages no geometry test.
constexpr int kRecBits = 28;
constexpr uint32_t kRecMask = (1u << kRecBits) - 1u;
__device__ __forceinline__ uint32_t block_mask(const SplatShape& s, int tx, int ty, int tile) {
  if (tile == 8) return 1u;
  const int h = tile / 2;
  uint32_t m = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const float x0 = static_cast<float>(tx * tile + (w & 1) * h), y0 = static_cast<float>(ty * tile + (w >> 1) * h);
    if (meets_centres(s, x0, x0 + h, y0, y0 + h)) m |= 1u << w;
  }
  return m;
}

// Tile (tx, ty) of a camera: its pixel-centre rectangle clipped to the image.
__device__ __forceinline__ bool tile_meets(const SplatShape& s, int tx, int ty, int tile, int W, int H) {
  return meets_centres(s, static_cast<float>(tx * tile), static_cast<float>(min((tx + 1) * tile, W)),
                       static_cast<float>(ty * tile), static_cast<float>(min((ty + 1) * tile, H)));
}


// MI355X dispatches workgroup i of a launch to accelerator die (XCD)
// i % kXcds, and each XCD has its own L2.  Renumbering the workgroups so that
// each XCD takes one contiguous range of (pose, tile) items keeps
// horizontally adjacent tiles -- which write the two halves of the same
// output cache lines and read many of the same splats -- in one L2.  The map
// is a permutation of [0, n), so results do not depend on the dispatch
// order.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_item(int b, int n) {
  const int x = b % kXcds, k = b / kXcds;
  const int per = n / kXcds, rem = n % kXcds;
  return x * per + min(x, rem) + k;
}

constexpr int kWaveSortCap = 256;   // lists this short are sorted by one wave

// Tile-id bits of a pose-major tile index (for key packing).
__device__ __forceinline__ uint32_t zbits(float z) { return __float_as_uint(z); }

}  // namespace hgsr
