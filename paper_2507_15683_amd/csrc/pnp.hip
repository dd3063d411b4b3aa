// 2D-3D pose solve of the dense stage (Sec. 3.4, Eq. 10) and Algorithm 2's
// pose consistency check.
//
// RANSAC over given minimal samples: pnp_hyp_kernel solves each 3-point
// sample by Gauss-Newton steps from the prior pose (one thread per
// hypothesis, FP64 -- a 3-point system is exactly determined, its normal
// matrix often ill-conditioned, and the singularity test needs the range --
// 6x6 Cholesky); pnp_score_mfma_kernel counts every hypothesis' inliers
// (reprojection error below tau, positive depth), the per-pair transform on
// the matrix cores; pnp_select_kernel takes the best (ties: lowest index).  The
// refinement (the truncated quadratic min(e^2, tau^2) of Eq. 10) alternates
// pnp_normal_kernel -- per point: inlier test, 2x6 Jacobian of the
// reprojection under the left perturbation, accumulation of J^T J and J^T r,
// reduced per workgroup in a fixed order -- and pnp_update_kernel, which sums
// the workgroup partials in FP64 in a fixed order, solves the 6x6 system and
// applies T <- Exp(delta) T on the device (no host round trip, capturable).
#include "hgsr_device.hpp"
#include "launch.hpp"

namespace hgsr {

// ------------------------------------------------------------ small algebra
template <class F>
__device__ __forceinline__ void se3_exp_left(const F xi[6], F T[12]) {
  // T <- Exp(xi) T, xi = (rho, phi): Rodrigues rotation, V rho translation
  const F wx = xi[3], wy = xi[4], wz = xi[5];
  const F th2 = wx * wx + wy * wy + wz * wz;
  F a, b, c;
  if (th2 < F(1e-12)) {
    a = F(1) - th2 / F(6);
    b = F(0.5) - th2 / F(24);
    c = F(1) / F(6) - th2 / F(120);
  } else {
    const F th = sqrt(th2);
    a = sin(th) / th;
    b = (F(1) - cos(th)) / th2;
    c = (th - sin(th)) / (th2 * th);
  }
  // K = hat(w), K^2 = w w^T - th2 I
  const F Kw[9] = {0, -wz, wy, wz, 0, -wx, -wy, wx, 0};
  F K2[9];
  const F w[3] = {wx, wy, wz};
  for (int r = 0; r < 3; ++r)
    for (int q = 0; q < 3; ++q) K2[3 * r + q] = w[r] * w[q] - (r == q ? th2 : F(0));
  F R[9], V[9];
  for (int k = 0; k < 9; ++k) {
    const F I = (k % 4 == 0) ? F(1) : F(0);
    R[k] = I + a * Kw[k] + b * K2[k];
    V[k] = I + b * Kw[k] + c * K2[k];
  }
  F tr[3];
  for (int r = 0; r < 3; ++r) tr[r] = V[3 * r] * xi[0] + V[3 * r + 1] * xi[1] + V[3 * r + 2] * xi[2];
  F out[12];
  for (int r = 0; r < 3; ++r) {
    for (int q = 0; q < 4; ++q)
      out[4 * r + q] = R[3 * r] * T[q] + R[3 * r + 1] * T[4 + q] + R[3 * r + 2] * T[8 + q];
    out[4 * r + 3] += tr[r];
  }
  for (int k = 0; k < 12; ++k) T[k] = out[k];
}

// Residual and Jacobian rows of one correspondence under T (left
// perturbation): r = pi(K T X) - p; J = dpi/dXc [I, -[Xc]x].  Computed
// whatever the depth (a hypothesis' Gauss-Newton step uses every sample
// point); returns whether the point is in front of the camera.
template <class F>
__device__ __forceinline__ bool reproj_rows(const F T[12], F fx, F fy, F cx, F cy, const F X[3], F pu, F pv,
                                            F r[2], F J[2][6]) {
  const F x = T[0] * X[0] + T[1] * X[1] + T[2] * X[2] + T[3];
  const F y = T[4] * X[0] + T[5] * X[1] + T[6] * X[2] + T[7];
  const F z = T[8] * X[0] + T[9] * X[1] + T[10] * X[2] + T[11];
  const F iz = F(1) / z;
  r[0] = fx * x * iz + cx - pu;
  r[1] = fy * y * iz + cy - pv;
  const F a0 = fx * iz, a2 = -fx * x * iz * iz;
  const F b1 = fy * iz, b2 = -fy * y * iz * iz;
  // row u: [a0, 0, a2] [I | -[Xc]x]
  J[0][0] = a0; J[0][1] = 0; J[0][2] = a2;
  J[0][3] = a2 * y;            // a0*0 + 0*(-z) + a2*y
  J[0][4] = a0 * z - a2 * x;
  J[0][5] = -a0 * y;
  J[1][0] = 0; J[1][1] = b1; J[1][2] = b2;
  J[1][3] = -b1 * z + b2 * y;
  J[1][4] = -b2 * x;
  J[1][5] = b1 * x;
  return z > F(0);
}

// Cholesky solve of the packed symmetric 6x6 system A x = b (upper triangle
// row by row, 21 values).  Returns false when a pivot is not positive
// relative to the matrix scale.
template <class F>
__device__ __forceinline__ bool chol6(const F A21[21], const F b[6], F x[6], F rel_eps) {
  F L[6][6];
  F scale = F(0);
  {
    int k = 0;
    for (int i = 0; i < 6; ++i)
      for (int j = i; j < 6; ++j, ++k) {
        L[j][i] = A21[k];
        if (i == j) scale = fmax(scale, A21[k]);
      }
  }
  for (int j = 0; j < 6; ++j) {
    F d = L[j][j];
    for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
    if (!(d > rel_eps * scale)) return false;
    const F s = sqrt(d);
    L[j][j] = s;
    for (int i = j + 1; i < 6; ++i) {
      F v = L[i][j];
      for (int k = 0; k < j; ++k) v -= L[i][k] * L[j][k];
      L[i][j] = v / s;
    }
  }
  F y[6];
  for (int i = 0; i < 6; ++i) {
    F v = b[i];
    for (int k = 0; k < i; ++k) v -= L[i][k] * y[k];
    y[i] = v / L[i][i];
  }
  for (int i = 5; i >= 0; --i) {
    F v = y[i];
    for (int k = i + 1; k < 6; ++k) v -= L[k][i] * x[k];
    x[i] = v / L[i][i];
  }
  return true;
}

template <class F>
__device__ __forceinline__ void accumulate_normal(const F r[2], const F J[2][6], F A21[21], F b[6]) {
  int k = 0;
  for (int i = 0; i < 6; ++i)
    for (int j = i; j < 6; ++j, ++k) A21[k] += J[0][i] * J[0][j] + J[1][i] * J[1][j];
  for (int i = 0; i < 6; ++i) b[i] += J[0][i] * r[0] + J[1][i] * r[1];
}

// ------------------------------------------------------------ hypotheses
__global__ void pnp_hyp_kernel(PnpArgs a) {
  const int h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= a.n_hyp) return;
  double T[12];
  for (int k = 0; k < 12; ++k) T[k] = a.pose0[k];
  int s[3];
  bool ok = true;
  for (int q = 0; q < 3; ++q) {
    s[q] = a.samples[3 * h + q];
    ok &= s[q] >= 0 && s[q] < a.n;
  }
  for (int it = 0; ok && it < a.gn_iters; ++it) {
    double A21[21] = {}, b[6] = {};
    for (int q = 0; q < 3; ++q) {
      const double X[3] = {a.x3d[3 * s[q]], a.x3d[3 * s[q] + 1], a.x3d[3 * s[q] + 2]};
      double r[2], J[2][6];
      reproj_rows<double>(T, a.fx, a.fy, a.cx, a.cy, X, a.p2d[2 * s[q]], a.p2d[2 * s[q] + 1], r, J);
      accumulate_normal(r, J, A21, b);
    }
    double nb[6], delta[6];
    for (int i = 0; i < 6; ++i) nb[i] = -b[i];
    if (!chol6(A21, nb, delta, 1e-12)) {  // singular (or not finite): invalid sample
      ok = false;
      break;
    }
    se3_exp_left(delta, T);
  }
  for (int k = 0; k < 12; ++k) a.hyp[12 * h + k] = static_cast<float>(T[k]);
  a.counts[h] = ok ? 0 : -1;
}

// ------------------------------------------------------------ scoring

// Inlier counts with the per-pair transform on the matrix cores: for 16
// hypotheses x 16 correspondences, (u, v, z) = (K [R | t] / tau) [X, Y, Z, 1]
// is three 16x16x4 FP32 products (v_mfma_f32_16x16x4_f32: lane l holds
// A[l % 16][l / 16], B[l / 16][l % 16] and D[4 (l / 16) + i][l % 16]); the
// VALU keeps the residual numerators, the squared error against z^2 and the
// count (~8 operations per pair instead of ~18 with the transform on the
// VALU); integer counts summed per workgroup in LDS, then one global atomic
// per (workgroup, hypothesis), so they do not depend on scheduling.  A workgroup stages 1,024
// correspondences in LDS and its four waves take 16 hypotheses each.
typedef float floatx4 __attribute__((ext_vector_type(4)));
constexpr int kMfPoints = 1024;
constexpr int kMfHyps = 64;

__global__ __launch_bounds__(256) void pnp_score_mfma_kernel(PnpArgs a) {
  // per correspondence X, Y, Z, 1 (all 0 past the end: z = 0 never counts),
  // interleaved so that the 64 lanes' B operands are 64 consecutive words
  __shared__ float s_b[kMfPoints][4];
  __shared__ float s_q[kMfPoints][2];  // p_u / tau, p_v / tau
  __shared__ int32_t s_c[kMfHyps];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t p0 = static_cast<int64_t>(blockIdx.x) * kMfPoints;
  const float it = 1.f / a.tau;
  for (int e = tid; e < kMfPoints; e += 256) {
    const int64_t i = p0 + e;
    const bool ok = i < a.n;
    s_b[e][0] = ok ? a.x3d[3 * i] : 0.f;
    s_b[e][1] = ok ? a.x3d[3 * i + 1] : 0.f;
    s_b[e][2] = ok ? a.x3d[3 * i + 2] : 0.f;
    s_b[e][3] = ok ? 1.f : 0.f;
    s_q[e][0] = ok ? a.p2d[2 * i] * it : 0.f;
    s_q[e][1] = ok ? a.p2d[2 * i + 1] * it : 0.f;
  }
  if (tid < kMfHyps) s_c[tid] = 0;
  // this lane's A entries: hypothesis row lane % 16 of the wave's 16, column k = lane / 16
  const int r = lane & 15, k = lane >> 4, col = lane & 15;
  const int h = blockIdx.y * kMfHyps + w * 16 + r;
  float au = 0.f, av = 0.f, az = 0.f;
  if (h < a.n_hyp) {
    const float* T = a.hyp + 12 * static_cast<int64_t>(h);
    au = (a.fx * T[k] + a.cx * T[8 + k]) * it;
    av = (a.fy * T[4 + k] + a.cy * T[8 + k]) * it;
    az = T[8 + k];
  }
  __syncthreads();
  int cnt[4] = {0, 0, 0, 0};
  const floatx4 zero = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
  for (int t = 0; t < kMfPoints; t += 16) {
    const float b = s_b[t + col][k];
    const float qu = s_q[t + col][0], qv = s_q[t + col][1];
    const floatx4 U = __builtin_amdgcn_mfma_f32_16x16x4f32(au, b, zero, 0, 0, 0);
    const floatx4 V = __builtin_amdgcn_mfma_f32_16x16x4f32(av, b, zero, 0, 0, 0);
    const floatx4 Z = __builtin_amdgcn_mfma_f32_16x16x4f32(az, b, zero, 0, 0, 0);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float du = fmaf(-qu, Z[q], U[q]), dv = fmaf(-qv, Z[q], V[q]);
      cnt[q] += (Z[q] > 0.f && fmaf(dv, dv, du * du) < Z[q] * Z[q]) ? 1 : 0;
    }
  }
  // rows 4 (lane / 16) + q: sum over the 16 lanes (columns) that share them
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    int c = cnt[q];
    c += __shfl_xor(c, 1, 64);
    c += __shfl_xor(c, 2, 64);
    c += __shfl_xor(c, 4, 64);
    c += __shfl_xor(c, 8, 64);
    if (col == 0 && c) atomicAdd(&s_c[w * 16 + 4 * (lane >> 4) + q], c);
  }
  __syncthreads();
  if (tid < kMfHyps) {
    const int hh = blockIdx.y * kMfHyps + tid;
    if (hh < a.n_hyp && s_c[tid] && a.counts[hh] >= 0) atomicAdd(&a.counts[hh], s_c[tid]);
  }
}

__global__ __launch_bounds__(256) void pnp_select_kernel(PnpArgs a) {
  __shared__ int32_t s_v[256], s_i[256];
  const int tid = threadIdx.x;
  int bv = -1, bi = -1;
  for (int h = tid; h < a.n_hyp; h += 256) {
    const int c = a.counts[h];
    if (c > bv) {  // increasing h per thread: keeps the lowest index
      bv = c;
      bi = h;
    }
  }
  s_v[tid] = bv;
  s_i[tid] = bi;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (tid < st) {
      const int ov = s_v[tid + st], oi = s_i[tid + st];
      if (oi >= 0 && (s_i[tid] < 0 || ov > s_v[tid] || (ov == s_v[tid] && oi < s_i[tid]))) {
        s_v[tid] = ov;
        s_i[tid] = oi;
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    const int b = s_i[0];
    *a.best = b;
    for (int k = 0; k < 12; ++k) a.T[k] = (b >= 0 && s_v[0] >= 0) ? a.hyp[12 * b + k] : a.pose0[k];
    a.state[0] = (b >= 0 && s_v[0] >= 0) ? 1 : 0;  // refinement enabled
  }
}

// ------------------------------------------------------------ refinement
constexpr int kPnpNormal = 28;  // J^T J (21), J^T r (6), inlier count

// Sum of v over the 64 lanes of a wave, the same butterfly on every lane.
template <class F>
__device__ __forceinline__ F wave_sum64(F v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__global__ __launch_bounds__(256) void pnp_normal_kernel(PnpArgs a, int final_pass) {
  __shared__ float s_w[4][kPnpNormal];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (!final_pass && !a.state[0]) return;  // uniform: refinement stopped
  float T[12];
  for (int k = 0; k < 12; ++k) T[k] = a.T[k];
  const float tau2 = a.tau * a.tau;
  float acc[kPnpNormal] = {};  // A21 (21), b (6), count
  // chunks of 4 x 256 correspondences: the four loads are issued before the
  // first use, one memory latency per chunk
  for (int64_t base = static_cast<int64_t>(blockIdx.x) * 1024; base < a.n;
       base += static_cast<int64_t>(gridDim.x) * 1024) {
    float P[4][5];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t i = base + q * 256 + tid;
      if (i < a.n) {
        P[q][0] = a.x3d[3 * i]; P[q][1] = a.x3d[3 * i + 1]; P[q][2] = a.x3d[3 * i + 2];
        P[q][3] = a.p2d[2 * i]; P[q][4] = a.p2d[2 * i + 1];
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t i = base + q * 256 + tid;
      if (i >= a.n) continue;
      float r[2], J[2][6];
      const bool front = reproj_rows(T, a.fx, a.fy, a.cx, a.cy, P[q], P[q][3], P[q][4], r, J);
      const bool inl = front && (r[0] * r[0] + r[1] * r[1] < tau2);
      if (final_pass) {
        if (a.inliers) a.inliers[i] = inl ? 1 : 0;
        acc[27] += inl ? 1.f : 0.f;
        continue;
      }
      if (!inl) continue;
      accumulate_normal(r, J, acc, acc + 21);
      acc[27] += 1.f;
    }
  }
  // lanes, then the four waves in order: a fixed summation order
#pragma unroll
  for (int k = 0; k < kPnpNormal; ++k) {
    const float v = wave_sum64(acc[k]);
    if (lane == 0) s_w[wv][k] = v;
  }
  __syncthreads();
  if (tid < kPnpNormal)
    a.part[static_cast<int64_t>(blockIdx.x) * kPnpNormal + tid] = ((s_w[0][tid] + s_w[1][tid]) + s_w[2][tid]) + s_w[3][tid];
}

// Sum of the workgroup partials in FP64 (thread t takes blocks t, t + 256,
// ..., then lanes and waves in a fixed order), then the 6x6 solve and
// T <- Exp(delta) T, or (final pass) the inlier count and the pose.
__global__ __launch_bounds__(256) void pnp_update_kernel(PnpArgs a, int n_blocks, int final_pass) {
  __shared__ double s_w[4][kPnpNormal];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  if (!final_pass && !a.state[0]) return;  // uniform
  double acc[kPnpNormal] = {};
  for (int bk = t; bk < n_blocks; bk += 256) {
    const float* q = a.part + static_cast<int64_t>(bk) * kPnpNormal;
#pragma unroll
    for (int k = 0; k < kPnpNormal; ++k) acc[k] += static_cast<double>(q[k]);
  }
#pragma unroll
  for (int k = 0; k < kPnpNormal; ++k) {
    const double v = wave_sum64(acc[k]);
    if (lane == 0) s_w[wv][k] = v;
  }
  __syncthreads();
  if (t != 0) return;
  double S[kPnpNormal];
  for (int k = 0; k < kPnpNormal; ++k) S[k] = ((s_w[0][k] + s_w[1][k]) + s_w[2][k]) + s_w[3][k];
  if (final_pass) {
    *a.n_inliers = static_cast<int32_t>(S[27]);
    for (int k = 0; k < 12; ++k) a.pose_out[k] = a.T[k];
    return;
  }
  double nb[6], delta[6];
  for (int i = 0; i < 6; ++i) nb[i] = -S[21 + i];
  if (!chol6(S, nb, delta, 1e-12)) {
    a.state[0] = 0;  // singular: keep the pose, stop refining
    return;
  }
  double T[12];
  for (int k = 0; k < 12; ++k) T[k] = a.T[k];
  se3_exp_left(delta, T);
  for (int k = 0; k < 12; ++k) a.T[k] = static_cast<float>(T[k]);
}

// ------------------------------------------------------------ back-projection
__global__ void backproject_kernel(const float* depth, int W, int H, const float* pose, float fx, float fy, float cx,
                                   float cy, const int32_t* pix, int n, float* x3d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t q = pix[i];
  if (q < 0 || q >= W * H) {
    x3d[3 * i] = x3d[3 * i + 1] = x3d[3 * i + 2] = 0.f;
    return;
  }
  const int y = q / W, x = q - y * W;
  const float d = depth[q];
  const float xc = d * ((static_cast<float>(x) + 0.5f - cx) / fx);
  const float yc = d * ((static_cast<float>(y) + 0.5f - cy) / fy);
  const float v[3] = {xc - pose[3], yc - pose[7], d - pose[11]};
  for (int r = 0; r < 3; ++r) x3d[3 * i + r] = pose[r] * v[0] + pose[4 + r] * v[1] + pose[8 + r] * v[2];
}

// ------------------------------------------------------------ Algorithm 2
__global__ void pose_consistency_kernel(const float* poses, int n, float tau_deg, int32_t* reliable,
                                        float* max_angle) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  float worst = 0.f;
  bool ok = true;
  for (int i = 0; i + 1 < n; ++i) {
    const float* A = poses + 12 * i;
    const float* B = poses + 12 * (i + 1);
    // trace(R_A R_B^T) = sum_rc A_rc B_rc
    float tr = 0.f;
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) tr += A[4 * r + c] * B[4 * r + c];
    tr = fminf(3.f, fmaxf(tr, -1.f));
    const float ang = acosf((tr - 1.f) * 0.5f) * (180.f / 3.14159265358979f);
    worst = fmaxf(worst, ang);
    ok &= ang <= tau_deg;
  }
  *reliable = ok ? 1 : 0;
  if (max_angle) *max_angle = worst;
}

// ------------------------------------------------------------ launchers
void launch_pnp(const PnpArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(pnp_hyp_kernel, dim3((a.n_hyp + 63) / 64), dim3(64), 0, s, a);
  const int pblocks = static_cast<int>((a.n + kMfPoints - 1) / kMfPoints);
  if (pblocks > 0)
    hipLaunchKernelGGL(pnp_score_mfma_kernel, dim3(pblocks, (a.n_hyp + kMfHyps - 1) / kMfHyps), dim3(256), 0, s,
                       a);
  hipLaunchKernelGGL(pnp_select_kernel, dim3(1), dim3(256), 0, s, a);
  const int nb = pnp_normal_blocks(a.n);
  for (int it = 0; it < a.refine_iters; ++it) {
    hipLaunchKernelGGL(pnp_normal_kernel, dim3(nb), dim3(256), 0, s, a, 0);
    hipLaunchKernelGGL(pnp_update_kernel, dim3(1), dim3(256), 0, s, a, nb, 0);
  }
  hipLaunchKernelGGL(pnp_normal_kernel, dim3(nb), dim3(256), 0, s, a, 1);
  hipLaunchKernelGGL(pnp_update_kernel, dim3(1), dim3(256), 0, s, a, nb, 1);
}

int pnp_normal_blocks(int64_t n) {
  int64_t b = (n + 1023) / 1024;  // about four correspondences per thread
  if (b > 1024) b = 1024;
  return static_cast<int>(b < 1 ? 1 : b);
}

void launch_backproject(const float* depth, int W, int H, const float* pose, float fx, float fy, float cx, float cy,
                        const int32_t* pix, int n, float* x3d, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(backproject_kernel, dim3((n + 255) / 256), dim3(256), 0, s, depth, W, H, pose, fx, fy, cx, cy,
                     pix, n, x3d);
}

void launch_pose_consistency(const float* poses, int n, float tau_deg, int32_t* reliable, float* max_angle,
                             hipStream_t s) {
  hipLaunchKernelGGL(pose_consistency_kernel, dim3(1), dim3(64), 0, s, poses, n, tau_deg, reliable, max_angle);
}

}  // namespace hgsr
