// Pose-refinement kernels around the renderer: the per-pose residual with
// its output gradients, an Adam step on the left-perturbation tangent
// followed by the update T <- Exp(-step) T, and the retraction T <- Exp(xi) T
// with the chain rule of its tangent (the left Jacobian of SE(3)).
#include "hgsr_device.hpp"
#include "launch.hpp"

namespace hgsr {

template <int D, bool BF16>
__global__ __launch_bounds__(256) void residual_kernel(const float* rgb, const void* feat, const float* rgb_t,
                                                       const float* feat_t, int P, int64_t HW, float lam_f,
                                                       float* loss, float* g_rgb, float* g_feat) {
  __shared__ float s_red[256];
  const int pose = blockIdx.y;
  const int64_t pix = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  float l = 0.f;
  if (pix < HW) {
    const float inv = 1.f / static_cast<float>(HW);
    const int64_t o3 = static_cast<int64_t>(pose) * 3 * HW + pix;
    for (int c = 0; c < 3; ++c) {
      const float d = rgb[o3 + c * HW] - rgb_t[o3 + c * HW];
      l += fabsf(d);
      g_rgb[o3 + c * HW] = d > 0.f ? inv : (d < 0.f ? -inv : 0.f);
    }
    if constexpr (D > 0) {
      const int64_t of = static_cast<int64_t>(pose) * D * HW + pix;
      float f[D];
      float dot = 0.f, na = 0.f, nb = 0.f;
#pragma unroll
      for (int k = 0; k < D; ++k) {
        if constexpr (BF16) f[k] = __uint_as_float(static_cast<uint32_t>(static_cast<const uint16_t*>(feat)[of + k * HW]) << 16);
        else f[k] = static_cast<const float*>(feat)[of + k * HW];
        const float t = feat_t[of + k * HW];
        dot = fmaf(f[k], t, dot);
        na = fmaf(f[k], f[k], na);
        nb = fmaf(t, t, nb);
      }
      na = sqrtf(na);
      nb = sqrtf(nb);
      const float n = na * nb + kCosEps;
      const float cosv = dot / n;
      l += lam_f * (1.f - cosv);
      const float s1 = -lam_f * inv / n;
      const float s2 = na > 0.f ? lam_f * inv * dot * nb / (n * n * na) : 0.f;
#pragma unroll
      for (int k = 0; k < D; ++k) g_feat[of + k * HW] = s1 * feat_t[of + k * HW] + s2 * f[k];
    }
    l *= inv;
  }
  s_red[threadIdx.x] = l;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) s_red[threadIdx.x] += s_red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(loss + pose, s_red[0]);
}

template <int D>
static void launch_res_d(const float* rgb, const void* feat, int bf16, const float* rgb_t, const float* feat_t, int P,
                         int64_t HW, float lam_f, float* loss, float* g_rgb, float* g_feat, hipStream_t s) {
  const dim3 grid(static_cast<unsigned>((HW + 255) / 256), P);
  if (bf16)
    hipLaunchKernelGGL((residual_kernel<D, true>), grid, dim3(256), 0, s, rgb, feat, rgb_t, feat_t, P, HW, lam_f,
                       loss, g_rgb, g_feat);
  else
    hipLaunchKernelGGL((residual_kernel<D, false>), grid, dim3(256), 0, s, rgb, feat, rgb_t, feat_t, P, HW, lam_f,
                       loss, g_rgb, g_feat);
}

void launch_residual(const float* rgb, const void* feat, int feat_bf16, const float* rgb_t, const float* feat_t,
                     int P, int H, int W, int D, float lam_f, float* loss, float* g_rgb, float* g_feat,
                     hipStream_t s) {
  const int64_t HW = static_cast<int64_t>(H) * W;
  launch_fill_f32(loss, 0.f, P, s);
  switch (D) {
    case 0: launch_res_d<0>(rgb, feat, 0, rgb_t, feat_t, P, HW, lam_f, loss, g_rgb, g_feat, s); break;
    case 8: launch_res_d<8>(rgb, feat, feat_bf16, rgb_t, feat_t, P, HW, lam_f, loss, g_rgb, g_feat, s); break;
    case 16: launch_res_d<16>(rgb, feat, feat_bf16, rgb_t, feat_t, P, HW, lam_f, loss, g_rgb, g_feat, s); break;
    case 32: launch_res_d<32>(rgb, feat, feat_bf16, rgb_t, feat_t, P, HW, lam_f, loss, g_rgb, g_feat, s); break;
    default: launch_res_d<64>(rgb, feat, feat_bf16, rgb_t, feat_t, P, HW, lam_f, loss, g_rgb, g_feat, s); break;
  }
}

// One block; thread p updates pose p (looping for P > 256).
__global__ __launch_bounds__(256) void pose_adam_kernel(float* poses, const float* grad, float* m, float* v,
                                                        int32_t* step, int P, float lr_rho, float lr_phi, float b1,
                                                        float b2, float eps) {
  const int t = *step + 1;
  __syncthreads();
  if (threadIdx.x == 0) *step = t;
  const float c1 = 1.f - powf(b1, static_cast<float>(t));
  const float c2 = 1.f - powf(b2, static_cast<float>(t));
  for (int p = threadIdx.x; p < P; p += blockDim.x) {
    float d[6];
    for (int k = 0; k < 6; ++k) {
      const float g = grad[6 * p + k];
      const float mk = b1 * m[6 * p + k] + (1.f - b1) * g;
      const float vk = b2 * v[6 * p + k] + (1.f - b2) * g * g;
      m[6 * p + k] = mk;
      v[6 * p + k] = vk;
      const float lr = k < 3 ? lr_rho : lr_phi;
      d[k] = -lr * (mk / c1) / (sqrtf(vk / c2) + eps);
    }
    // Exp(d): Rodrigues rotation and V rho
    const float wx = d[3], wy = d[4], wz = d[5];
    const float th2 = wx * wx + wy * wy + wz * wz;
    const float th = sqrtf(th2);
    float A, B, Cq;
    if (th < 1e-4f) {
      A = 1.f - th2 / 6.f;
      B = 0.5f - th2 / 24.f;
      Cq = 1.f / 6.f - th2 / 120.f;
    } else {
      A = sinf(th) / th;
      B = (1.f - cosf(th)) / th2;
      Cq = (th - sinf(th)) / (th2 * th);
    }
    const float K[3][3] = {{0.f, -wz, wy}, {wz, 0.f, -wx}, {-wy, wx, 0.f}};
    float K2[3][3];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) K2[r][c] = K[r][0] * K[0][c] + K[r][1] * K[1][c] + K[r][2] * K[2][c];
    float Rd[3][3], V[3][3];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        const float I = r == c ? 1.f : 0.f;
        Rd[r][c] = I + A * K[r][c] + B * K2[r][c];
        V[r][c] = I + B * K[r][c] + Cq * K2[r][c];
      }
    float* T = poses + 12 * p;
    float R[3][3], tt[3];
    for (int r = 0; r < 3; ++r) {
      for (int c = 0; c < 3; ++c) R[r][c] = T[4 * r + c];
      tt[r] = T[4 * r + 3];
    }
    for (int r = 0; r < 3; ++r) {
      for (int c = 0; c < 3; ++c) T[4 * r + c] = Rd[r][0] * R[0][c] + Rd[r][1] * R[1][c] + Rd[r][2] * R[2][c];
      T[4 * r + 3] = Rd[r][0] * tt[0] + Rd[r][1] * tt[1] + Rd[r][2] * tt[2] + V[r][0] * d[0] + V[r][1] * d[1] +
                     V[r][2] * d[2];
    }
  }
}

// FP64 Exp of the twist (rho, phi): Rodrigues rotation and V rho.
__device__ void exp_se3_f64(const double* xi, double Rd[3][3], double td[3]) {
  const double wx = xi[3], wy = xi[4], wz = xi[5];
  const double th2 = wx * wx + wy * wy + wz * wz;
  const double th = sqrt(th2);
  double A, B, C;
  if (th < 1e-4) {  // series, truncation below double rounding
    A = 1.0 - th2 / 6.0;
    B = 0.5 - th2 / 24.0;
    C = 1.0 / 6.0 - th2 / 120.0;
  } else {
    A = sin(th) / th;
    B = (1.0 - cos(th)) / th2;
    C = (th - sin(th)) / (th2 * th);
  }
  const double K[3][3] = {{0.0, -wz, wy}, {wz, 0.0, -wx}, {-wy, wx, 0.0}};
  for (int r = 0; r < 3; ++r) {
    double v[3];
    for (int c = 0; c < 3; ++c) {
      const double k2 = K[r][0] * K[0][c] + K[r][1] * K[1][c] + K[r][2] * K[2][c];
      const double I = r == c ? 1.0 : 0.0;
      Rd[r][c] = I + A * K[r][c] + B * k2;
      v[c] = I + B * K[r][c] + C * k2;
    }
    td[r] = v[0] * xi[0] + v[1] * xi[1] + v[2] * xi[2];
  }
}

// out = Exp(xi) T per pose, one thread per pose.
__global__ __launch_bounds__(64) void pose_retract_kernel(const float* poses, const float* xi, int P, float* out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  double x[6], Rd[3][3], td[3], T[12];
  for (int k = 0; k < 6; ++k) x[k] = xi[6 * p + k];
  for (int k = 0; k < 12; ++k) T[k] = poses[12 * p + k];
  exp_se3_f64(x, Rd, td);
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c)
      out[12 * p + 4 * r + c] = static_cast<float>(Rd[r][0] * T[c] + Rd[r][1] * T[4 + c] + Rd[r][2] * T[8 + c]);
    out[12 * p + 4 * r + 3] =
        static_cast<float>(Rd[r][0] * T[3] + Rd[r][1] * T[7] + Rd[r][2] * T[11] + td[r]);
  }
}

// g_xi = J_l(xi)^T g with J_l = sum_n ad(xi)^n / (n + 1)!, ad(rho, phi) =
// [[phi^, rho^], [0, phi^]]; one thread per pose, FP64.
__global__ __launch_bounds__(64) void pose_tangent_grad_kernel(const float* xi, const float* g, int P, float* g_xi) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const double r0 = xi[6 * p], r1 = xi[6 * p + 1], r2 = xi[6 * p + 2];
  const double w0 = xi[6 * p + 3], w1 = xi[6 * p + 4], w2 = xi[6 * p + 5];
  double ad[6][6] = {};
  const double W[3][3] = {{0.0, -w2, w1}, {w2, 0.0, -w0}, {-w1, w0, 0.0}};
  const double Rh[3][3] = {{0.0, -r2, r1}, {r2, 0.0, -r0}, {-r1, r0, 0.0}};
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      ad[r][c] = W[r][c];
      ad[r][3 + c] = Rh[r][c];
      ad[3 + r][3 + c] = W[r][c];
    }
  double M[6][6], J[6][6];
  for (int r = 0; r < 6; ++r)
    for (int c = 0; c < 6; ++c) M[r][c] = J[r][c] = r == c ? 1.0 : 0.0;
  for (int n = 1; n <= 40; ++n) {
    double Mn[6][6];
    const double inv = 1.0 / static_cast<double>(n + 1);
    for (int r = 0; r < 6; ++r)
      for (int c = 0; c < 6; ++c) {
        double acc = 0.0;
        for (int k = 0; k < 6; ++k) acc += M[r][k] * ad[k][c];
        Mn[r][c] = acc * inv;
      }
    for (int r = 0; r < 6; ++r)
      for (int c = 0; c < 6; ++c) {
        M[r][c] = Mn[r][c];
        J[r][c] += Mn[r][c];
      }
  }
  double gi[6];
  for (int k = 0; k < 6; ++k) gi[k] = g[6 * p + k];
  for (int c = 0; c < 6; ++c) {
    double acc = 0.0;
    for (int r = 0; r < 6; ++r) acc += J[r][c] * gi[r];
    g_xi[6 * p + c] = static_cast<float>(acc);
  }
}

void launch_pose_retract(const float* poses, const float* xi, int P, float* out, hipStream_t s) {
  hipLaunchKernelGGL(pose_retract_kernel, dim3((P + 63) / 64), dim3(64), 0, s, poses, xi, P, out);
}

void launch_pose_tangent_grad(const float* xi, const float* g, int P, float* g_xi, hipStream_t s) {
  hipLaunchKernelGGL(pose_tangent_grad_kernel, dim3((P + 63) / 64), dim3(64), 0, s, xi, g, P, g_xi);
}

void launch_pose_adam(float* poses, const float* grad, float* m, float* v, int32_t* step, int P, float lr_rho,
                      float lr_phi, float b1, float b2, float eps, hipStream_t s) {
  hipLaunchKernelGGL(pose_adam_kernel, dim3(1), dim3(256), 0, s, poses, grad, m, v, step, P, lr_rho, lr_phi, b1, b2,
                     eps);
}

}  // namespace hgsr
