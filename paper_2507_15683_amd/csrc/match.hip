// Coarse-to-fine probabilistic mutual matching of query and rendered feature
// maps (Sec. 3.4, Eq. 11).
//
// Coarse level, for N_q query and N_r rendered positions with cosine matrix
// M (never stored):
//   P_ij = softmax_j(M/tau)_ij softmax_i(M/tau)_ij = exp(2 S_ij - a_i - b_j),
//   S = M / tau, a_i = LSE_j S_ij, b_j = LSE_i S_ij,
// so row i's best j maximises 2 S_ij - b_j and column j's best i maximises
// 2 S_ij - a_i.  Two passes of the same tiled product M = Q R^T on the
// matrix cores (v_mfma_f32_32x32x8_bf16: the bf16 feature vectors enter
// exactly, products accumulate in FP32):
//   stats pass   per row and per column sum of exp(S - 1/tau) (cosines are at
//                most 1, so the shift needs no max pass; tau >= 1/40 keeps
//                every row's sum above the FP32 range's low end);
//   argmax pass  per row the best column of 2 S - b, per column the best row
//                of 2 S - a (ties: lowest index).
// A workgroup owns 128 query rows (a wave 32 of them) and sweeps every column
// tile of 32; row results stay in registers, column results are combined in
// LDS over the workgroup's waves and written as one partial per (row block,
// column), then reduced.  MNN keeps (i, j) when column j's best row is i; the
// correspondences are compacted in query order by a scan.
//
// Fine level: one workgroup of 64 threads per coarse correspondence; thread
// t owns query window position t and computes its 64 cosines against the
// render window (staged in LDS), the window's 64 x 64 matrix goes to LDS for
// the column statistics, and each thread reports its position's mutual match.
#include "hgsr_device.hpp"
#include "launch.hpp"

namespace hgsr {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef short shortx4 __attribute__((ext_vector_type(4)));

constexpr int kRowBlock = kMatchRowBlock;  // query rows per workgroup (4 waves x 32)
constexpr float kLog2e = 1.4426950408889634f;

// ------------------------------------------------------------ preparation
// Planar bf16 map (D x n positions) -> position-major vectors (n x D) and
// FP32 norms.
__global__ void match_prep_kernel(const uint16_t* map, int D, int64_t n, uint16_t* vec, float* norm) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n) return;
  float ss = 0.f;
  for (int d = 0; d < D; ++d) {
    const uint16_t b = map[static_cast<int64_t>(d) * n + p];
    vec[p * D + d] = b;
    const float f = __uint_as_float(static_cast<uint32_t>(b) << 16);
    ss = fmaf(f, f, ss);
  }
  norm[p] = sqrtf(ss);
}

// The tile product: acc[r] = Q_i . R_j for this lane's 16 rows
// i = 8 (r/4) + 4 (lane/32) + r%4 of the wave's 32 and column j = lane % 32
// of the tile.  A operands (the wave's rows) are loaded once by the caller.
template <int D>
__device__ __forceinline__ floatx16 tile_dot(const uint2 (&aop)[D / 8], const uint16_t* rvec, int col, int nr,
                                             int half) {
  floatx16 acc = {};
#pragma unroll
  for (int ks = 0; ks < D / 8; ++ks) {
    uint2 bv = make_uint2(0u, 0u);
    if (col < nr) bv = *reinterpret_cast<const uint2*>(rvec + static_cast<int64_t>(col) * D + 8 * ks + 4 * half);
    shortx4 A, B;
    __builtin_memcpy(&A, &aop[ks], 8);
    __builtin_memcpy(&B, &bv, 8);
    acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(A, B, acc, 0, 0, 0);
  }
  return acc;
}

struct MatchArgs {
  const uint16_t* qvec;
  const uint16_t* rvec;
  const float* qnorm;
  const float* rnorm;
  int32_t nq, nr;
  float inv_tau;       // 1 / tau
  float* row_sum;      // stats: sum_j exp(S_ij - 1/tau)
  float* col_part;     // stats: per (row block, column) partial sums
  const float* row_lse;  // argmax: a_i
  const float* col_lse;  // argmax: b_j
  int32_t* row_arg;    // argmax: best column per row
  float* colp_val;     // argmax: per (row block, column) best value
  int32_t* colp_idx;   //          and its row
};

template <int D, bool ARGMAX>
__global__ __launch_bounds__(256) void match_pass_kernel(MatchArgs a) {
  __shared__ float s_cv[4][32];
  __shared__ int32_t s_ci[4][32];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, half = lane >> 5, cl = lane & 31;
  const int rb = blockIdx.x;
  const int row0 = rb * kRowBlock + wave * 32;
  // A operands: row row0 + cl, channels 8 ks + 4 half .. + 3
  uint2 aop[D / 8];
#pragma unroll
  for (int ks = 0; ks < D / 8; ++ks) {
    aop[ks] = make_uint2(0u, 0u);
    if (row0 + cl < a.nq)
      aop[ks] = *reinterpret_cast<const uint2*>(a.qvec + static_cast<int64_t>(row0 + cl) * D + 8 * ks + 4 * half);
  }
  float nq[16], rs[16], ra[16];
  int32_t ri[16];
  bool rv[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int i = row0 + 8 * (r / 4) + 4 * half + (r % 4);
    rv[r] = i < a.nq;
    nq[r] = rv[r] ? a.qnorm[i] : 1.f;
    rs[r] = 0.f;
    ra[r] = ARGMAX && rv[r] ? a.row_lse[i] : 0.f;
    ri[r] = -1;
    if (ARGMAX) rs[r] = -INFINITY;  // best value of 2 S - b
  }
  const float k1 = kLog2e * a.inv_tau;
  for (int c0 = 0; c0 < a.nr; c0 += 32) {
    const int col = c0 + cl;
    const bool cv = col < a.nr;
    const floatx16 acc = tile_dot<D>(aop, a.rvec, col, a.nr, half);
    const float nr = cv ? a.rnorm[col] : 1.f;
    const float cb = ARGMAX && cv ? a.col_lse[col] : 0.f;
    float cacc = ARGMAX ? -INFINITY : 0.f;
    int32_t cidx = -1;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float m = acc[r] * __builtin_amdgcn_rcpf(fmaf(nq[r], nr, kCosEps));  // cosine
      const bool ok = rv[r] && cv;
      if constexpr (!ARGMAX) {
        // exp(S - 1/tau) = 2^((m - 1) log2(e) / tau)
        const float e = ok ? __builtin_amdgcn_exp2f(fmaf(m, k1, -k1)) : 0.f;
        rs[r] += e;
        cacc += e;
      } else {
        const float s2 = 2.f * m * a.inv_tau;
        const float vr = s2 - cb;       // row i's objective at column j
        const float vc = s2 - ra[r];    // column j's objective at row i
        if (ok && vr > rs[r]) {         // columns arrive in increasing order per lane
          rs[r] = vr;
          ri[r] = col;
        }
        const int i = row0 + 8 * (r / 4) + 4 * half + (r % 4);
        if (ok && vc > cacc) {          // rows increase with r within a lane
          cacc = vc;
          cidx = i;
        }
      }
    }
    // the column over this wave's 32 rows: combine the two lane halves
    if constexpr (!ARGMAX) {
      cacc += __shfl_xor(cacc, 32, 64);
    } else {
      const float ov = __shfl_xor(cacc, 32, 64);
      const int32_t oi = __shfl_xor(cidx, 32, 64);
      if (ov > cacc || (ov == cacc && oi >= 0 && (cidx < 0 || oi < cidx))) {
        cacc = ov;
        cidx = oi;
      }
    }
    if (half == 0) {
      s_cv[wave][cl] = cacc;
      s_ci[wave][cl] = cidx;
    }
    __syncthreads();
    if (tid < 32 && c0 + tid < a.nr) {
      const int64_t o = static_cast<int64_t>(rb) * a.nr + c0 + tid;
      if constexpr (!ARGMAX) {
        a.col_part[o] = s_cv[0][tid] + s_cv[1][tid] + s_cv[2][tid] + s_cv[3][tid];
      } else {
        float bv = -INFINITY;
        int32_t bi = -1;
#pragma unroll
        for (int w = 0; w < 4; ++w) {  // waves hold increasing rows
          if (s_ci[w][tid] >= 0 && s_cv[w][tid] > bv) {
            bv = s_cv[w][tid];
            bi = s_ci[w][tid];
          }
        }
        a.colp_val[o] = bv;
        a.colp_idx[o] = bi;
      }
    }
    __syncthreads();
  }
  // rows: combine the 32 lanes of each half (columns cl + 32 t)
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    float v = rs[r];
    int32_t idx = ri[r];
#pragma unroll
    for (int off = 16; off > 0; off >>= 1) {
      const float ov = __shfl_xor(v, off, 64);
      const int32_t oi = __shfl_xor(idx, off, 64);
      if constexpr (!ARGMAX) {
        v += ov;
      } else if (oi >= 0 && (idx < 0 || ov > v || (ov == v && oi < idx))) {
        v = ov;
        idx = oi;
      }
    }
    const int i = row0 + 8 * (r / 4) + 4 * half + (r % 4);
    if (cl == 0 && rv[r]) {
      if constexpr (!ARGMAX) a.row_sum[i] = v;
      else a.row_arg[i] = idx;
    }
  }
}

// Row and column log-sum-exps: a_i = 1/tau + log(row sum), b_j likewise from
// the partials (summed over the row blocks in order).
__global__ void match_lse_kernel(MatchArgs a, int n_rb, float* row_lse, float* col_lse) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < a.nq) row_lse[t] = a.inv_tau + __logf(a.row_sum[t]);
  if (t < a.nr) {
    float s = 0.f;
    for (int b = 0; b < n_rb; ++b) s += a.col_part[static_cast<int64_t>(b) * a.nr + t];
    col_lse[t] = a.inv_tau + __logf(s);
  }
}

// Column winners from the per-row-block partials, then the mutual flags.
__global__ void match_colarg_kernel(MatchArgs a, int n_rb, int32_t* col_arg) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= a.nr) return;
  float bv = -INFINITY;
  int32_t bi = -1;
  for (int b = 0; b < n_rb; ++b) {  // row blocks hold increasing rows
    const int64_t o = static_cast<int64_t>(b) * a.nr + j;
    const int32_t i = a.colp_idx[o];
    if (i >= 0 && a.colp_val[o] > bv) {
      bv = a.colp_val[o];
      bi = i;
    }
  }
  col_arg[j] = bi;
}

__global__ void match_flag_kernel(const int32_t* row_arg, const int32_t* col_arg, int nq, uint32_t* flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nq) return;
  const int32_t j = row_arg[i];
  flag[i] = (j >= 0 && col_arg[j] == i) ? 1u : 0u;
}

// P_ij of each correspondence (the cosine recomputed in FP32), compacted.
template <int D>
__global__ void match_emit_kernel(MatchArgs a, const uint32_t* flag, const uint32_t* offs, const float* row_lse,
                                  const float* col_lse, int32_t* out_q, int32_t* out_r, float* out_p) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.nq || !flag[i]) return;
  const int32_t j = a.row_arg[i];
  float dot = 0.f;
  for (int d = 0; d < D; ++d) {
    const float x = __uint_as_float(static_cast<uint32_t>(a.qvec[static_cast<int64_t>(i) * D + d]) << 16);
    const float y = __uint_as_float(static_cast<uint32_t>(a.rvec[static_cast<int64_t>(j) * D + d]) << 16);
    dot = fmaf(x, y, dot);
  }
  const float m = dot / fmaf(a.qnorm[i], a.rnorm[j], kCosEps);
  const uint32_t k = offs[i];
  out_q[k] = i;
  out_r[k] = j;
  out_p[k] = __expf(2.f * m * a.inv_tau - row_lse[i] - col_lse[j]);
}

// ------------------------------------------------------------ fine level
struct FineArgs {
  const uint16_t* qf;  // D x Hf x Wf planar
  const uint16_t* rf;
  int32_t Wc, Wf, Hf;
  int64_t plane;       // Hf * Wf
  float inv_tau;
  const int32_t* cq;   // coarse correspondences
  const int32_t* cr;
  const uint32_t* n_coarse;
  int32_t* fq;         // per coarse correspondence w*w slots
  int32_t* fr;
  float* fp;
};

// w = 8: 64 window positions, one thread each.
template <int D>
__global__ __launch_bounds__(64) void match_fine_kernel(FineArgs a) {
  constexpr int WW = 64, w = 8;
  __shared__ float s_r[WW][D + 1];   // render window vectors (FP32)
  __shared__ float s_m[WW][WW + 1];  // the window's cosines [query][render]
  __shared__ float s_rn[WW];
  __shared__ float s_cl[WW];         // column log-sum-exps
  __shared__ int32_t s_ca[WW];       // column winners
  const int k = blockIdx.x;
  const int t = threadIdx.x;
  if (static_cast<uint32_t>(k) >= *a.n_coarse) return;  // uniform
  const int cq = a.cq[k], cr = a.cr[k];
  const int qy0 = (cq / a.Wc) * w, qx0 = (cq % a.Wc) * w;
  const int ry0 = (cr / a.Wc) * w, rx0 = (cr % a.Wc) * w;
  const int ty = t / w, tx = t % w;
  const int64_t qpix = static_cast<int64_t>(qy0 + ty) * a.Wf + qx0 + tx;
  const int64_t rpix = static_cast<int64_t>(ry0 + ty) * a.Wf + rx0 + tx;
  float q[D];
  float qq = 0.f, rr = 0.f;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    q[d] = __uint_as_float(static_cast<uint32_t>(a.qf[d * a.plane + qpix]) << 16);
    qq = fmaf(q[d], q[d], qq);
    const float rv = __uint_as_float(static_cast<uint32_t>(a.rf[d * a.plane + rpix]) << 16);
    s_r[t][d] = rv;
    rr = fmaf(rv, rv, rr);
  }
  const float nq = sqrtf(qq);
  s_rn[t] = sqrtf(rr);
  __syncthreads();
  // row t: cosines, and the row log-sum-exp with its exact maximum
  float mx = -INFINITY;
  for (int j = 0; j < WW; ++j) {
    float dot = 0.f;
#pragma unroll
    for (int d = 0; d < D; ++d) dot = fmaf(q[d], s_r[j][d], dot);
    const float m = dot / fmaf(nq, s_rn[j], kCosEps);
    s_m[t][j] = m;
    mx = fmaxf(mx, m);
  }
  float se = 0.f;
  for (int j = 0; j < WW; ++j) se += __expf((s_m[t][j] - mx) * a.inv_tau);
  const float row_lse = mx * a.inv_tau + __logf(se);
  __syncthreads();
  // column t: log-sum-exp
  float cmx = -INFINITY;
  for (int i = 0; i < WW; ++i) cmx = fmaxf(cmx, s_m[i][t]);
  float cse = 0.f;
  for (int i = 0; i < WW; ++i) cse += __expf((s_m[i][t] - cmx) * a.inv_tau);
  s_cl[t] = cmx * a.inv_tau + __logf(cse);
  __syncthreads();
  // column t's best row of 2 S - a_i needs every row's a_i: stage them
  __shared__ float s_rl[WW];
  s_rl[t] = row_lse;
  __syncthreads();
  float bcv = -INFINITY;
  int32_t bci = 0;
  for (int i = 0; i < WW; ++i) {
    const float v = 2.f * s_m[i][t] * a.inv_tau - s_rl[i];
    if (v > bcv) {
      bcv = v;
      bci = i;
    }
  }
  s_ca[t] = bci;
  __syncthreads();
  // row t's best column of 2 S - b_j
  float brv = -INFINITY;
  int32_t brj = 0;
  for (int j = 0; j < WW; ++j) {
    const float v = 2.f * s_m[t][j] * a.inv_tau - s_cl[j];
    if (v > brv) {
      brv = v;
      brj = j;
    }
  }
  const int64_t o = static_cast<int64_t>(k) * WW + t;
  if (s_ca[brj] == t) {
    a.fq[o] = static_cast<int32_t>(qpix);
    a.fr[o] = static_cast<int32_t>(static_cast<int64_t>(ry0 + brj / w) * a.Wf + rx0 + brj % w);
    a.fp[o] = __expf(brv - row_lse);  // P = exp(2 S - b_j - a_i)
  } else {
    a.fq[o] = -1;
    a.fr[o] = -1;
    a.fp[o] = 0.f;
  }
}

// ------------------------------------------------------------ launchers
void launch_match(const MatchLaunch& L, hipStream_t s) {
  const int nq = L.nq, nr = L.nr, D = L.D;
  const int n_rb = (nq + kRowBlock - 1) / kRowBlock;
  hipLaunchKernelGGL(match_prep_kernel, dim3((nq + 255) / 256), dim3(256), 0, s, L.q_coarse, D,
                     static_cast<int64_t>(nq), L.qvec, L.qnorm);
  hipLaunchKernelGGL(match_prep_kernel, dim3((nr + 255) / 256), dim3(256), 0, s, L.r_coarse, D,
                     static_cast<int64_t>(nr), L.rvec, L.rnorm);
  MatchArgs a;
  a.qvec = L.qvec;
  a.rvec = L.rvec;
  a.qnorm = L.qnorm;
  a.rnorm = L.rnorm;
  a.nq = nq;
  a.nr = nr;
  a.inv_tau = 1.f / L.tau_coarse;
  a.row_sum = L.row_sum;
  a.col_part = L.col_part;
  a.row_lse = L.row_lse;
  a.col_lse = L.col_lse;
  a.row_arg = L.row_arg;
  a.colp_val = L.col_part;  // the stats partials are dead once reduced
  a.colp_idx = L.colp_idx;
  switch (D) {
    case 8: hipLaunchKernelGGL((match_pass_kernel<8, false>), dim3(n_rb), dim3(256), 0, s, a); break;
    case 16: hipLaunchKernelGGL((match_pass_kernel<16, false>), dim3(n_rb), dim3(256), 0, s, a); break;
    case 64: hipLaunchKernelGGL((match_pass_kernel<64, false>), dim3(n_rb), dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL((match_pass_kernel<32, false>), dim3(n_rb), dim3(256), 0, s, a); break;
  }
  const int nmax = nq > nr ? nq : nr;
  hipLaunchKernelGGL(match_lse_kernel, dim3((nmax + 255) / 256), dim3(256), 0, s, a, n_rb, L.row_lse, L.col_lse);
  switch (D) {
    case 8: hipLaunchKernelGGL((match_pass_kernel<8, true>), dim3(n_rb), dim3(256), 0, s, a); break;
    case 16: hipLaunchKernelGGL((match_pass_kernel<16, true>), dim3(n_rb), dim3(256), 0, s, a); break;
    case 64: hipLaunchKernelGGL((match_pass_kernel<64, true>), dim3(n_rb), dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL((match_pass_kernel<32, true>), dim3(n_rb), dim3(256), 0, s, a); break;
  }
  hipLaunchKernelGGL(match_colarg_kernel, dim3((nr + 255) / 256), dim3(256), 0, s, a, n_rb, L.col_arg);
  hipLaunchKernelGGL(match_flag_kernel, dim3((nq + 255) / 256), dim3(256), 0, s, L.row_arg, L.col_arg, nq, L.flag);
  launch_scan(L.flag, nq, L.offs, nullptr, L.scan_tmp, L.n_coarse, ~0ull, nullptr, 0, s);
  switch (D) {
    case 8: hipLaunchKernelGGL((match_emit_kernel<8>), dim3((nq + 255) / 256), dim3(256), 0, s, a, L.flag, L.offs,
                               L.row_lse, L.col_lse, L.out_cq, L.out_cr, L.out_cp); break;
    case 16: hipLaunchKernelGGL((match_emit_kernel<16>), dim3((nq + 255) / 256), dim3(256), 0, s, a, L.flag, L.offs,
                                L.row_lse, L.col_lse, L.out_cq, L.out_cr, L.out_cp); break;
    case 64: hipLaunchKernelGGL((match_emit_kernel<64>), dim3((nq + 255) / 256), dim3(256), 0, s, a, L.flag, L.offs,
                                L.row_lse, L.col_lse, L.out_cq, L.out_cr, L.out_cp); break;
    default: hipLaunchKernelGGL((match_emit_kernel<32>), dim3((nq + 255) / 256), dim3(256), 0, s, a, L.flag, L.offs,
                                L.row_lse, L.col_lse, L.out_cq, L.out_cr, L.out_cp); break;
  }
  if (!L.q_fine) return;
  FineArgs f;
  f.qf = L.q_fine;
  f.rf = L.r_fine;
  f.Wc = L.Wc;
  f.Wf = L.Wc * 8;
  f.Hf = L.Hc * 8;
  f.plane = static_cast<int64_t>(f.Wf) * f.Hf;
  f.inv_tau = 1.f / L.tau_fine;
  f.cq = L.out_cq;
  f.cr = L.out_cr;
  f.n_coarse = L.n_coarse;
  f.fq = L.out_fq;
  f.fr = L.out_fr;
  f.fp = L.out_fp;
  switch (D) {
    case 8: hipLaunchKernelGGL(match_fine_kernel<8>, dim3(nq), dim3(64), 0, s, f); break;
    case 16: hipLaunchKernelGGL(match_fine_kernel<16>, dim3(nq), dim3(64), 0, s, f); break;
    case 64: hipLaunchKernelGGL(match_fine_kernel<64>, dim3(nq), dim3(64), 0, s, f); break;
    default: hipLaunchKernelGGL(match_fine_kernel<32>, dim3(nq), dim3(64), 0, s, f); break;
  }
}

}  // namespace hgsr
