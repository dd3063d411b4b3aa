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
// Fine level: one workgroup of 64 threads per coarse correspondence; the
// two windows' vectors are staged in LDS, the window's 64 x 64 cosine matrix
// comes from the matrix cores and goes to LDS, thread t takes row t's and
// column t's statistics and reports query position t's mutual match.
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

struct MatchArgs {
  const uint16_t* qvec;
  const uint16_t* rvec;
  const float* qnorm;
  const float* rnorm;
  int32_t nq, nr;
  int32_t n_split;     // column ranges per row block (grid y)
  int32_t split_cols;  // columns per range (a multiple of 128)
  float inv_tau;       // 1 / tau
  float* row_part;     // stats: per (range, row) sums; argmax: per (range, row) best values
  int32_t* rowp_idx;   // argmax: per (range, row) best column
  float* col_part;     // stats: per (row block, column) sums; argmax: best values
  int32_t* colp_idx;   // argmax: per (row block, column) best row
  const float* row_lse;  // argmax: a_i
  const float* col_lse;  // argmax: b_j
};

constexpr int kTilesPerRound = 2;  // column tiles of 32 per LDS combine

// Stats (ARGMAX false) or argmax (true) over the column range
// [blockIdx.y * split_cols, + split_cols) for the workgroup's 128 rows.
template <int D, bool ARGMAX>
__global__ __launch_bounds__(256) void match_pass_kernel(MatchArgs a) {
  constexpr int RC = 32 * kTilesPerRound;  // columns per round
  __shared__ float s_cv[4][RC];
  __shared__ int32_t s_ci[4][RC];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, half = lane >> 5, cl = lane & 31;
  const int rb = blockIdx.x, sp = blockIdx.y;
  const int row0 = rb * kRowBlock + wave * 32;
  const int c_begin = sp * a.split_cols;
  const int c_end = min(a.nr, c_begin + a.split_cols);
  // A operands: row row0 + cl, channels 8 ks + 4 half .. + 3
  uint2 aop[D / 8];
#pragma unroll
  for (int ks = 0; ks < D / 8; ++ks) {
    aop[ks] = make_uint2(0u, 0u);
    if (row0 + cl < a.nq)
      aop[ks] = *reinterpret_cast<const uint2*>(a.qvec + static_cast<int64_t>(row0 + cl) * D + 8 * ks + 4 * half);
  }
  // Per row 1/|q| and a bias that removes rows past the end: stats adds
  // exp2(-inf) = 0 for them, argmax compares 2 S - inf = -inf, which never
  // wins.  With the column's scale w_j (1/|r| times 2/tau or log2(e)/tau)
  // an entry costs one product iq_i w_j instead of a reciprocal of
  // |q||r| + eps: the two differ by a relative eps / (|q||r|), and for a
  // zero vector both give a cosine of 0.
  float iq[16], rs[16], ra[16];
  int32_t ri[16];
  bool rv[16];
  const float k1 = kLog2e * a.inv_tau;
  const float two_tau = 2.f * a.inv_tau;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int i = row0 + 8 * (r / 4) + 4 * half + (r % 4);
    rv[r] = i < a.nq;
    const float n = rv[r] ? a.qnorm[i] : 0.f;
    iq[r] = n > 0.f ? 1.f / n : 0.f;
    rs[r] = ARGMAX ? -INFINITY : 0.f;  // stats: sum; argmax: best value of 2 S - b
    // stats: exponent bias -log2(e)/tau; argmax: a_i
    ra[r] = ARGMAX ? (rv[r] ? a.row_lse[i] : INFINITY) : (rv[r] ? -k1 : -INFINITY);
    ri[r] = -1;
  }
  // Stats: a round's B operands and column norms are loaded one round ahead,
  // so their latency hides behind the previous round's products.  Argmax
  // (more registers live, two waves per SIMD) loads them at the round's
  // start: ahead it was measured slower.
  constexpr bool kAhead = !ARGMAX;
  uint2 bop[kTilesPerRound][D / 8];
  float nrm[kTilesPerRound], lse[kTilesPerRound];
  auto load_round = [&](int c0, uint2 (&b)[kTilesPerRound][D / 8], float (&n)[kTilesPerRound],
                        float (&l)[kTilesPerRound]) {
#pragma unroll
    for (int t = 0; t < kTilesPerRound; ++t) {
      const int col = c0 + 32 * t + cl;
      const bool cv = col < c_end;
#pragma unroll
      for (int ks = 0; ks < D / 8; ++ks) {
        b[t][ks] = make_uint2(0u, 0u);
        if (cv) b[t][ks] = *reinterpret_cast<const uint2*>(a.rvec + static_cast<int64_t>(col) * D + 8 * ks + 4 * half);
      }
      n[t] = cv ? a.rnorm[col] : 0.f;
      // argmax: b_j, +inf past the end (row objectives -inf there)
      l[t] = ARGMAX ? (cv ? a.col_lse[col] : INFINITY) : 0.f;
    }
  };
  if constexpr (kAhead) load_round(c_begin, bop, nrm, lse);
  for (int c0 = c_begin; c0 < c_end; c0 += RC) {
    uint2 bnext[kTilesPerRound][D / 8];
    float nnext[kTilesPerRound], lnext[kTilesPerRound];
    if constexpr (kAhead) load_round(c0 + RC, bnext, nnext, lnext);  // all zero past c_end
    else load_round(c0, bop, nrm, lse);
#pragma unroll
    for (int t = 0; t < kTilesPerRound; ++t) {
      const int col = c0 + 32 * t + cl;
      const bool cv = col < c_end;
      floatx16 acc = {};
#pragma unroll
      for (int ks = 0; ks < D / 8; ++ks) {
        shortx4 A, B;
        __builtin_memcpy(&A, &aop[ks], 8);
        __builtin_memcpy(&B, &bop[t][ks], 8);
        acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(A, B, acc, 0, 0, 0);
      }
      const float nr = nrm[t];
      const float wc = (nr > 0.f ? __builtin_amdgcn_rcpf(nr) : 0.f) * (ARGMAX ? two_tau : k1);
      const float cb = lse[t];
      float cacc = ARGMAX ? -INFINITY : 0.f;
      int32_t cidx = -1;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float sc = iq[r] * wc;  // the cosine is acc / (|q||r|); times 2/tau or log2(e)/tau
        if constexpr (!ARGMAX) {
          // exp(S - 1/tau) = 2^((m - 1) log2(e) / tau)
          const float e = cv ? __builtin_amdgcn_exp2f(fmaf(acc[r], sc, ra[r])) : 0.f;
          rs[r] += e;
          cacc += e;
        } else {
          // a product and two differences: the same with two fused multiply-adds
          // measured slower
          const float x = acc[r] * sc;
          const float vr = x - cb;     // row i's objective 2 S - b at column j
          const float vc = x - ra[r];  // column j's objective 2 S - a at row i
          if (vr > rs[r]) {            // a lane's columns arrive in increasing order
            rs[r] = vr;
            ri[r] = col;
          }
          if (vc > cacc) {             // a lane's rows increase with r
            cacc = vc;
            cidx = row0 + 8 * (r / 4) + 4 * half + (r % 4);
          }
        }
      }
      // the column over this wave's 32 rows: combine the two lane halves
      if constexpr (!ARGMAX) {
        cacc += __shfl_xor(cacc, 32, 64);
      } else {
        const float ov = __shfl_xor(cacc, 32, 64);
        const int32_t oi = __shfl_xor(cidx, 32, 64);
        if (oi >= 0 && (cidx < 0 || ov > cacc || (ov == cacc && oi < cidx))) {
          cacc = ov;
          cidx = oi;
        }
      }
      if (half == 0) {
        s_cv[wave][32 * t + cl] = cacc;
        s_ci[wave][32 * t + cl] = cidx;
      }
    }
    __syncthreads();
    if (tid < RC && c0 + tid < c_end) {
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
        a.col_part[o] = bv;
        a.colp_idx[o] = bi;
      }
    }
    __syncthreads();
    if constexpr (kAhead) {
#pragma unroll
      for (int t = 0; t < kTilesPerRound; ++t) {
#pragma unroll
        for (int ks = 0; ks < D / 8; ++ks) bop[t][ks] = bnext[t][ks];
        nrm[t] = nnext[t];
        lse[t] = lnext[t];
      }
    }
  }
  // rows: combine the 32 lanes of each half (the lanes hold different columns)
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
      a.row_part[static_cast<int64_t>(sp) * a.nq + i] = v;
      if constexpr (ARGMAX) a.rowp_idx[static_cast<int64_t>(sp) * a.nq + i] = idx;
    }
  }
}

// Reductions of the partials, 8 threads per row or column (partials k, k+8,
// ...; then combined in a fixed order): the log-sum-exps
// a_i = 1/tau + log(sum), b_j likewise (STATS), or the best column per row
// and best row per column (ties: lowest index).
template <bool STATS>
__global__ __launch_bounds__(256) void match_reduce_kernel(MatchArgs a, int n_rb, float* row_lse, float* col_lse,
                                                           int32_t* row_arg, int32_t* col_arg) {
  __shared__ float s_v[32][8];
  __shared__ int32_t s_i[32][8];
  const int part = threadIdx.x & 7, slot = threadIdx.x >> 3;
  const int64_t u = static_cast<int64_t>(blockIdx.x) * 32 + slot;  // rows first, then columns
  const bool is_row = u < a.nq;
  const int64_t x = is_row ? u : u - a.nq;
  const bool live = is_row || x < a.nr;
  const int n = is_row ? a.n_split : n_rb;
  const int64_t stride = is_row ? a.nq : a.nr;
  const float* vals = is_row ? a.row_part : a.col_part;
  const int32_t* idxs = is_row ? a.rowp_idx : a.colp_idx;
  float v = STATS ? 0.f : -INFINITY;
  int32_t bi = -1;
  if (live) {
    for (int k = part; k < n; k += 8) {
      const float w = vals[k * stride + x];
      if constexpr (STATS) {
        v += w;
      } else {
        const int32_t wi = idxs[k * stride + x];  // partials in increasing index order
        if (wi >= 0 && (bi < 0 || w > v)) {
          v = w;
          bi = wi;
        }
      }
    }
  }
  s_v[slot][part] = v;
  s_i[slot][part] = bi;
  __syncthreads();
  if (part == 0 && live) {
    float t = STATS ? 0.f : -INFINITY;
    int32_t ti = -1;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if constexpr (STATS) {
        t += s_v[slot][q];
      } else {
        const int32_t qi = s_i[slot][q];
        if (qi >= 0 && (ti < 0 || s_v[slot][q] > t || (s_v[slot][q] == t && qi < ti))) {
          t = s_v[slot][q];
          ti = qi;
        }
      }
    }
    if constexpr (STATS) {
      (is_row ? row_lse : col_lse)[x] = a.inv_tau + __logf(t);
    } else {
      (is_row ? row_arg : col_arg)[x] = ti;
    }
  }
}

__global__ void match_flag_kernel(const int32_t* row_arg, const int32_t* col_arg, int nq, uint32_t* flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nq) return;
  const int32_t j = row_arg[i];
  flag[i] = (j >= 0 && col_arg[j] == i) ? 1u : 0u;
}

// P_ij of each correspondence (the cosine recomputed in FP32), compacted.
template <int D>
__global__ void match_emit_kernel(MatchArgs a, const int32_t* row_arg, const uint32_t* flag, const uint32_t* offs,
                                  const float* row_lse, const float* col_lse, int32_t* out_q, int32_t* out_r,
                                  float* out_p) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.nq || !flag[i]) return;
  const int32_t j = row_arg[i];
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

// w = 8: 64 window positions, one thread each.  The window's 64 x 64
// products run on the matrix cores (v_mfma_f32_32x32x8_bf16: four 32 x 32
// tiles, K = D in steps of 8; the bf16 vectors enter exactly, the sums are
// FP32), staged through LDS as position-major bf16 vectors.
template <int D>
__global__ __launch_bounds__(64) void match_fine_kernel(FineArgs a) {
  constexpr int WW = 64, w = 8;
  constexpr int VS = D + 4;            // bf16 vector stride: rows 8-byte aligned, banks spread
  __shared__ __align__(16) uint16_t s_qv[WW * VS];  // query window vectors
  __shared__ __align__(16) uint16_t s_rv[WW * VS];  // render window vectors
  __shared__ float s_m[WW][WW + 1];  // the window's cosines [query][render]
  __shared__ float s_qn[WW];
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
  float qq = 0.f, rr = 0.f;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const uint16_t qb = a.qf[d * a.plane + qpix];
    const uint16_t rb = a.rf[d * a.plane + rpix];
    s_qv[t * VS + d] = qb;
    s_rv[t * VS + d] = rb;
    const float qv = __uint_as_float(static_cast<uint32_t>(qb) << 16);
    const float rv = __uint_as_float(static_cast<uint32_t>(rb) << 16);
    qq = fmaf(qv, qv, qq);
    rr = fmaf(rv, rv, rr);
  }
  s_qn[t] = sqrtf(qq);
  s_rn[t] = sqrtf(rr);
  __syncthreads();
  {
    // lane l: operand row / column l % 32 of its tile, channels 8 ks + 4 (l / 32) .. + 3
    const int cl = t & 31, half = t >> 5;
    floatx16 acc[2][2];
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj) acc[ti][tj] = floatx16{};
#pragma unroll
    for (int ks = 0; ks < D / 8; ++ks) {
      shortx4 A[2], B[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        __builtin_memcpy(&A[u], &s_qv[(32 * u + cl) * VS + 8 * ks + 4 * half], 8);
        __builtin_memcpy(&B[u], &s_rv[(32 * u + cl) * VS + 8 * ks + 4 * half], 8);
      }
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj)
          acc[ti][tj] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(A[ti], B[tj], acc[ti][tj], 0, 0, 0);
    }
    // result r of a tile: row 8 (r / 4) + 4 half + r % 4, column cl
#pragma unroll
    for (int tj = 0; tj < 2; ++tj) {
      const int j = 32 * tj + cl;
      const float nr = s_rn[j];
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int i = 32 * ti + 8 * (r / 4) + 4 * half + (r % 4);
          s_m[i][j] = acc[ti][tj][r] * __builtin_amdgcn_rcpf(fmaf(s_qn[i], nr, kCosEps));
        }
    }
  }
  __syncthreads();
  // row t: the row log-sum-exp with its exact maximum
  float mx = -INFINITY;
  for (int j = 0; j < WW; ++j) mx = fmaxf(mx, s_m[t][j]);
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
int match_splits(int nq) {
  // enough workgroups to fill the chip: about 2048 (row block, column range)
  const int n_rb = (nq + kRowBlock - 1) / kRowBlock;
  int sp = (2048 + n_rb - 1) / n_rb;
  return sp < 1 ? 1 : (sp > 32 ? 32 : sp);
}

template <int D>
static void launch_passes(MatchArgs a, const MatchLaunch& L, int n_rb, hipStream_t s) {
  const dim3 grid(n_rb, a.n_split);
  const int nred = (a.nq + a.nr + 31) / 32;
  hipLaunchKernelGGL((match_pass_kernel<D, false>), grid, dim3(256), 0, s, a);
  hipLaunchKernelGGL(match_reduce_kernel<true>, dim3(nred), dim3(256), 0, s, a, n_rb, L.row_lse, L.col_lse,
                     L.row_arg, L.col_arg);
  hipLaunchKernelGGL((match_pass_kernel<D, true>), grid, dim3(256), 0, s, a);
  hipLaunchKernelGGL(match_reduce_kernel<false>, dim3(nred), dim3(256), 0, s, a, n_rb, L.row_lse, L.col_lse,
                     L.row_arg, L.col_arg);
  hipLaunchKernelGGL(match_flag_kernel, dim3((a.nq + 255) / 256), dim3(256), 0, s, L.row_arg, L.col_arg, a.nq,
                     L.flag);
  launch_scan(L.flag, a.nq, L.offs, nullptr, L.scan_tmp, L.n_coarse, ~0ull, nullptr, 0, s);
  hipLaunchKernelGGL((match_emit_kernel<D>), dim3((a.nq + 255) / 256), dim3(256), 0, s, a, L.row_arg, L.flag,
                     L.offs, L.row_lse, L.col_lse, L.out_cq, L.out_cr, L.out_cp);
}

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
  a.n_split = L.n_split;
  const int tiles = (nr + 31) / 32;
  const int per = (tiles + a.n_split - 1) / a.n_split;
  a.split_cols = (per + kTilesPerRound - 1) / kTilesPerRound * kTilesPerRound * 32;
  a.inv_tau = 1.f / L.tau_coarse;
  a.row_part = L.row_part;
  a.rowp_idx = L.rowp_idx;
  a.col_part = L.col_part;
  a.colp_idx = L.colp_idx;
  a.row_lse = L.row_lse;
  a.col_lse = L.col_lse;
  switch (D) {
    case 8: launch_passes<8>(a, L, n_rb, s); break;
    case 16: launch_passes<16>(a, L, n_rb, s); break;
    case 64: launch_passes<64>(a, L, n_rb, s); break;
    default: launch_passes<32>(a, L, n_rb, s); break;
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
