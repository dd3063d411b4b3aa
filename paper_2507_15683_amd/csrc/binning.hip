// Tile binning: exclusive scans, tile-entry emission, and the two sorts that
// put every tile's entries in (camera depth, Gaussian index) order:
//   bucket: the tile id is one radix digit resolved by a counting pass
//           (per-tile counts -> scan -> atomic slots), then each tile's
//           (depth bits << 32 | index) keys are sorted in LDS;
//   lsd:    a device least-significant-digit radix sort of
//           (tile, depth, index) keys, 8-bit digits, stable passes.
#include <algorithm>

#include "hgsr_device.hpp"
#include "launch.hpp"

namespace hgsr {

// ------------------------------------------------------------ fills
__global__ void fill_u32_kernel(uint32_t* p, uint32_t v, int64_t n) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[i] = v;
}
__global__ void fill_f32_kernel(float* p, float v, int64_t n) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[i] = v;
}

__global__ void copy_u32_kernel(uint32_t* dst, const uint32_t* src, int64_t n) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    dst[i] = src[i];
}

// Zero up to four u32 ranges in one launch.
__global__ void clear4_kernel(uint32_t* p0, int64_t n0, uint32_t* p1, int64_t n1, uint32_t* p2, int64_t n2,
                              uint32_t* p3, int64_t n3) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  for (int64_t i = t; i < n0; i += stride) p0[i] = 0u;
  for (int64_t i = t; i < n1; i += stride) p1[i] = 0u;
  for (int64_t i = t; i < n2; i += stride) p2[i] = 0u;
  for (int64_t i = t; i < n3; i += stride) p3[i] = 0u;
}

static unsigned fill_grid(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 8192) b = 8192;
  return static_cast<unsigned>(b < 1 ? 1 : b);
}

void launch_fill_u32(uint32_t* p, uint32_t value, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(fill_u32_kernel, dim3(fill_grid(n)), dim3(256), 0, s, p, value, n);
}
void launch_clear4(uint32_t* p0, int64_t n0, uint32_t* p1, int64_t n1, uint32_t* p2, int64_t n2, uint32_t* p3,
                   int64_t n3, hipStream_t s) {
  const int64_t mx = std::max(std::max(n0, n1), std::max(n2, n3));
  hipLaunchKernelGGL(clear4_kernel, dim3(fill_grid(mx)), dim3(256), 0, s, p0, n0, p1, n1, p2, n2, p3, n3);
}

void launch_copy_u32(uint32_t* dst, const uint32_t* src, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(copy_u32_kernel, dim3(fill_grid(n)), dim3(256), 0, s, dst, src, n);
}

void launch_fill_f32(float* p, float value, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(fill_f32_kernel, dim3(fill_grid(n)), dim3(256), 0, s, p, value, n);
}

// ------------------------------------------------------------ block scan
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const uint32_t o = __shfl_up(v, off, kWave);
    if (lane >= off) v += o;
  }
  return v;
}

// Exclusive scan of one value per thread over a 256-thread block; returns the
// exclusive prefix and writes the block total to *total_out (all threads).
__device__ __forceinline__ uint32_t block_excl_scan256(uint32_t v, uint32_t* s_w, uint32_t* total_out) {
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x >> 6;
  const uint32_t inc = wave_incl_scan(v);
  if (lane == kWave - 1) s_w[w] = inc;
  __syncthreads();
  uint32_t before = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint32_t x = s_w[k];
    before += (k < w) ? x : 0u;
    tot += x;
  }
  __syncthreads();
  *total_out = tot;
  return before + inc - v;
}

constexpr int kScanItems = 16;
constexpr int kScanChunk = 256 * kScanItems;

__global__ __launch_bounds__(256) void scan_reduce_kernel(const uint32_t* in, int64_t n, uint32_t* block_sums) {
  __shared__ uint32_t s_w[4];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanChunk;
  uint32_t sum = 0;
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + static_cast<int64_t>(k) * 256 + threadIdx.x;
    if (i < n) sum += in[i];
  }
  uint32_t tot;
  block_excl_scan256(sum, s_w, &tot);
  if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
}

// Single block: exclusive scan of the block sums in place; total and capacity
// check.
__global__ __launch_bounds__(256) void scan_top_kernel(uint32_t* sums, int64_t nb, uint32_t* total, uint64_t cap,
                                                       int32_t* flags, int32_t flag_bit) {
  __shared__ uint32_t s_w[4];
  const int64_t per = (nb + 255) / 256;
  const int64_t b0 = threadIdx.x * per;
  uint32_t local = 0;
  for (int64_t k = 0; k < per; ++k)
    if (b0 + k < nb) local += sums[b0 + k];
  uint32_t tot;
  uint32_t run = block_excl_scan256(local, s_w, &tot);
  for (int64_t k = 0; k < per; ++k)
    if (b0 + k < nb) {
      const uint32_t x = sums[b0 + k];
      sums[b0 + k] = run;
      run += x;
    }
  if (threadIdx.x == 0) {
    if (total) *total = tot;
    if (flags && static_cast<uint64_t>(tot) > cap) atomicOr(flags, flag_bit);
  }
}

__global__ __launch_bounds__(256) void scan_down_kernel(const uint32_t* in, int64_t n, const uint32_t* offsets,
                                                        uint32_t* out, uint2* ranges) {
  __shared__ uint32_t s_w[4];
  __shared__ uint32_t s_v[kScanChunk];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanChunk;
  // coalesced load into LDS, then each thread scans 16 consecutive values
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + static_cast<int64_t>(k) * 256 + threadIdx.x;
    s_v[k * 256 + threadIdx.x] = i < n ? in[i] : 0u;
  }
  __syncthreads();
  uint32_t vals[kScanItems];
  uint32_t sum = 0;
  for (int k = 0; k < kScanItems; ++k) {
    vals[k] = s_v[threadIdx.x * kScanItems + k];
    sum += vals[k];
  }
  uint32_t tot;
  uint32_t run = block_excl_scan256(sum, s_w, &tot) + offsets[blockIdx.x];
  for (int k = 0; k < kScanItems; ++k) {
    s_v[threadIdx.x * kScanItems + k] = run;
    run += vals[k];
  }
  __syncthreads();
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + static_cast<int64_t>(k) * 256 + threadIdx.x;
    if (i < n) {
      const uint32_t st = s_v[k * 256 + threadIdx.x];
      if (ranges) ranges[i] = make_uint2(st, st + in[i]);
      else out[i] = st;
    }
  }
}

// One 1024-thread block scans up to kWideChunk values in a single pass: each
// thread loads 16 consecutive values (four 16-byte loads, all in flight at
// once), the block scans the per-thread sums, and each thread writes its 16
// results (eight 16-byte stores for ranges).  One global round trip instead
// of one per chunk.
constexpr int kWideThreads = 1024;
constexpr int kWideItems = 16;
constexpr int64_t kWideChunk = static_cast<int64_t>(kWideThreads) * kWideItems;

__global__ __launch_bounds__(1024) void scan_wide_kernel(const uint32_t* in, int64_t n, uint32_t* out, uint2* ranges,
                                                        uint32_t* total, uint64_t cap, int32_t* flags,
                                                        int32_t flag_bit) {
  __shared__ uint32_t s_w[kWideThreads / kWave];
  const int t = threadIdx.x, lane = t & (kWave - 1), w = t >> 6;
  const int64_t b = static_cast<int64_t>(t) * kWideItems;
  const bool full = b + kWideItems <= n;
  uint32_t v[kWideItems];
  if (full && (reinterpret_cast<uintptr_t>(in) & 15) == 0) {
    const uint4* p = reinterpret_cast<const uint4*>(in + b);
#pragma unroll
    for (int k = 0; k < kWideItems / 4; ++k) {
      const uint4 q = p[k];
      v[4 * k] = q.x;
      v[4 * k + 1] = q.y;
      v[4 * k + 2] = q.z;
      v[4 * k + 3] = q.w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < kWideItems; ++k) v[k] = b + k < n ? in[b + k] : 0u;
  }
  uint32_t sum = 0;
#pragma unroll
  for (int k = 0; k < kWideItems; ++k) sum += v[k];
  const uint32_t inc = wave_incl_scan(sum);
  if (lane == kWave - 1) s_w[w] = inc;
  __syncthreads();
  uint32_t before = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < kWideThreads / kWave; ++k) {
    const uint32_t x = s_w[k];
    before += k < w ? x : 0u;
    tot += x;
  }
  uint32_t run = before + inc - sum;
  if (ranges) {
    if (full && (reinterpret_cast<uintptr_t>(ranges) & 15) == 0) {
      uint4* q = reinterpret_cast<uint4*>(ranges + b);
#pragma unroll
      for (int k = 0; k < kWideItems / 2; ++k) {
        const uint32_t s0 = run, e0 = s0 + v[2 * k], e1 = e0 + v[2 * k + 1];
        q[k] = make_uint4(s0, e0, e0, e1);
        run = e1;
      }
    } else {
#pragma unroll
      for (int k = 0; k < kWideItems; ++k) {
        if (b + k < n) ranges[b + k] = make_uint2(run, run + v[k]);
        run += v[k];
      }
    }
  } else {
    if (full && (reinterpret_cast<uintptr_t>(out) & 15) == 0) {
      uint4* q = reinterpret_cast<uint4*>(out + b);
#pragma unroll
      for (int k = 0; k < kWideItems / 4; ++k) {
        uint4 o;
        o.x = run; run += v[4 * k];
        o.y = run; run += v[4 * k + 1];
        o.z = run; run += v[4 * k + 2];
        o.w = run; run += v[4 * k + 3];
        q[k] = o;
      }
    } else {
#pragma unroll
      for (int k = 0; k < kWideItems; ++k) {
        if (b + k < n) out[b + k] = run;
        run += v[k];
      }
    }
  }
  if (t == 0) {
    if (total) *total = tot;
    if (flags && static_cast<uint64_t>(tot) > cap) atomicOr(flags, flag_bit);
  }
}

int64_t scan_block_count(int64_t n) { return (n + kScanChunk - 1) / kScanChunk; }

void launch_scan(const uint32_t* in, int64_t n, uint32_t* out, uint2* ranges, uint32_t* block_sums,
                 uint32_t* total, uint64_t cap, int32_t* flags, int32_t flag_bit, hipStream_t s) {
  const int64_t nb = scan_block_count(n);
  if (nb == 0) return;
  if (n <= kWideChunk) {
    hipLaunchKernelGGL(scan_wide_kernel, dim3(1), dim3(kWideThreads), 0, s, in, n, out, ranges, total, cap, flags,
                       flag_bit);
    return;
  }
  hipLaunchKernelGGL(scan_reduce_kernel, dim3(static_cast<unsigned>(nb)), dim3(256), 0, s, in, n, block_sums);
  hipLaunchKernelGGL(scan_top_kernel, dim3(1), dim3(256), 0, s, block_sums, nb, total, cap, flags, flag_bit);
  hipLaunchKernelGGL(scan_down_kernel, dim3(static_cast<unsigned>(nb)), dim3(256), 0, s, in, n, block_sums, out,
                     ranges);
}

// ------------------------------------------------------------ tile counts
// Largest per-pose tile count whose counters fit an LDS copy (64 KB).
constexpr int kLdsTileMax = 16384;

// One thread per record: the tiles of its pixel rectangle that the support
// ellipse meets (row spans), counted per (pose, tile) for the bucket path and
// per record for the LSD path.  The emit kernels walk the same spans.
__global__ __launch_bounds__(256) void count_tiles_kernel(BinArgs a, uint32_t* tile_count, uint32_t* rec_keys) {
  if (a.flags[0] & 1) return;
  const int pose = blockIdx.y;
  const uint32_t slot = blockIdx.x * 256 + threadIdx.x;
  if (slot >= a.rec_cap || !rec_in_use(a.pose_count, a.rec_cap, pose, slot)) return;
  const int64_t idx = static_cast<int64_t>(pose) * a.rec_cap + slot;
  const uint2 r = a.rects[idx];
  const float4* rp = reinterpret_cast<const float4*>(a.recs + idx);
  const float4 geo = rp[0], hdr = rp[1];
  const SplatShape shp = splat_shape(geo.x, geo.y, geo.z, geo.w, hdr.x, -2.f * rp[2].w);
  const int tx0 = r.x & 0xffff, tx1 = r.x >> 16, ty0 = r.y & 0xffff, ty1 = r.y >> 16;
  uint32_t* tc = tile_count ? tile_count + static_cast<int64_t>(pose) * a.c.tiles_per_pose : nullptr;
  uint32_t ntiles = 0;
  for (int ty = ty0; ty <= ty1; ++ty) {
    int ta, tb;
    row_span(shp, ty, a.c.tile, a.c.W, a.c.H, tx0, tx1, &ta, &tb);
    for (int tx = ta; tx <= tb; ++tx) {
      ++ntiles;
      if (tc) atomicAdd(&tc[ty * a.c.ntx + tx], 1u);
    }
  }
  if (rec_keys) rec_keys[idx] = ntiles;
}

// Many poses (bucket path): a workgroup takes a chunk of kRecChunk in-use
// records of one pose (compacted through the prefix of the pose's
// sub-segment counters, so no thread waits on empty slots; consecutive
// records share tiles) and counts their tile entries in an LDS copy of that
// pose's tile counters, then adds each nonzero counter to global memory once
// (one global atomic per (workgroup, tile) instead of one per entry).  Each
// thread reads its kRecChunk / 256 records with all their loads in flight.
constexpr uint32_t kRecChunk = 1024;
constexpr int kRecPerThread = static_cast<int>(kRecChunk / 256);

// The prefix of one pose's clamped sub-segment counters (s_pre[0] = 0,
// s_pre[kSub] = in-use records), by the first wave; the caller synchronises.
__device__ __forceinline__ void sub_prefix(const uint32_t* pose_count, int pose, uint32_t sub_cap, uint32_t* s_pre) {
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
}

// The slot of compacted record c (binary search of the prefix).
__device__ __forceinline__ uint32_t compact_slot(const uint32_t* s_pre, uint32_t c, uint32_t sub_cap) {
  int lo = 0, hi = kSub;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (s_pre[mid] <= c) lo = mid;
    else hi = mid;
  }
  return static_cast<uint32_t>(lo) * sub_cap + (c - s_pre[lo]);
}

// One thread's records of a chunk: rectangle, geometry and header.
struct ChunkRecs {
  bool ok[kRecPerThread];
  int64_t idx[kRecPerThread];
  uint2 rect[kRecPerThread];
  float4 geo[kRecPerThread], hdr[kRecPerThread];
  float pmin[kRecPerThread];
};

__device__ __forceinline__ void load_chunk_recs(const BinArgs& a, int pose, const uint32_t* s_pre, uint32_t c0,
                                                uint32_t total, ChunkRecs& r) {
  const uint32_t sub_cap = a.rec_cap / kSub;
#pragma unroll
  for (int q = 0; q < kRecPerThread; ++q) {
    const uint32_t c = c0 + threadIdx.x + 256u * q;
    r.ok[q] = c < total;
    r.idx[q] = 0;
    if (r.ok[q]) {
      r.idx[q] = static_cast<int64_t>(pose) * a.rec_cap + compact_slot(s_pre, c, sub_cap);
      const float4* rp = reinterpret_cast<const float4*>(a.recs + r.idx[q]);
      r.rect[q] = a.rects[r.idx[q]];
      r.geo[q] = rp[0];
      r.hdr[q] = rp[1];
      r.pmin[q] = rp[2].w;
    }
  }
}

__global__ __launch_bounds__(256) void count_tiles_lds_kernel(BinArgs a, uint32_t* tile_count) {
  extern __shared__ uint32_t s_hist[];  // tiles_per_pose counters
  __shared__ uint32_t s_pre[kSub + 1];
  if (a.flags[0] & 1) return;
  const int pose = blockIdx.y;
  const int T = a.c.tiles_per_pose;
  sub_prefix(a.pose_count, pose, a.rec_cap / kSub, s_pre);
  __syncthreads();
  const uint32_t total = s_pre[kSub];
  const uint32_t c0 = blockIdx.x * kRecChunk;
  if (c0 >= total) return;  // uniform
  ChunkRecs r;
  load_chunk_recs(a, pose, s_pre, c0, total, r);
  for (int t = threadIdx.x; t < T; t += 256) s_hist[t] = 0;
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kRecPerThread; ++q) {
    if (!r.ok[q]) continue;
    const SplatShape shp = splat_shape(r.geo[q].x, r.geo[q].y, r.geo[q].z, r.geo[q].w, r.hdr[q].x, -2.f * r.pmin[q]);
    const int tx0 = r.rect[q].x & 0xffff, tx1 = r.rect[q].x >> 16, ty0 = r.rect[q].y & 0xffff, ty1 = r.rect[q].y >> 16;
    for (int ty = ty0; ty <= ty1; ++ty) {
      int ta, tb;
      row_span(shp, ty, a.c.tile, a.c.W, a.c.H, tx0, tx1, &ta, &tb);
      for (int tx = ta; tx <= tb; ++tx) atomicAdd(&s_hist[ty * a.c.ntx + tx], 1u);
    }
  }
  __syncthreads();
  uint32_t* tc = tile_count + static_cast<int64_t>(pose) * T;
  for (int t = threadIdx.x; t < T; t += 256) {
    const uint32_t c = s_hist[t];
    if (c) atomicAdd(&tc[t], c);
  }
}

void launch_count_tiles(const BinArgs& a, uint32_t* tile_count, uint32_t* rec_keys, hipStream_t s) {
  if (tile_count && !rec_keys && a.c.tiles_per_pose <= kLdsTileMax) {
    const dim3 grid((a.rec_cap + kRecChunk - 1) / kRecChunk, a.P);
    hipLaunchKernelGGL(count_tiles_lds_kernel, grid, dim3(256), a.c.tiles_per_pose * sizeof(uint32_t), s, a,
                       tile_count);
    return;
  }
  const dim3 grid((a.rec_cap + 255) / 256, a.P);
  hipLaunchKernelGGL(count_tiles_kernel, grid, dim3(256), 0, s, a, tile_count, rec_keys);
}

// ------------------------------------------------------------ bucket path
// Four threads per record, each claiming slots in every fourth overlapped
// tile's bucket (enough waves in flight to hide the atomics' latency).
constexpr int kEmitLanes = 4;

// The pose's used record slots, compacted: records of sub-segment s occupy
// the first min(count_s, sub_cap) of its slots; the prefix over the kSub
// counters maps a compacted index to its slot, so the workgroups walk only
// records (a grid-stride loop) instead of a grid over the whole capacity, most
// of whose waves would find empty slots.
constexpr int kEmitRecsPerBlock = 256 / kEmitLanes;
constexpr int kEmitBlocksPerPose = 2048;

__global__ __launch_bounds__(256) void emit_bucket_kernel(BinArgs a) {
  __shared__ uint32_t s_pre[kSub + 1];
  if (a.flags[0] & 1) return;
  const int pose = blockIdx.y;
  const uint32_t sub_cap = a.rec_cap / kSub;
  if (threadIdx.x < kWave) {
    // inclusive scan of the clamped counters over the first kSub lanes
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
  const uint32_t sub = threadIdx.x % kEmitLanes;
  const int64_t tbase = static_cast<int64_t>(pose) * a.c.tiles_per_pose;
  for (uint32_t c = blockIdx.x * kEmitRecsPerBlock + threadIdx.x / kEmitLanes; c < total;
       c += gridDim.x * kEmitRecsPerBlock) {
    // the sub-segment holding compacted record c (binary search of the prefix)
    int lo = 0, hi = kSub;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (s_pre[mid] <= c) lo = mid;
      else hi = mid;
    }
    const uint32_t slot = static_cast<uint32_t>(lo) * sub_cap + (c - s_pre[lo]);
    const int64_t idx = static_cast<int64_t>(pose) * a.rec_cap + slot;
    const uint2 r = a.rects[idx];
    const float4* rp = reinterpret_cast<const float4*>(a.recs + idx);
    const float4 geo = rp[0], hdr = rp[1];  // u, v, ca, cb | cc, o, z, gid
    const SplatShape shp = splat_shape(geo.x, geo.y, geo.z, geo.w, hdr.x, -2.f * rp[2].w);
    const uint64_t key = (static_cast<uint64_t>(zbits(hdr.z)) << 32) | static_cast<uint64_t>(__float_as_uint(hdr.w));
    const int tx0 = r.x & 0xffff, tx1 = r.x >> 16, ty0 = r.y & 0xffff, ty1 = r.y >> 16;
    // the record's tiles row by row (the projection counted the same spans);
    // the kEmitLanes lanes of a record take every kEmitLanes-th tile in order
    int q = 0;
    for (int ty = ty0; ty <= ty1; ++ty) {
      int ta, tb;
      row_span(shp, ty, a.c.tile, a.c.W, a.c.H, tx0, tx1, &ta, &tb);
      const int first = ta + ((static_cast<int>(sub) - q) % kEmitLanes + kEmitLanes) % kEmitLanes;
      if (tb >= ta) q += tb - ta + 1;
      for (int tx = first; tx <= tb; tx += kEmitLanes) {
        const int64_t tg = tbase + ty * a.c.ntx + tx;
        const uint64_t pos = static_cast<uint64_t>(a.ranges[tg].x) + atomicAdd(&a.tile_cursor[tg], 1u);
        if (pos < a.key_cap) {
          a.keys[pos] = key;
          a.vals[pos] = static_cast<uint32_t>(idx) | (block_mask(shp, tx, ty, a.c.tile) << kRecBits);
        }
      }
    }
  }
}

// Many poses: the same chunk of in-use records as count_tiles_lds_kernel
// counts its entries per tile in LDS, reserves each tile's range with one
// global atomic, and places its entries from LDS cursors.
__global__ __launch_bounds__(256) void emit_bucket_lds_kernel(BinArgs a) {
  extern __shared__ uint32_t s_pos[];  // per tile: count, then next position
  __shared__ uint32_t s_pre[kSub + 1];
  if (a.flags[0] & 1) return;
  const int pose = blockIdx.y;
  const int T = a.c.tiles_per_pose;
  sub_prefix(a.pose_count, pose, a.rec_cap / kSub, s_pre);
  __syncthreads();
  const uint32_t total = s_pre[kSub];
  const uint32_t c0 = blockIdx.x * kRecChunk;
  if (c0 >= total) return;  // uniform
  ChunkRecs r;
  load_chunk_recs(a, pose, s_pre, c0, total, r);
  for (int t = threadIdx.x; t < T; t += 256) s_pos[t] = 0;
  __syncthreads();
  const int64_t tbase = static_cast<int64_t>(pose) * T;
#pragma unroll
  for (int q = 0; q < kRecPerThread; ++q) {
    if (!r.ok[q]) continue;
    const SplatShape shp = splat_shape(r.geo[q].x, r.geo[q].y, r.geo[q].z, r.geo[q].w, r.hdr[q].x, -2.f * r.pmin[q]);
    const int tx0 = r.rect[q].x & 0xffff, tx1 = r.rect[q].x >> 16, ty0 = r.rect[q].y & 0xffff, ty1 = r.rect[q].y >> 16;
    for (int ty = ty0; ty <= ty1; ++ty) {
      int ta, tb;
      row_span(shp, ty, a.c.tile, a.c.W, a.c.H, tx0, tx1, &ta, &tb);
      for (int tx = ta; tx <= tb; ++tx) atomicAdd(&s_pos[ty * a.c.ntx + tx], 1u);
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < T; t += 256) {
    const uint32_t c = s_pos[t];
    if (c) s_pos[t] = a.ranges[tbase + t].x + atomicAdd(&a.tile_cursor[tbase + t], c);
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kRecPerThread; ++q) {
    if (!r.ok[q]) continue;
    const float4 geo = r.geo[q], hdr = r.hdr[q];  // u, v, ca, cb | cc, o, z, gid
    const SplatShape shp = splat_shape(geo.x, geo.y, geo.z, geo.w, hdr.x, -2.f * r.pmin[q]);
    const uint64_t key = (static_cast<uint64_t>(zbits(hdr.z)) << 32) | static_cast<uint64_t>(__float_as_uint(hdr.w));
    const int tx0 = r.rect[q].x & 0xffff, tx1 = r.rect[q].x >> 16, ty0 = r.rect[q].y & 0xffff, ty1 = r.rect[q].y >> 16;
    for (int ty = ty0; ty <= ty1; ++ty) {
      int ta, tb;
      row_span(shp, ty, a.c.tile, a.c.W, a.c.H, tx0, tx1, &ta, &tb);
      for (int tx = ta; tx <= tb; ++tx) {
        const uint64_t pos = atomicAdd(&s_pos[ty * a.c.ntx + tx], 1u);
        if (pos < a.key_cap) {
          a.keys[pos] = key;
          a.vals[pos] = static_cast<uint32_t>(r.idx[q]) | (block_mask(shp, tx, ty, a.c.tile) << kRecBits);
        }
      }
    }
  }
}

void launch_emit_bucket(const BinArgs& a, bool lds, hipStream_t s) {
  if (lds && a.c.tiles_per_pose <= kLdsTileMax) {
    const dim3 grid((a.rec_cap + kRecChunk - 1) / kRecChunk, a.P);
    hipLaunchKernelGGL(emit_bucket_lds_kernel, grid, dim3(256), a.c.tiles_per_pose * sizeof(uint32_t), s, a);
    return;
  }
  const uint32_t blocks = std::min<uint32_t>((a.rec_cap + kEmitRecsPerBlock - 1) / kEmitRecsPerBlock,
                                             static_cast<uint32_t>(kEmitBlocksPerPose));
  hipLaunchKernelGGL(emit_bucket_kernel, dim3(blocks, a.P), dim3(256), 0, s, a);
}

// Short lists (<= 256 entries): one wave per tile (4 tiles per workgroup).
// The wave copies the tile's keys to LDS and each entry's final position is
// its rank, the number of keys below it (keys are unique: the same Gaussian
// enters a tile once); the loop over the keys is uniform, each step one LDS
// broadcast and a 64-bit compare, with no dependent shuffle chain.
template <int RR>
__device__ __forceinline__ void rank_keys(const uint64_t* sk, uint32_t n, const uint64_t* key, uint32_t* rank) {
  uint32_t j = 0;
  for (; j + 4 <= n; j += 4) {
    const uint64_t k0 = sk[j], k1 = sk[j + 1], k2 = sk[j + 2], k3 = sk[j + 3];
#pragma unroll
    for (int q = 0; q < RR; ++q)
      rank[q] += static_cast<uint32_t>(k0 < key[q]) + static_cast<uint32_t>(k1 < key[q]) +
                 static_cast<uint32_t>(k2 < key[q]) + static_cast<uint32_t>(k3 < key[q]);
  }
  for (; j < n; ++j) {
    const uint64_t k0 = sk[j];
#pragma unroll
    for (int q = 0; q < RR; ++q) rank[q] += static_cast<uint32_t>(k0 < key[q]);
  }
}

__global__ __launch_bounds__(256) void tile_sort_wave_kernel(TileSortArgs a) {
  __shared__ uint64_t s_k[4][kWaveSortCap];
  if (a.flags[0] & 3) return;
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x >> 6;
  const int tg = blockIdx.x * 4 + w;
  if (tg >= a.n_tiles) return;
  uint2 r = a.ranges[tg];
  r.x = __builtin_amdgcn_readfirstlane(r.x);  // one tile per wave: uniform
  r.y = __builtin_amdgcn_readfirstlane(r.y);
  const uint32_t n = r.y - r.x;
  if (n <= 1 || n > static_cast<uint32_t>(min(a.lds_cap, kWaveSortCap))) {
    if (n == 1 && lane == 0) {
      a.list[r.x] = a.vals[r.x];
      a.list_gid[r.x] = static_cast<uint32_t>(a.keys[r.x]);
    }
    return;
  }
  const int R = static_cast<int>((n + kWave - 1) / kWave);  // keys per lane, 1..4
  uint64_t key[4];
  uint32_t val[4], rank[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint32_t e = q * kWave + lane;
    key[q] = ~0ull;
    val[q] = 0;
    rank[q] = 0;
    if (q < R && e < n) {
      key[q] = a.keys[r.x + e];
      val[q] = a.vals[r.x + e];
      s_k[w][e] = key[q];
    }
  }
  // the wave's own LDS writes complete before its reads
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  switch (R) {
    case 1: rank_keys<1>(s_k[w], n, key, rank); break;
    case 2: rank_keys<2>(s_k[w], n, key, rank); break;
    default: rank_keys<4>(s_k[w], n, key, rank); break;
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint32_t e = q * kWave + lane;
    if (q < R && e < n) {
      a.list[r.x + rank[q]] = val[q];
      a.list_gid[r.x + rank[q]] = static_cast<uint32_t>(key[q]);
    }
  }
}

// Medium lists (256 < n <= LDS capacity): the workgroup runs a bitonic
// network on (depth bits, gid) keys in LDS.
constexpr int kLdsSortCap = 4096;

__device__ void tile_sort_lds(const TileSortArgs& a, uint2 r, uint32_t n, uint64_t* s_key, uint32_t* s_val) {
  uint32_t m = 2;
  while (m < n) m <<= 1;
  for (uint32_t k = threadIdx.x; k < m; k += 256) {
    if (k < n) {
      s_key[k] = a.keys[r.x + k];
      s_val[k] = a.vals[r.x + k];
    } else {
      s_key[k] = ~0ull;
      s_val[k] = 0;
    }
  }
  __syncthreads();
  for (uint32_t k = 2; k <= m; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t i = threadIdx.x; i < m; i += 256) {
        const uint32_t ixj = i ^ j;
        if (ixj > i) {
          const uint64_t ki = s_key[i], kj = s_key[ixj];
          const bool up = (i & k) == 0;
          if ((ki > kj) == up) {
            s_key[i] = kj;
            s_key[ixj] = ki;
            const uint32_t t = s_val[i];
            s_val[i] = s_val[ixj];
            s_val[ixj] = t;
          }
        }
      }
      __syncthreads();
    }
  }
  for (uint32_t k = threadIdx.x; k < n; k += 256) {
    a.list[r.x + k] = s_val[k];
    a.list_gid[r.x + k] = static_cast<uint32_t>(s_key[k]);
  }
}

// Stable rank of one element per thread within a 256-element chunk, by 8-bit
// digit.  s_wc: 4 x 256 per-wave digit counts (zeroed by the caller).
// Returns the element's rank among equal digits in earlier waves and lanes.
__device__ __forceinline__ uint32_t chunk_rank(uint32_t d, bool valid, uint32_t (*s_wc)[256]) {
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x >> 6;
  uint64_t peers = __ballot(valid);
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t m = __ballot(bit);
    peers &= bit ? m : ~m;
  }
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const uint32_t rank = static_cast<uint32_t>(__popcll(peers & lt));
  if (valid && rank == 0) s_wc[w][d] = static_cast<uint32_t>(__popcll(peers));
  __syncthreads();
  uint32_t before = 0;
  if (valid)
    for (int k = 0; k < w; ++k) before += s_wc[k][d];
  return before + rank;
}

// Lists longer than the LDS capacity: one block runs a stable LSD radix sort
// of that tile's keys in global memory (ping-pong with the alternate buffers).
__device__ void tile_sort_global(const TileSortArgs& a, uint2 r, uint32_t n, uint32_t* s_off, uint32_t (*s_wc)[256],
                                 uint32_t* s_w) {
  uint64_t* sk = a.keys + r.x;
  uint32_t* sv = a.vals + r.x;
  uint64_t* dk = a.keys_alt + r.x;
  uint32_t* dv = a.vals_alt + r.x;
  const int gid_passes = (a.gid_bits + 7) / 8;
  const int passes = gid_passes + 4;
  for (int p = 0; p < passes; ++p) {
    const int shift = p < gid_passes ? 8 * p : 32 + 8 * (p - gid_passes);
    s_off[threadIdx.x] = 0;
    __syncthreads();
    for (uint32_t e = threadIdx.x; e < n; e += 256) atomicAdd(&s_off[(sk[e] >> shift) & 0xff], 1u);
    __syncthreads();
    uint32_t tot;
    const uint32_t ex = block_excl_scan256(s_off[threadIdx.x], s_w, &tot);
    __syncthreads();
    s_off[threadIdx.x] = ex;
    for (uint32_t base = 0; base < n; base += 256) {
      for (int w = 0; w < 4; ++w) s_wc[w][threadIdx.x] = 0;
      __syncthreads();
      const uint32_t e = base + threadIdx.x;
      const bool valid = e < n;
      uint64_t key = 0;
      uint32_t val = 0, d = 0;
      if (valid) {
        key = sk[e];
        val = sv[e];
        d = static_cast<uint32_t>((key >> shift) & 0xff);
      }
      const uint32_t rk = chunk_rank(d, valid, s_wc);
      if (valid) {
        const uint32_t pos = s_off[d] + rk;
        dk[pos] = key;
        dv[pos] = val;
      }
      __syncthreads();
      s_off[threadIdx.x] += s_wc[0][threadIdx.x] + s_wc[1][threadIdx.x] + s_wc[2][threadIdx.x] + s_wc[3][threadIdx.x];
      __syncthreads();
    }
    uint64_t* tk = sk; sk = dk; dk = tk;
    uint32_t* tv = sv; sv = dv; dv = tv;
    __syncthreads();
  }
  for (uint32_t k = threadIdx.x; k < n; k += 256) {
    a.list[r.x + k] = sv[k];
    a.list_gid[r.x + k] = static_cast<uint32_t>(sk[k]);
  }
}

// Lists longer than one wave sorts: the workgroup sorts them in LDS up to the
// LDS capacity, or with a stable LSD radix sort in global memory beyond it.
constexpr int kLongSortCtas = 768;  // three workgroups per CU

// Lists too long for one wave: each workgroup walks every gridDim.x-th tile
// (most have short lists and are skipped; the 48 KB of LDS leaves room for
// only three workgroups per CU, so a workgroup per tile would mostly queue).
__global__ __launch_bounds__(256) void tile_sort_long_kernel(TileSortArgs a) {
  __shared__ uint64_t s_key[kLdsSortCap];
  __shared__ uint32_t s_val[kLdsSortCap];
  __shared__ uint64_t s_long[256 / kWave];  // per wave: which of its lanes' tiles are long
  if (a.flags[0] & 3) return;
  const uint32_t short_max = static_cast<uint32_t>(min(a.lds_cap, kWaveSortCap));
  // the workgroup's tiles (every gridDim.x-th) looked at 256 at a time, one
  // range load per thread, and only the long ones sorted
  for (int64_t t0 = blockIdx.x; t0 < a.n_tiles; t0 += static_cast<int64_t>(gridDim.x) * 256) {
    const int64_t t = t0 + static_cast<int64_t>(threadIdx.x) * gridDim.x;
    bool is_long = false;
    if (t < a.n_tiles) {
      const uint2 r = a.ranges[t];
      is_long = r.y - r.x > short_max;
    }
    const uint64_t bal = __ballot(is_long);
    if ((threadIdx.x & (kWave - 1)) == 0) s_long[threadIdx.x / kWave] = bal;
    __syncthreads();
    for (int w = 0; w < 256 / kWave; ++w) {
      uint64_t m = s_long[w];  // uniform
      while (m) {
        const int l = __builtin_ctzll(m);
        m &= m - 1;
        const int64_t tl = t0 + static_cast<int64_t>(w * kWave + l) * gridDim.x;
        const uint2 r = a.ranges[tl];
        const uint32_t n = r.y - r.x;
        if (n <= static_cast<uint32_t>(a.lds_cap)) {
          tile_sort_lds(a, r, n, s_key, s_val);
        } else {
          // reuse the key array's LDS for the radix pass state
          uint32_t* base = reinterpret_cast<uint32_t*>(s_key);
          tile_sort_global(a, r, n, base, reinterpret_cast<uint32_t(*)[256]>(base + 256), base + 256 + 4 * 256);
        }
        __syncthreads();  // the LDS is reused by the next tile
      }
    }
    __syncthreads();  // s_long is rewritten by the next round
  }
}

void launch_tile_sort(const TileSortArgs& a, bool short_lists, hipStream_t s) {
  if (a.n_tiles <= 0) return;
  if (short_lists) hipLaunchKernelGGL(tile_sort_wave_kernel, dim3((a.n_tiles + 3) / 4), dim3(256), 0, s, a);
  hipLaunchKernelGGL(tile_sort_long_kernel, dim3(a.n_tiles < kLongSortCtas ? a.n_tiles : kLongSortCtas), dim3(256), 0,
                     s, a);
}

// ------------------------------------------------------------ LSD path
__global__ __launch_bounds__(256) void emit_lsd_kernel(BinArgs a, const uint32_t* rec_offsets, uint64_t* keys,
                                                       uint32_t* gids, uint32_t* vals) {
  if (a.flags[0] & 3) return;
  const int pose = blockIdx.y;
  const uint32_t slot = blockIdx.x * 256 + threadIdx.x;
  if (slot >= a.rec_cap || !rec_in_use(a.pose_count, a.rec_cap, pose, slot)) return;
  const int64_t idx = static_cast<int64_t>(pose) * a.rec_cap + slot;
  const uint2 r = a.rects[idx];
  const float4* rp = reinterpret_cast<const float4*>(a.recs + idx);
  const float4 geo = rp[0], hdr = rp[1];
  const SplatShape shp = splat_shape(geo.x, geo.y, geo.z, geo.w, hdr.x, -2.f * rp[2].w);
  const uint32_t zb = zbits(hdr.z), gid = __float_as_uint(hdr.w);
  const int tx0 = r.x & 0xffff, tx1 = r.x >> 16, ty0 = r.y & 0xffff, ty1 = r.y >> 16;
  uint64_t pos = rec_offsets[idx];
  const int64_t tbase = static_cast<int64_t>(pose) * a.c.tiles_per_pose;
  for (int ty = ty0; ty <= ty1; ++ty) {
    int ta, tb;
    row_span(shp, ty, a.c.tile, a.c.W, a.c.H, tx0, tx1, &ta, &tb);
    for (int tx = ta; tx <= tb; ++tx) {
      if (pos >= a.key_cap) {
        ++pos;
        continue;
      }
      keys[pos] = (static_cast<uint64_t>(tbase + ty * a.c.ntx + tx) << 32) | zb;
      gids[pos] = gid;
      vals[pos] = static_cast<uint32_t>(idx) | (block_mask(shp, tx, ty, a.c.tile) << kRecBits);
      ++pos;
    }
  }
}

void launch_emit_lsd(const BinArgs& a, const uint32_t* rec_offsets, uint64_t* keys, uint32_t* gids,
                     uint32_t* vals, hipStream_t s) {
  const dim3 grid((a.rec_cap + 255) / 256, a.P);
  hipLaunchKernelGGL(emit_lsd_kernel, grid, dim3(256), 0, s, a, rec_offsets, keys, gids, vals);
}

constexpr int kLsdItems = 8;
constexpr int kLsdChunk = 256 * kLsdItems;

__device__ __forceinline__ uint32_t lsd_digit(uint64_t key, uint32_t gid, int shift) {
  // shift < 0: gid digit at bit -shift-1 ... encoded as shift = -(8k + 1)
  return shift >= 0 ? static_cast<uint32_t>((key >> shift) & 0xff) : ((gid >> (-shift - 1)) & 0xffu);
}

__global__ __launch_bounds__(256) void lsd_hist_kernel(LsdArgs a, int src, int shift) {
  __shared__ uint32_t s_h[256];
  s_h[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t total = (a.flags[0] & 3) ? 0u : min(*a.total, static_cast<uint32_t>(a.key_cap));
  const uint64_t base = static_cast<uint64_t>(blockIdx.x) * kLsdChunk;
  for (int k = 0; k < kLsdItems; ++k) {
    const uint64_t e = base + k * 256 + threadIdx.x;
    if (e < total) atomicAdd(&s_h[lsd_digit(a.keys[src][e], a.gids[src][e], shift)], 1u);
  }
  __syncthreads();
  a.hist[static_cast<int64_t>(threadIdx.x) * a.n_blocks + blockIdx.x] = s_h[threadIdx.x];
}

__global__ __launch_bounds__(256) void lsd_scatter_kernel(LsdArgs a, int src, int shift) {
  __shared__ uint32_t s_off[256];
  __shared__ uint32_t s_wc[4][256];
  const uint32_t total = (a.flags[0] & 3) ? 0u : min(*a.total, static_cast<uint32_t>(a.key_cap));
  const uint64_t base = static_cast<uint64_t>(blockIdx.x) * kLsdChunk;
  if (base >= total) return;
  s_off[threadIdx.x] = a.hist[static_cast<int64_t>(threadIdx.x) * a.n_blocks + blockIdx.x];
  const int dst = src ^ 1;
  for (int k = 0; k < kLsdItems; ++k) {
    for (int w = 0; w < 4; ++w) s_wc[w][threadIdx.x] = 0;
    __syncthreads();
    const uint64_t e = base + k * 256 + threadIdx.x;
    const bool valid = e < total;
    uint64_t key = 0;
    uint32_t gid = 0, val = 0, d = 0;
    if (valid) {
      key = a.keys[src][e];
      gid = a.gids[src][e];
      val = a.vals[src][e];
      d = lsd_digit(key, gid, shift);
    }
    const uint32_t rk = chunk_rank(d, valid, s_wc);
    if (valid) {
      const uint32_t pos = s_off[d] + rk;
      a.keys[dst][pos] = key;
      a.gids[dst][pos] = gid;
      a.vals[dst][pos] = val;
    }
    __syncthreads();
    s_off[threadIdx.x] += s_wc[0][threadIdx.x] + s_wc[1][threadIdx.x] + s_wc[2][threadIdx.x] + s_wc[3][threadIdx.x];
    __syncthreads();
  }
}

void launch_lsd_sort(LsdArgs& a, int passes_gid, int passes_z, int passes_tile, int* out_buffer, hipStream_t s) {
  int src = 0;
  const int passes = passes_gid + passes_z + passes_tile;
  const int64_t nh = static_cast<int64_t>(a.n_blocks) * 256;
  for (int p = 0; p < passes; ++p) {
    int shift;
    if (p < passes_gid) shift = -(8 * p + 1);
    else if (p < passes_gid + passes_z) shift = 8 * (p - passes_gid);
    else shift = 32 + 8 * (p - passes_gid - passes_z);
    hipLaunchKernelGGL(lsd_hist_kernel, dim3(a.n_blocks), dim3(256), 0, s, a, src, shift);
    launch_scan(a.hist, nh, a.hist, nullptr, a.hist + nh, nullptr, ~0ull, nullptr, 0, s);
    hipLaunchKernelGGL(lsd_scatter_kernel, dim3(a.n_blocks), dim3(256), 0, s, a, src, shift);
    src ^= 1;
  }
  *out_buffer = src;
}

__global__ void ranges_from_sorted_kernel(const uint64_t* keys, const uint32_t* total_p, uint64_t key_cap,
                                          uint2* ranges, const int32_t* flags) {
  if (flags[0] & 3) return;
  const uint32_t total = min(*total_p, static_cast<uint32_t>(key_cap));
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < total;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const uint32_t t = static_cast<uint32_t>(keys[i] >> 32);
    if (i == 0 || static_cast<uint32_t>(keys[i - 1] >> 32) != t) ranges[t].x = static_cast<uint32_t>(i);
    if (i + 1 == total || static_cast<uint32_t>(keys[i + 1] >> 32) != t) ranges[t].y = static_cast<uint32_t>(i + 1);
  }
}

void launch_ranges_from_sorted(const uint64_t* keys, const uint32_t* total, uint64_t key_cap, uint2* ranges,
                               int32_t n_tiles, const int32_t* flags, hipStream_t s) {
  launch_fill_u32(reinterpret_cast<uint32_t*>(ranges), 0u, 2 * static_cast<int64_t>(n_tiles), s);
  hipLaunchKernelGGL(ranges_from_sorted_kernel, dim3(fill_grid(static_cast<int64_t>(key_cap))), dim3(256), 0, s,
                     keys, total, key_cap, ranges, flags);
}

}  // namespace hgsr
