// Partition streaming: the partitioned scene (Sec. 3.1's spatial cells) kept
// in pinned host memory, a fixed device budget of slots, and per batch of
// poses the uploads that make the cells it may see resident (Sec. 3.2's
// batch processing under a memory budget with intermediate data released).
//
// Device layout: every per-Gaussian array of the descriptor is n_slots x
// capacity entries, slot s holding one partition at [s x capacity, s x
// capacity + count) and opacity 0 behind it; per-slot offsets and boxes make
// the slots the descriptor's partitions, so the renderer's partition test
// skips slots a pose cannot see and empty slots (empty boxes) always.
//
// Ordering without host waits: uploads run on the cache's copy stream, each
// slot's followed by an event of its own.  At the start of a prepare one
// event is recorded on the render stream (it completes once the previous
// batches' work has); a slot's data is overwritten only after the copy
// stream has waited for the event of the first batch after the slot's last
// use, so uploads into least recently used slots overlap the previous
// batch's renders.  The slot table (offsets are fixed; boxes change) is rewritten by
// a kernel on the render stream, after the previous renders by stream order
// and after the uploads of exactly the slots it makes visible -- uploads for
// upcoming views stay invisible, and unwaited, until a later table shows
// them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/hgsr.h"
#include "host.hpp"
#include "launch.hpp"

using namespace hgsr;
using host::SlotPolicy;

namespace {

constexpr int kMaxSlots = host::kMaxSlots;

hgsr_status err(hgsr_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
hgsr_status err(hgsr_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  return report_error(st, buf);
}

#define PC_HIP(expr)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) return err(HGSR_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// Per-Gaussian array sizes in bytes.
struct Widths {
  size_t means, ls, quats, opac, sh, feat;
  explicit Widths(int sh_degree, int feat_dim)
      : means(12), ls(12), quats(16), opac(4), sh(12 * static_cast<size_t>((sh_degree + 1) * (sh_degree + 1))),
        feat(2 * static_cast<size_t>(feat_dim)) {}
  size_t total() const { return means + ls + quats + opac + sh + feat; }
};

// Slot boxes passed by value (a kernel argument is copied at launch, so the
// host table may change right after the call).
struct SlotBoxes {
  float b[kMaxSlots][6];
};

__global__ void write_boxes_kernel(SlotBoxes t, int n, float* out) {
  const int i = threadIdx.x;
  if (i < n)
    for (int k = 0; k < 6; ++k) out[6 * i + k] = t.b[i][k];
}

__global__ void zero_tail_kernel(float* opac, int64_t count) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < count) opac[i] = 0.f;
}

}  // namespace

struct hgsr_pcache {
  int device = 0;
  int64_t n = 0;
  int32_t sh_degree = 0, feat_dim = 0, n_parts = 0;
  std::vector<int64_t> offs;
  std::vector<float> bounds;  // n_parts x 6
  // pinned host copy
  char* host = nullptr;
  const char *h_means = nullptr, *h_ls = nullptr, *h_quats = nullptr, *h_opac = nullptr, *h_sh = nullptr,
             *h_feat = nullptr;
  // device slots
  int32_t n_slots = 0;
  int64_t cap = 0;
  char* dev = nullptr;
  size_t dev_bytes = 0;
  char *d_means = nullptr, *d_ls = nullptr, *d_quats = nullptr, *d_opac = nullptr, *d_sh = nullptr,
       *d_feat = nullptr;
  int64_t* d_offs = nullptr;
  float* d_bounds = nullptr;
  std::vector<float> slot_box;      // n_slots x 6
  // which partition each slot holds; each upload's release batch
  SlotPolicy pol{1, 1};
  // batch_ev[b % kRing], recorded on the render stream at the start of
  // prepare b, completes once every batch before b has; a slot last used by
  // batch L may be overwritten after batch_ev of L + 1 (or of a later batch)
  static constexpr int kRing = SlotPolicy::kRing;
  std::vector<hipEvent_t> batch_ev;
  std::vector<hipEvent_t> slot_ready;  // recorded on the copy stream after a slot's upload
  std::vector<uint8_t> slot_pending;   // uploaded, not yet waited for by the render stream
  bool table_dirty = false;         // slot boxes changed since the device table was written
  hipStream_t copy = nullptr;
  hgsr_pcache_stats st{};
};

namespace {

void release_all(hgsr_pcache* pc) {
  if (pc->copy) (void)hipStreamSynchronize(pc->copy);
  for (hipEvent_t e : pc->batch_ev)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : pc->slot_ready)
    if (e) (void)hipEventDestroy(e);
  if (pc->copy) (void)hipStreamDestroy(pc->copy);
  if (pc->dev) (void)hipFree(pc->dev);
  if (pc->host) (void)hipHostFree(pc->host);
}

}  // namespace

extern "C" {

hgsr_status hgsr_pcache_create(hgsr_pcache** out, const hgsr_host_scene* scene, int32_t n_slots) {
  if (!out) return err(HGSR_ERR_INVALID_ARG, "NULL output");
  *out = nullptr;
  hgsr_status s = host::check_host_scene(scene);
  if (s != HGSR_OK) return s;
  if (n_slots < 1 || n_slots > kMaxSlots || n_slots > scene->n_parts)
    return err(HGSR_ERR_INVALID_ARG, "n_slots must be 1..min(64, n_parts)");
  hgsr_pcache* pc = new hgsr_pcache();
  pc->n = scene->n;
  pc->sh_degree = scene->sh_degree;
  pc->feat_dim = scene->feat_dim;
  pc->n_parts = scene->n_parts;
  pc->offs.assign(scene->part_offsets, scene->part_offsets + scene->n_parts + 1);
  pc->bounds.resize(6 * static_cast<size_t>(scene->n_parts));
  host::partition_bounds(scene, pc->bounds.data());
  for (int k = 0; k < pc->n_parts; ++k) pc->cap = std::max<int64_t>(pc->cap, pc->offs[k + 1] - pc->offs[k]);
  pc->cap = std::max<int64_t>(pc->cap, 1);
  if (static_cast<int64_t>(n_slots) * pc->cap >= (1ll << 31)) {
    delete pc;
    return err(HGSR_ERR_INVALID_ARG, "n_slots x largest partition must stay below 2^31 Gaussians");
  }
  pc->n_slots = n_slots;
  const Widths w(pc->sh_degree, pc->feat_dim);
  auto fail_free = [&](hgsr_status st) {
    release_all(pc);
    delete pc;
    return st;
  };
  if (hipGetDevice(&pc->device) != hipSuccess) return fail_free(err(HGSR_ERR_HIP, "hipGetDevice failed"));
  // pinned host copy, one block, arrays 256-byte aligned
  const int64_t n = pc->n;
  const size_t hb[6] = {align256(n * w.means), align256(n * w.ls), align256(n * w.quats), align256(n * w.opac),
                        align256(n * w.sh), align256(n * w.feat)};
  size_t htotal = 0;
  for (size_t b : hb) htotal += b;
  hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&pc->host), std::max<size_t>(htotal, 256), hipHostMallocDefault);
  if (e != hipSuccess) {
    pc->host = nullptr;
    return fail_free(err(HGSR_ERR_HIP, "hipHostMalloc(%zu): %s", htotal, hipGetErrorString(e)));
  }
  {
    char* p = pc->host;
    const void* src[6] = {scene->means, scene->log_scales, scene->quats, scene->opacities, scene->sh, scene->feat};
    const size_t bytes[6] = {n * w.means, n * w.ls, n * w.quats, n * w.opac, n * w.sh, n * w.feat};
    const char** dst[6] = {&pc->h_means, &pc->h_ls, &pc->h_quats, &pc->h_opac, &pc->h_sh, &pc->h_feat};
    for (int a = 0; a < 6; ++a) {
      *dst[a] = p;
      if (bytes[a]) std::memcpy(p, src[a], bytes[a]);
      p += hb[a];
    }
  }
  // device slots + tables
  const int64_t m = static_cast<int64_t>(n_slots) * pc->cap;
  const size_t db[8] = {align256(m * w.means), align256(m * w.ls), align256(m * w.quats), align256(m * w.opac),
                        align256(m * w.sh), align256(m * w.feat),
                        align256((n_slots + 1) * sizeof(int64_t)), align256(6 * n_slots * sizeof(float))};
  size_t dtotal = 0;
  for (size_t b : db) dtotal += b;
  e = hipMalloc(reinterpret_cast<void**>(&pc->dev), dtotal);
  if (e != hipSuccess) {
    pc->dev = nullptr;
    return fail_free(err(HGSR_ERR_HIP, "hipMalloc(%zu) for %d slots: %s", dtotal, n_slots, hipGetErrorString(e)));
  }
  pc->dev_bytes = dtotal;
  {
    char* p = pc->dev;
    char** dst[6] = {&pc->d_means, &pc->d_ls, &pc->d_quats, &pc->d_opac, &pc->d_sh, &pc->d_feat};
    for (int a = 0; a < 6; ++a) {
      *dst[a] = p;
      p += db[a];
    }
    pc->d_offs = reinterpret_cast<int64_t*>(p);
    p += db[6];
    pc->d_bounds = reinterpret_cast<float*>(p);
  }
  if (hipMemset(pc->dev, 0, dtotal) != hipSuccess) return fail_free(err(HGSR_ERR_HIP, "hipMemset failed"));
  std::vector<int64_t> so(n_slots + 1);
  for (int sl = 0; sl <= n_slots; ++sl) so[sl] = sl * pc->cap;
  pc->slot_box.assign(6 * static_cast<size_t>(n_slots), 0.f);
  for (int sl = 0; sl < n_slots; ++sl)
    for (int a = 0; a < 3; ++a) {
      pc->slot_box[6 * sl + a] = 1.f;
      pc->slot_box[6 * sl + 3 + a] = -1.f;
    }
  if (hipMemcpy(pc->d_offs, so.data(), so.size() * sizeof(int64_t), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(pc->d_bounds, pc->slot_box.data(), pc->slot_box.size() * sizeof(float), hipMemcpyHostToDevice) !=
          hipSuccess)
    return fail_free(err(HGSR_ERR_HIP, "hipMemcpy of the slot tables failed"));
  pc->pol = SlotPolicy(pc->n_parts, n_slots);
  pc->batch_ev.assign(hgsr_pcache::kRing, nullptr);
  pc->slot_ready.assign(n_slots, nullptr);
  pc->slot_pending.assign(n_slots, 0);
  for (int sl = 0; sl < n_slots; ++sl)
    if (hipEventCreateWithFlags(&pc->slot_ready[sl], hipEventDisableTiming) != hipSuccess)
      return fail_free(err(HGSR_ERR_HIP, "hipEventCreate failed"));
  for (int r = 0; r < hgsr_pcache::kRing; ++r)
    if (hipEventCreateWithFlags(&pc->batch_ev[r], hipEventDisableTiming) != hipSuccess)
      return fail_free(err(HGSR_ERR_HIP, "hipEventCreate failed"));
  if (hipStreamCreateWithFlags(&pc->copy, hipStreamNonBlocking) != hipSuccess)
    return fail_free(err(HGSR_ERR_HIP, "stream or event creation failed"));
  pc->st.n_slots = n_slots;
  pc->st.slot_capacity = pc->cap;
  pc->st.device_bytes = static_cast<int64_t>(dtotal);
  *out = pc;
  return HGSR_OK;
}

hgsr_status hgsr_pcache_destroy(hgsr_pcache* pc) {
  if (!pc) return HGSR_OK;
  release_all(pc);
  delete pc;
  return HGSR_OK;
}

hgsr_status hgsr_pcache_evict_all(hgsr_pcache* pc) {
  if (!pc) return err(HGSR_ERR_INVALID_ARG, "NULL cache");
  PC_HIP(hipStreamSynchronize(pc->copy));
  // the slots' last uses stay recorded: their next uploads still wait for them
  pc->pol.evict_all();
  for (int sl = 0; sl < pc->n_slots; ++sl) {
    for (int a = 0; a < 3; ++a) {  // empty box: never drawn again
      pc->slot_box[6 * sl + a] = 1.f;
      pc->slot_box[6 * sl + 3 + a] = -1.f;
    }
    pc->slot_pending[sl] = 0;  // the copy stream has finished
  }
  pc->table_dirty = true;  // written by the next prepare, after the work already enqueued
  return HGSR_OK;
}

hgsr_status hgsr_pcache_prepare(hgsr_pcache* pc, const float* poses, int32_t P, int32_t n_render,
                                const hgsr_intrinsics* K, float near_z, float motion_margin, hgsr_gaussians* out,
                                hgsr_pcache_stats* stats, hgsr_stream stream) {
  if (!pc || !out) return err(HGSR_ERR_INVALID_ARG, "NULL cache or output");
  hgsr_status s = host::check_plan_args(pc->n_parts, poses, P, K, near_z, motion_margin);
  if (s != HGSR_OK) return s;
  if (n_render < 1 || n_render > P) return err(HGSR_ERR_INVALID_ARG, "n_render must be 1..P");
  const float nz = near_z > 0.f ? near_z : 0.2f;
  // partitions the rendered views may see (need 1) and, not among them, the
  // ones only the upcoming views may see (need 2)
  std::vector<uint8_t> need(pc->n_parts, 0);
  for (int k = 0; k < pc->n_parts; ++k) {
    const float* B = pc->bounds.data() + 6 * k;
    for (int p = 0; p < n_render && !need[k]; ++p)
      need[k] = host::box_may_be_seen(B, poses + 12 * p, *K, nz, motion_margin) ? 1 : 0;
    for (int p = n_render; p < P && !need[k]; ++p)
      need[k] = host::box_may_be_seen(B, poses + 12 * p, *K, nz, motion_margin) ? 2 : 0;
  }
  hgsr_pcache_stats& st = pc->st;
  const int64_t batch = pc->pol.batch;
  s = pc->pol.step(need.data(), &st);  // nothing changes on HGSR_ERR_CAPACITY
  if (s != HGSR_OK) return s;
  hipStream_t rs = reinterpret_cast<hipStream_t>(stream);
  // everything enqueued before this batch (the release point of the slots the
  // previous batch used)
  PC_HIP(hipEventRecord(pc->batch_ev[batch % hgsr_pcache::kRing], rs));
  st.bytes_uploaded = 0;
  const Widths w(pc->sh_degree, pc->feat_dim);
  const float kEmpty[6] = {1.f, 1.f, 1.f, -1.f, -1.f, -1.f};
  // uploads in the policy's order (the rendered views' misses, then the
  // upcoming views'), each after the release point of its slot's previous use
  for (int u = 0; u < st.uploads; ++u) {
    const hgsr_slot_upload& up = st.upload[u];
    const int k = up.part, v = up.slot;
    if (up.release >= 0) PC_HIP(hipStreamWaitEvent(pc->copy, pc->batch_ev[up.release % hgsr_pcache::kRing], 0));
    const int64_t b = pc->offs[k], cnt = pc->offs[k + 1] - pc->offs[k];
    const int64_t d0 = static_cast<int64_t>(v) * pc->cap;
    const char* hsrc[6] = {pc->h_means, pc->h_ls, pc->h_quats, pc->h_opac, pc->h_sh, pc->h_feat};
    char* ddst[6] = {pc->d_means, pc->d_ls, pc->d_quats, pc->d_opac, pc->d_sh, pc->d_feat};
    const size_t wid[6] = {w.means, w.ls, w.quats, w.opac, w.sh, w.feat};
    for (int a = 0; a < 6; ++a) {
      if (!wid[a] || !cnt) continue;
      PC_HIP(hipMemcpyAsync(ddst[a] + d0 * wid[a], hsrc[a] + b * wid[a], cnt * wid[a], hipMemcpyHostToDevice,
                            pc->copy));
    }
    const int64_t tail = pc->cap - cnt;
    if (tail > 0)
      hipLaunchKernelGGL(zero_tail_kernel, dim3(static_cast<unsigned>((tail + 255) / 256)), dim3(256), 0, pc->copy,
                         reinterpret_cast<float*>(pc->d_opac) + d0 + cnt, tail);
    PC_HIP(hipGetLastError());
    PC_HIP(hipEventRecord(pc->slot_ready[v], pc->copy));
    pc->slot_pending[v] = 1;
    st.bytes_uploaded += cnt * static_cast<int64_t>(w.total());
    // an upcoming view's slot stays empty in this batch's table
    const float* box = up.ahead ? kEmpty : pc->bounds.data() + 6 * k;
    std::copy(box, box + 6, pc->slot_box.begin() + 6 * v);
    pc->table_dirty = true;
  }
  // the slot table on the render stream: after the previous renders (stream
  // order) and after the uploads of the slots it shows
  if (pc->table_dirty) {
    SlotBoxes t;
    std::memset(&t, 0, sizeof(t));
    for (int sl = 0; sl < pc->n_slots; ++sl) {
      for (int a = 0; a < 6; ++a) t.b[sl][a] = pc->slot_box[6 * sl + a];
      if (pc->slot_pending[sl] && !host::empty_box(&pc->slot_box[6 * sl])) {
        PC_HIP(hipStreamWaitEvent(rs, pc->slot_ready[sl], 0));
        pc->slot_pending[sl] = 0;
      }
    }
    hipLaunchKernelGGL(write_boxes_kernel, dim3(1), dim3(64), 0, rs, t, pc->n_slots, pc->d_bounds);
    PC_HIP(hipGetLastError());
    pc->table_dirty = false;
  }
  // the upcoming views' slots show their boxes from the next table on
  for (int u = 0; u < st.uploads; ++u)
    if (st.upload[u].ahead) {
      const float* box = pc->bounds.data() + 6 * st.upload[u].part;
      std::copy(box, box + 6, pc->slot_box.begin() + 6 * st.upload[u].slot);
      pc->table_dirty = true;
    }
  st.total_uploads += st.uploads;
  st.total_bytes += st.bytes_uploaded;
  out->n = static_cast<int64_t>(pc->n_slots) * pc->cap;
  out->means = reinterpret_cast<const float*>(pc->d_means);
  out->log_scales = reinterpret_cast<const float*>(pc->d_ls);
  out->quats = reinterpret_cast<const float*>(pc->d_quats);
  out->opacities = reinterpret_cast<const float*>(pc->d_opac);
  out->sh = reinterpret_cast<const float*>(pc->d_sh);
  out->sh_degree = pc->sh_degree;
  out->feat_dim = pc->feat_dim;
  out->feat = pc->feat_dim ? reinterpret_cast<const uint16_t*>(pc->d_feat) : nullptr;
  out->n_parts = pc->n_slots;
  out->part_offsets = pc->d_offs;
  out->part_bounds = pc->d_bounds;
  if (stats) *stats = st;
  return HGSR_OK;
}

}  // extern "C"
