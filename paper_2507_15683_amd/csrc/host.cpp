// Host-only parts of the library: partition boxes and the per-pose plan of
// a partitioned scene (Sec. 3.1's spatial cells), the partition cache's slot
// policy (Sec. 3.2's batches under a memory budget, intermediate data
// released), and the spatial (Morton) order in which scenes are stored.
#include "host.hpp"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <vector>

namespace hgsr {
namespace host {

hgsr_status fail(hgsr_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  return report_error(st, buf);
}

bool empty_box(const float* B) { return !(B[0] <= B[3] && B[1] <= B[4] && B[2] <= B[5]); }

hgsr_status check_host_scene(const hgsr_host_scene* s) {
  if (!s) return fail(HGSR_ERR_INVALID_ARG, "NULL scene");
  if (s->n < 0) return fail(HGSR_ERR_INVALID_ARG, "n < 0");
  if (s->sh_degree < 0 || s->sh_degree > 3) return fail(HGSR_ERR_INVALID_ARG, "sh_degree must be 0..3");
  if (!(s->feat_dim == 0 || s->feat_dim == 8 || s->feat_dim == 16 || s->feat_dim == 32 || s->feat_dim == 64))
    return fail(HGSR_ERR_INVALID_ARG, "feat_dim must be 0, 8, 16, 32 or 64");
  if (s->n > 0 && (!s->means || !s->log_scales || !s->quats || !s->opacities || !s->sh))
    return fail(HGSR_ERR_INVALID_ARG, "scene arrays are NULL");
  if (s->n > 0 && s->feat_dim > 0 && !s->feat) return fail(HGSR_ERR_INVALID_ARG, "feat is NULL");
  if (s->n_parts < 1 || !s->part_offsets) return fail(HGSR_ERR_INVALID_ARG, "need n_parts >= 1 and part_offsets");
  if (s->part_offsets[0] != 0 || s->part_offsets[s->n_parts] != s->n)
    return fail(HGSR_ERR_INVALID_ARG, "part_offsets must run from 0 to n");
  for (int k = 0; k < s->n_parts; ++k)
    if (s->part_offsets[k + 1] < s->part_offsets[k]) return fail(HGSR_ERR_INVALID_ARG, "part_offsets decrease");
  return HGSR_OK;
}

void partition_bounds(const hgsr_host_scene* s, float* out) {
  for (int k = 0; k < s->n_parts; ++k) {
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = s->part_offsets[k]; i < s->part_offsets[k + 1]; ++i) {
      const float* l = s->log_scales + 3 * i;
      const double r = kSupport * std::exp(static_cast<double>(std::max(l[0], std::max(l[1], l[2]))));
      for (int a = 0; a < 3; ++a) {
        const double m = s->means[3 * i + a];
        lo[a] = std::min(lo[a], m - r);
        hi[a] = std::max(hi[a], m + r);
      }
    }
    for (int a = 0; a < 3; ++a) {
      // outward rounding to float
      float fl = static_cast<float>(lo[a]), fh = static_cast<float>(hi[a]);
      if (static_cast<double>(fl) > lo[a]) fl = std::nextafter(fl, -INFINITY);
      if (static_cast<double>(fh) < hi[a]) fh = std::nextafter(fh, INFINITY);
      out[6 * k + a] = fl;
      out[6 * k + 3 + a] = fh;
    }
    if (s->part_offsets[k + 1] == s->part_offsets[k]) {
      for (int a = 0; a < 3; ++a) {
        out[6 * k + a] = 1.f;
        out[6 * k + 3 + a] = -1.f;
      }
    }
  }
}

bool box_may_be_seen(const float* B, const float* T, const hgsr_intrinsics& K, double near_z, double grow) {
  if (empty_box(B)) return false;
  const double margin = 9.0 + 0.05 * std::max(K.width, K.height);
  const double l = (-margin - K.cx) / K.fx, r = (K.width + margin - K.cx) / K.fx;
  const double t = (-margin - K.cy) / K.fy, b = (K.height + margin - K.cy) / K.fy;
  bool all_near = true, all_l = true, all_r = true, all_t = true, all_b = true;
  for (int q = 0; q < 8; ++q) {
    const double w[3] = {(q & 1) ? B[3] + grow : B[0] - grow, (q & 2) ? B[4] + grow : B[1] - grow,
                         (q & 4) ? B[5] + grow : B[2] - grow};
    double m[3];
    for (int r3 = 0; r3 < 3; ++r3)
      m[r3] = T[4 * r3] * w[0] + T[4 * r3 + 1] * w[1] + T[4 * r3 + 2] * w[2] + T[4 * r3 + 3];
    all_near &= m[2] < near_z;
    all_l &= m[0] < l * m[2];
    all_r &= m[0] > r * m[2];
    all_t &= m[1] < t * m[2];
    all_b &= m[1] > b * m[2];
  }
  return !(all_near || all_l || all_r || all_t || all_b);
}

hgsr_status check_plan_args(int32_t n_parts, const float* poses, int32_t P, const hgsr_intrinsics* K, float near_z,
                            float motion_margin) {
  if (n_parts < 0) return fail(HGSR_ERR_INVALID_ARG, "n_parts < 0");
  if (P < 1 || !poses) return fail(HGSR_ERR_INVALID_ARG, "need P >= 1 host poses");
  if (!K || !(K->fx > 0.f) || !(K->fy > 0.f) || K->width <= 0 || K->height <= 0)
    return fail(HGSR_ERR_INVALID_ARG, "bad intrinsics");
  if (!(near_z >= 0.f) || !(motion_margin >= 0.f) || !std::isfinite(motion_margin))
    return fail(HGSR_ERR_INVALID_ARG, "near_z and motion_margin must be finite and non-negative");
  for (int64_t k = 0; k < 12ll * P; ++k)
    if (!std::isfinite(poses[k])) return fail(HGSR_ERR_INVALID_ARG, "non-finite pose entry");
  return HGSR_OK;
}

SlotPolicy::SlotPolicy(int32_t parts, int32_t slots)
    : n_parts(parts), n_slots(slots), slot_part(slots, -1), part_slot(parts, -1), slot_last(slots, -1) {}

hgsr_status SlotPolicy::step(const uint8_t* need, hgsr_pcache_stats* st) {
  int n_need = 0;
  for (int k = 0; k < n_parts; ++k) n_need += need[k] == 1;
  if (n_need > n_slots)
    return fail(HGSR_ERR_CAPACITY, "the rendered views may see %d partitions but the cache has %d slots", n_need,
                n_slots);
  st->needed = n_need;
  st->hits = st->uploads = st->evictions = st->prefetched = 0;
  std::vector<uint8_t> taken(n_slots, 0);
  for (int k = 0; k < n_parts; ++k)
    if (need[k] == 1 && part_slot[k] >= 0) {
      taken[part_slot[k]] = 1;
      slot_last[part_slot[k]] = batch;
      ++st->hits;
    }
  // an empty slot (least recently used first), else the least recently
  // used slot not taken; ties to the lower slot
  auto victim = [&]() {
    int v = -1;
    for (int sl = 0; sl < n_slots; ++sl)
      if (!taken[sl] && slot_part[sl] < 0 && (v < 0 || slot_last[sl] < slot_last[v])) v = sl;
    if (v < 0)
      for (int sl = 0; sl < n_slots; ++sl)
        if (!taken[sl] && (v < 0 || slot_last[sl] < slot_last[v])) v = sl;
    return v;
  };
  auto claim = [&](int k, int v, int ahead) {
    // the release point comes from the slot's previous use, read before the
    // slot is marked as used by this batch
    const int64_t prev = slot_last[v];
    const int64_t rel = prev < 0 ? -1 : std::max<int64_t>(prev + 1, batch - (kRing - 1));
    if (slot_part[v] >= 0) {
      part_slot[slot_part[v]] = -1;
      ++st->evictions;
    }
    slot_part[v] = k;
    part_slot[k] = v;
    slot_last[v] = batch;
    taken[v] = 1;
    hgsr_slot_upload& u = st->upload[st->uploads++];
    u.part = k;
    u.slot = v;
    u.release = rel;
    u.ahead = ahead;
    u.reserved = 0;
  };
  // 1. the rendered views' misses
  for (int k = 0; k < n_parts; ++k) {
    if (need[k] != 1 || part_slot[k] >= 0) continue;
    const int v = victim();
    if (v < 0) return fail(HGSR_ERR_STATE, "no free slot (internal)");
    claim(k, v, 0);
  }
  // 2. upcoming views: resident ones stay warm, missing ones take what is left
  for (int k = 0; k < n_parts; ++k)
    if (need[k] == 2 && part_slot[k] >= 0) {
      taken[part_slot[k]] = 1;
      slot_last[part_slot[k]] = batch;
    }
  for (int k = 0; k < n_parts; ++k) {
    if (need[k] != 2 || part_slot[k] >= 0) continue;
    const int v = victim();
    if (v < 0) continue;
    claim(k, v, 1);
    ++st->prefetched;
  }
  ++batch;
  return HGSR_OK;
}

void SlotPolicy::evict_all() {
  for (int sl = 0; sl < n_slots; ++sl) {
    if (slot_part[sl] >= 0) part_slot[slot_part[sl]] = -1;
    slot_part[sl] = -1;
  }
}

// 21 bits of v spread to every third bit.
uint64_t spread3(uint64_t v) {
  v &= 0x1fffffull;
  v = (v | (v << 32)) & 0x1f00000000ffffull;
  v = (v | (v << 16)) & 0x1f0000ff0000ffull;
  v = (v | (v << 8)) & 0x100f00f00f00f00full;
  v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
  v = (v | (v << 2)) & 0x1249249249249249ull;
  return v;
}

// Morton order of means[b, e) within the range's bounding cube.
void order_range(const float* means, int64_t b, int64_t e, int64_t* perm) {
  if (e <= b) return;
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = b; i < e; ++i)
    for (int a = 0; a < 3; ++a) {
      const double v = means[3 * i + a];
      if (std::isfinite(v)) {
        lo[a] = std::min(lo[a], v);
        hi[a] = std::max(hi[a], v);
      }
    }
  // one scale for all axes (cells stay cubes)
  double ext = 0.0;
  for (int a = 0; a < 3; ++a) ext = std::max(ext, hi[a] - lo[a]);
  const double sc = ext > 0.0 ? 2097151.0 / ext : 0.0;
  std::vector<std::pair<uint64_t, int64_t>> key(static_cast<size_t>(e - b));
  for (int64_t i = b; i < e; ++i) {
    uint64_t c = 0;
    for (int a = 0; a < 3; ++a) {
      double q = (static_cast<double>(means[3 * i + a]) - lo[a]) * sc;
      q = std::isfinite(q) ? std::min(std::max(q, 0.0), 2097151.0) : 0.0;
      c |= spread3(static_cast<uint64_t>(q)) << a;
    }
    key[i - b] = {c, i};
  }
  std::sort(key.begin(), key.end());  // ties: lower index first
  for (int64_t k = 0; k < e - b; ++k) perm[b + k] = key[k].second;
}

}  // namespace host
}  // namespace hgsr

using namespace hgsr::host;

struct hgsr_slot_policy {
  SlotPolicy pol;
  hgsr_slot_policy(int32_t parts, int32_t slots) : pol(parts, slots) {}
};

extern "C" {

hgsr_status hgsr_host_partition_bounds(const hgsr_host_scene* scene, float* bounds) {
  hgsr_status s = check_host_scene(scene);
  if (s != HGSR_OK) return s;
  if (!bounds) return fail(HGSR_ERR_INVALID_ARG, "NULL output");
  partition_bounds(scene, bounds);
  return HGSR_OK;
}

hgsr_status hgsr_partition_plan(const float* bounds, int32_t n_parts, const float* poses, int32_t P,
                                const hgsr_intrinsics* K, float near_z, float motion_margin, uint8_t* seen) {
  hgsr_status s = check_plan_args(n_parts, poses, P, K, near_z, motion_margin);
  if (s != HGSR_OK) return s;
  if (n_parts > 0 && (!bounds || !seen)) return fail(HGSR_ERR_INVALID_ARG, "NULL bounds or output");
  for (int p = 0; p < P; ++p)
    for (int k = 0; k < n_parts; ++k)
      seen[static_cast<int64_t>(p) * n_parts + k] =
          box_may_be_seen(bounds + 6 * k, poses + 12 * p, *K, near_z, motion_margin) ? 1 : 0;
  return HGSR_OK;
}

hgsr_status hgsr_host_spatial_order(const float* means, int64_t n, const int64_t* part_offsets, int32_t n_parts,
                                    int64_t* perm) {
  if (n < 0) return fail(HGSR_ERR_INVALID_ARG, "n < 0");
  if (n > 0 && (!means || !perm)) return fail(HGSR_ERR_INVALID_ARG, "NULL means or output");
  if (n_parts < 0 || (n_parts > 0 && !part_offsets))
    return fail(HGSR_ERR_INVALID_ARG, "partitions need part_offsets");
  if (n_parts > 0) {
    if (part_offsets[0] != 0 || part_offsets[n_parts] != n)
      return fail(HGSR_ERR_INVALID_ARG, "part_offsets must run from 0 to n");
    for (int k = 0; k < n_parts; ++k)
      if (part_offsets[k + 1] < part_offsets[k]) return fail(HGSR_ERR_INVALID_ARG, "part_offsets decrease");
    for (int k = 0; k < n_parts; ++k) order_range(means, part_offsets[k], part_offsets[k + 1], perm);
  } else {
    order_range(means, 0, n, perm);
  }
  return HGSR_OK;
}

hgsr_status hgsr_slot_policy_create(hgsr_slot_policy** out, int32_t n_parts, int32_t n_slots) {
  if (!out) return fail(HGSR_ERR_INVALID_ARG, "NULL output");
  *out = nullptr;
  if (n_parts < 1 || n_slots < 1 || n_slots > kMaxSlots || n_slots > n_parts)
    return fail(HGSR_ERR_INVALID_ARG, "need n_parts >= 1 and 1 <= n_slots <= min(64, n_parts)");
  *out = new hgsr_slot_policy(n_parts, n_slots);
  return HGSR_OK;
}

hgsr_status hgsr_slot_policy_destroy(hgsr_slot_policy* p) {
  delete p;
  return HGSR_OK;
}

hgsr_status hgsr_slot_policy_step(hgsr_slot_policy* p, const uint8_t* need, hgsr_pcache_stats* st) {
  if (!p || !need || !st) return fail(HGSR_ERR_INVALID_ARG, "NULL argument");
  for (int k = 0; k < p->pol.n_parts; ++k)
    if (need[k] > 2) return fail(HGSR_ERR_INVALID_ARG, "need entries must be 0, 1 or 2");
  return p->pol.step(need, st);
}

hgsr_status hgsr_slot_policy_evict_all(hgsr_slot_policy* p) {
  if (!p) return fail(HGSR_ERR_INVALID_ARG, "NULL policy");
  p->pol.evict_all();
  return HGSR_OK;
}

}  // extern "C"
