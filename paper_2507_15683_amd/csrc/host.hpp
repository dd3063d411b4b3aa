// Host-only parts of the library (no device code, no HIP headers): the
// partition boxes and per-pose plan of a partitioned scene, the slot policy
// of the partition cache, and the spatial order of a scene.  Plain C++, so
// that the same source also builds under the host sanitizers.
#pragma once

#include <stdint.h>

#include <vector>

#include "../../include/hgsr.h"

namespace hgsr {

// Sets the thread's hgsr_last_error() text; returns st.
hgsr_status report_error(hgsr_status st, const char* msg);

namespace host {

constexpr int kMaxSlots = HGSR_MAX_SLOTS;  // the renderer's per-pose partition mask
constexpr double kSupport = 3.33;          // box radius per largest scale

hgsr_status fail(hgsr_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));

bool empty_box(const float* B);
hgsr_status check_host_scene(const hgsr_host_scene* s);
// Per partition the box around every Gaussian's ball of radius 3.33 x its
// largest scale, rounded outward to float; an empty partition gets min > max.
void partition_bounds(const hgsr_host_scene* s, float* out);
hgsr_status check_plan_args(int32_t n_parts, const float* poses, int32_t P, const hgsr_intrinsics* K, float near_z,
                            float motion_margin);
// The renderer's partition test in double, with one more pixel of margin and
// the box grown by `grow` metres.
bool box_may_be_seen(const float* B, const float* T, const hgsr_intrinsics& K, double near_z, double grow);

// Which partition each device slot holds, batch by batch.  A batch names,
// per partition, whether its rendered views may see it (1), only its
// upcoming views may (2) or neither (0).  Rendered views' partitions that
// are missing take an empty slot, else the least recently used slot the
// batch does not need; upcoming views' partitions then take what is left
// (best effort).  Each upload records the release batch its copy must wait
// for: the first batch after the slot's previous last use (work enqueued
// before that batch's start may still read the slot), clamped to the oldest
// batch a ring of kRing start events still holds; -1 for a slot never used.
struct SlotPolicy {
  static constexpr int kRing = 16;
  int32_t n_parts = 0, n_slots = 0;
  int64_t batch = 0;                 // index of the next batch
  std::vector<int32_t> slot_part;    // resident partition, -1 for none
  std::vector<int32_t> part_slot;    // slot of a resident partition, -1 otherwise
  std::vector<int64_t> slot_last;    // last batch that needed the slot, -1 for none

  SlotPolicy(int32_t parts, int32_t slots);
  // One batch.  Fills needed, hits, uploads, evictions, prefetched and the
  // upload list of *st (the byte counts are the caller's).  Returns
  // HGSR_ERR_CAPACITY, with the state unchanged, when the rendered views need
  // more partitions than there are slots.
  hgsr_status step(const uint8_t* need, hgsr_pcache_stats* st);
  // Forget every resident partition; last uses stay recorded.
  void evict_all();
};

}  // namespace host
}  // namespace hgsr
