// Drives the library's host-only code (host.cpp: partition boxes and plan,
// the partition cache's slot policy, the spatial order) under the host
// sanitizers.  Exit status 0 when every call behaves; a sanitizer report
// aborts the process.
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "../../include/hgsr.h"

namespace hgsr {
hgsr_status report_error(hgsr_status st, const char*) { return st; }
}  // namespace hgsr

#define CHECK(c)                                               \
  do {                                                         \
    if (!(c)) {                                                \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      return 1;                                                \
    }                                                          \
  } while (0)

int main() {
  std::mt19937_64 rng(7);
  std::normal_distribution<float> nd(0.f, 1.f);
  std::uniform_real_distribution<float> ud(-400.f, 400.f);
  // a scene of 5,000 Gaussians in 9 partitions, one of them empty, one NaN mean
  const int64_t n = 5000;
  const int parts = 9;
  std::vector<float> means(3 * n), ls(3 * n), quats(4 * n), opac(n), sh(3 * n);
  for (int64_t i = 0; i < n; ++i) {
    means[3 * i] = ud(rng);
    means[3 * i + 1] = ud(rng);
    means[3 * i + 2] = 2.f * nd(rng);
    for (int a = 0; a < 3; ++a) ls[3 * i + a] = -0.5f + 0.3f * nd(rng);
    for (int a = 0; a < 4; ++a) quats[4 * i + a] = nd(rng);
    opac[i] = 0.5f;
    for (int a = 0; a < 3; ++a) sh[3 * i + a] = nd(rng);
  }
  means[3 * 17] = NAN;
  std::vector<int64_t> offs(parts + 1);
  for (int k = 0; k <= parts; ++k) offs[k] = n * k / parts;
  offs[4] = offs[3];  // partition 3 is empty
  hgsr_host_scene hs{n, means.data(), ls.data(), quats.data(), opac.data(), sh.data(), 0, 0, nullptr, parts,
                     offs.data()};
  std::vector<float> bounds(6 * parts);
  CHECK(hgsr_host_partition_bounds(&hs, bounds.data()) == HGSR_OK);
  CHECK(bounds[6 * 3] > bounds[6 * 3 + 3]);  // the empty partition's box is empty
  CHECK(hgsr_host_partition_bounds(nullptr, bounds.data()) == HGSR_ERR_INVALID_ARG);
  // plan for 40 poses looking down from 100-300 m
  const int P = 40;
  std::vector<float> poses(12 * P);
  for (int p = 0; p < P; ++p) {
    float* T = poses.data() + 12 * p;
    const float cx = ud(rng), cy = ud(rng), h = 100.f + 200.f * std::abs(nd(rng));
    // R = diag(1, -1, -1) (looking down), t = -R C
    const float R[9] = {1, 0, 0, 0, -1, 0, 0, 0, -1};
    const float C[3] = {cx, cy, h};
    for (int r = 0; r < 3; ++r) {
      for (int c = 0; c < 3; ++c) T[4 * r + c] = R[3 * r + c];
      T[4 * r + 3] = -(R[3 * r] * C[0] + R[3 * r + 1] * C[1] + R[3 * r + 2] * C[2]);
    }
  }
  hgsr_intrinsics K{500.f, 500.f, 320.f, 240.f, 640, 480};
  std::vector<uint8_t> seen(static_cast<size_t>(P) * parts);
  CHECK(hgsr_partition_plan(bounds.data(), parts, poses.data(), P, &K, 0.2f, 5.f, seen.data()) == HGSR_OK);
  for (int p = 0; p < P; ++p) CHECK(seen[p * parts + 3] == 0);
  poses[5] = INFINITY;
  CHECK(hgsr_partition_plan(bounds.data(), parts, poses.data(), P, &K, 0.2f, 5.f, seen.data()) ==
        HGSR_ERR_INVALID_ARG);
  // spatial order: a permutation of each partition's range
  std::vector<int64_t> perm(n, -1);
  CHECK(hgsr_host_spatial_order(means.data(), n, offs.data(), parts, perm.data()) == HGSR_OK);
  std::vector<int> hit(n, 0);
  for (int k = 0; k < parts; ++k)
    for (int64_t i = offs[k]; i < offs[k + 1]; ++i) {
      CHECK(perm[i] >= offs[k] && perm[i] < offs[k + 1]);
      hit[perm[i]]++;
    }
  for (int64_t i = 0; i < n; ++i) CHECK(hit[i] == 1);
  CHECK(hgsr_host_spatial_order(means.data(), 0, nullptr, 0, nullptr) == HGSR_OK);
  // slot policy: random batches including capacity errors and evictions
  for (int slots : {1, 3, 9}) {
    hgsr_slot_policy* pol = nullptr;
    CHECK(hgsr_slot_policy_create(&pol, parts, slots) == HGSR_OK);
    std::uniform_int_distribution<int> need_d(0, 5);
    hgsr_pcache_stats st{};
    for (int it = 0; it < 2000; ++it) {
      std::vector<uint8_t> need(parts);
      for (auto& v : need) v = static_cast<uint8_t>(std::min(need_d(rng), 2) * (need_d(rng) < 2));
      const hgsr_status s = hgsr_slot_policy_step(pol, need.data(), &st);
      CHECK(s == HGSR_OK || s == HGSR_ERR_CAPACITY);
      if (s == HGSR_OK) CHECK(st.uploads <= slots);
      if (it % 500 == 499) CHECK(hgsr_slot_policy_evict_all(pol) == HGSR_OK);
    }
    CHECK(hgsr_slot_policy_destroy(pol) == HGSR_OK);
  }
  hgsr_slot_policy* bad = nullptr;
  CHECK(hgsr_slot_policy_create(&bad, 4, 5) == HGSR_ERR_INVALID_ARG && bad == nullptr);
  std::puts("host driver ok");
  return 0;
}
