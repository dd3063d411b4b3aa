// Scene layout: a spatial (Morton) order of the Gaussians, computed on the
// host once per scene.  Neighbouring Gaussians then share workgroups, so a
// view's visible Gaussians fill whole waves of the projection, a workgroup's
// records fall in a few tiles (their tile counts aggregate in LDS) and a
// tile's records sit close together in memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "../../include/hgsr.h"
#include "launch.hpp"

namespace {

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

}  // namespace

extern "C" hgsr_status hgsr_host_spatial_order(const float* means, int64_t n, const int64_t* part_offsets,
                                               int32_t n_parts, int64_t* perm) {
  if (n < 0) return hgsr::report_error(HGSR_ERR_INVALID_ARG, "n < 0");
  if (n > 0 && (!means || !perm)) return hgsr::report_error(HGSR_ERR_INVALID_ARG, "NULL means or output");
  if (n_parts < 0 || (n_parts > 0 && !part_offsets))
    return hgsr::report_error(HGSR_ERR_INVALID_ARG, "partitions need part_offsets");
  if (n_parts > 0) {
    if (part_offsets[0] != 0 || part_offsets[n_parts] != n)
      return hgsr::report_error(HGSR_ERR_INVALID_ARG, "part_offsets must run from 0 to n");
    for (int k = 0; k < n_parts; ++k)
      if (part_offsets[k + 1] < part_offsets[k])
        return hgsr::report_error(HGSR_ERR_INVALID_ARG, "part_offsets decrease");
    for (int k = 0; k < n_parts; ++k) order_range(means, part_offsets[k], part_offsets[k + 1], perm);
  } else {
    order_range(means, 0, n, perm);
  }
  return HGSR_OK;
}
