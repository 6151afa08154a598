// Internal declarations shared by the library's host sources.
#pragma once

#include <cstdint>
#include <mutex>
#include <vector>

#include "../../include/median_filter.h"

struct mf_footprint {
  // kind: 0 = disc given by an integer squared limit; 1 = general convex
  // shape given only by its spans.  Both carry the spans.
  int kind = 1;
  long long limit = 0;
  int dx_min = 0, dx_max = 0, dy_min = 0, dy_max = 0;
  int taps = 0;
  std::vector<int> row_lo, row_hi;  // index dy - dy_min: dx range of that row
  std::vector<int> col_lo, col_hi;  // index dx - dx_min: dy range of that column

  // Per-device copies of the span tables (int16 pairs: rows then columns).
  struct DevCopy {
    int device;
    void* ptr;
  };
  mutable std::mutex mu;
  mutable std::vector<DevCopy> dev;
};

namespace mf {

// Upload (once per device) and return the device span table of `fp`:
// [row (lo,hi) pairs as int16][column (lo,hi) pairs as int16].
int footprint_device_table(const mf_footprint* fp, int device, const void** table);

inline int elem_size(int dtype) { return dtype == MF_U8 ? 1 : dtype == MF_U16 ? 2 : 4; }

}  // namespace mf
