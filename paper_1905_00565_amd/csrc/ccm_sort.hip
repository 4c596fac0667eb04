// ccm_sort.hip -- visiting orders of the series' time points (stable
// segmented radix sort of 32-bit keys).
//
// The orders are used only to decide in which order the cross-map kernel
// visits queries and library candidates (nearest first, so the running
// top-(E+1) lists settle early).  Results do not depend on it: neighbours are selected
// by the exact (d2, index) key whatever the visiting order.
#include <hipcub/hipcub.hpp>

#include "ccm_internal.h"

namespace ccmk {

hipError_t sort_series(void* temp, size_t& temp_bytes, const uint32_t* keys_in,
                       uint32_t* keys_out, const int32_t* idx_in, int32_t* idx_out,
                       int64_t n_series, int32_t segs, const int32_t* seg_offsets,
                       hipStream_t st) {
  const int n = (int)(n_series * segs);
  return hipcub::DeviceSegmentedRadixSort::SortPairs(
      temp, temp_bytes, keys_in, keys_out, idx_in, idx_out, n, segs, seg_offsets,
      seg_offsets + 1, 0, (int)(sizeof(uint32_t) * 8), st);
}

}  // namespace ccmk
