// ccm_sort.hip -- order of each series' values (stable segmented radix sort).
//
// The order is used only to decide in which order the cross-map kernel visits
// queries and library candidates (nearest first, so the running top-(E+1)
// lists settle early).  Results do not depend on it: neighbours are selected
// by the exact (d2, index) key whatever the visiting order.
#include <hipcub/hipcub.hpp>

#include "ccm_internal.h"

namespace ccmk {

hipError_t sort_series(void* temp, size_t& temp_bytes, const float* keys_in,
                       float* keys_out, const int32_t* idx_in, int32_t* idx_out,
                       int64_t n_series, int32_t segs, const int32_t* seg_offsets,
                       hipStream_t st) {
  const int n = (int)(n_series * segs);
  return hipcub::DeviceSegmentedRadixSort::SortPairs(
      temp, temp_bytes, keys_in, keys_out, idx_in, idx_out, n, segs, seg_offsets,
      seg_offsets + 1, 0, (int)(sizeof(float) * 8), st);
}

}  // namespace ccmk
