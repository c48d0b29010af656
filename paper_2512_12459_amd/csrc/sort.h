// Device-wide stable key-value radix sort used by the builds that run every
// step (cull grid, centre grid, photon map) and by the query binning.
#pragma once
#include <rocprim/device/device_radix_sort.hpp>

namespace gpf {

// rocPRIM's default configuration sorts fewer than 2^20 items with a block
// merge sort: about twenty short launches, most of them launch-bound at the
// sizes here (around a million cell entries).  A merge-sort limit of zero
// selects the onesweep path at every size above one block instead: a
// histogram pass, its scan and one pass per 8 key bits.  Both are stable.
using OnesweepSortConfig = rocprim::radix_sort_config<rocprim::default_config,
                                                      rocprim::default_config,
                                                      rocprim::default_config, 0>;

template <class K, class V>
hipError_t sort_pairs(void* tmp, size_t& bytes, K* keys_in, K* keys_out, V* vals_in, V* vals_out,
                      size_t n, int begin_bit, int end_bit, hipStream_t s) {
  return rocprim::radix_sort_pairs<OnesweepSortConfig>(tmp, bytes, keys_in, keys_out, vals_in,
                                                       vals_out, n, (unsigned)begin_bit,
                                                       (unsigned)end_bit, s);
}

}  // namespace gpf
