// Stable device sort of (uint64 key, uint32 value) pairs.  Internal header.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lrqo.h"

namespace lrqo {

// Entries of the digit-count scratch radix_sort_pairs needs for n keys.
size_t radix_hist_entries(int64_t n);

// Ascending, stable (equal keys keep their input order) LSD radix sort with
// 8-bit digits.  Pass d (bits 8d .. 8d+7) runs only when bit d of
// digit_mask is set: a digit that is the same in every key leaves the order
// unchanged.  Input in (keys, vals); the sorted pairs end in (keys, vals)
// or in (keys_tmp, vals_tmp), as *in_tmp reports.  hist holds
// radix_hist_entries(n) counters.  1 <= n <= 2^31 - 1.
lrqo_status radix_sort_pairs(unsigned long long* keys, uint32_t* vals, unsigned long long* keys_tmp,
                             uint32_t* vals_tmp, uint32_t* hist, int64_t n, unsigned digit_mask,
                             hipStream_t st, bool* in_tmp);

}  // namespace lrqo
