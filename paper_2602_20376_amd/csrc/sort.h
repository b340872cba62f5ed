// Stable device sort of (uint64 key, uint32 value) pairs.  Internal header.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lrqo.h"

namespace lrqo {

// Entries of the digit-count scratch radix_sort_pairs needs for n keys.
size_t radix_hist_entries(int64_t n);

// Where the sorted pairs ended up (one of the two work buffers).
struct SortedPairs {
    const unsigned long long* keys;
    const uint32_t* vals;
};
struct SortedPairs32 {
    const uint32_t* keys;
    const uint32_t* vals;
};

// Ascending, stable (equal keys keep their input order) LSD radix sort with
// 8-bit digits of the n keys in `keys`, which stay as they are; the value
// paired with each key is its position 0 .. n-1.  Pass d (bits 8d .. 8d+7)
// runs only when bit d of digit_mask is set: a digit that is the same in
// every key leaves the order unchanged.  The passes alternate between the
// work buffers (keys_a, vals_a) and (keys_b, vals_b); *out names the one
// holding the result.  hist holds radix_hist_entries(n) counters.
// 1 <= n <= 2^31 - 1.
lrqo_status radix_sort_pairs(const unsigned long long* keys, unsigned long long* keys_a, uint32_t* vals_a,
                             unsigned long long* keys_b, uint32_t* vals_b, uint32_t* hist, int64_t n,
                             unsigned digit_mask, hipStream_t st, SortedPairs* out);

// The same for 32-bit keys (four digits; bits 0-3 of digit_mask).
lrqo_status radix_sort_pairs32(const uint32_t* keys, uint32_t* keys_a, uint32_t* vals_a, uint32_t* keys_b,
                               uint32_t* vals_b, uint32_t* hist, int64_t n, unsigned digit_mask, hipStream_t st,
                               SortedPairs32* out);

}  // namespace lrqo
