// Top-T selection of packed (objective, index) keys.  Internal header.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lrqo.h"

namespace lrqo {

// Keys needed in each of the two ping-pong buffers of topk_select.
size_t topk_buffer_keys(uint32_t count, int T);

// Best T keys of f[0..count) (key = FP32 bits of f above, complemented index
// below: larger f first, lower index first among equal f), sorted
// descending, at *out (one of buf_a / buf_b).  Requires 1 <= T <= 64 and
// T <= count; f must be finite and >= 0.  distinct: one key per value of f
// (its lowest index); then fewer than T values leave padding keys 0 at the end.
// floor_f (device pointer, may be null; read when the selection runs): values
// of f strictly below *floor_f are left out when *floor_f >= 0 (their places
// become padding keys 0 at the end).
lrqo_status topk_select(const float* f, uint32_t count, int T, unsigned long long* buf_a,
                        unsigned long long* buf_b, hipStream_t st,
                        const unsigned long long** out, bool distinct = false,
                        const float* floor_f = nullptr);

// The same from keys already sorted in lists of 64 (lists[64 q + l] the
// l-th largest of list q, padding keys 0); count a multiple of 64.
lrqo_status topk_select_lists(const unsigned long long* lists, uint32_t count, int T,
                              unsigned long long* buf_a, unsigned long long* buf_b, hipStream_t st,
                              const unsigned long long** out);

}  // namespace lrqo
