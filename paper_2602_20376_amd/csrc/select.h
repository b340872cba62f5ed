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

// A floor for a distinct top-T selection of f[0..count) that drops nothing
// the selection keeps: the T-th largest distinct value among the maxima of
// the groups of scores (2,048 each) that the selection's first pass takes,
// since at least T distinct scores reach it; -1 when the maxima hold fewer
// than T distinct values.  *floor_out (device) receives the larger of it and
// *floor_in (device, may be null).  Needs count >= 2,048 T; uses buf_a and
// buf_b as topk_select does.
lrqo_status topk_block_floor(const float* f, uint32_t count, int T, const float* floor_in, float* floor_out,
                             unsigned long long* buf_a, unsigned long long* buf_b, hipStream_t st);

// The same from keys already sorted in lists of 64 (lists[64 q + l] the
// l-th largest of list q, padding keys 0); count a multiple of 64.
lrqo_status topk_select_lists(const unsigned long long* lists, uint32_t count, int T,
                              unsigned long long* buf_a, unsigned long long* buf_b, hipStream_t st,
                              const unsigned long long** out);

}  // namespace lrqo
