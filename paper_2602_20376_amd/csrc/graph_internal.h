// Graph argument checks shared by the graph and spectral modules.  Internal
// header.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lrqo.h"

namespace lrqo {

// Host checks of the descriptor: pointers, n, nnz, device memory.
lrqo_status check_graph_args(const lrqo_graph* g);

// Device checks of the CSR layout (row pointer first: the second pass reads
// col through it) and, when z is not null, of the labels (< K).  d_flag is
// device scratch and h_flag pinned host memory of one int each.
lrqo_status validate_graph(const lrqo_graph* g, int K, const uint8_t* z, int* d_flag, int* h_flag,
                           hipStream_t st);

}  // namespace lrqo
