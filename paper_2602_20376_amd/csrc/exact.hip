// Exact maximisation (Sec. 3, Alg. 2): placeholder until the vertex
// enumeration kernels land.
#include "lrqo_runtime.h"

extern "C" {

lrqo_status lrqo_solve_exact_ex(const double* V, int64_t n, int32_t r, int32_t K,
                                int64_t max_sets, uint8_t* z, lrqo_exact_result* res) {
    (void)V; (void)n; (void)r; (void)K; (void)max_sets; (void)z; (void)res;
    return lrqo::fail(LRQO_EINVAL, "exact solver not built yet");
}

lrqo_status lrqo_solve_exact(const double* V, int64_t n, int32_t r, int32_t K, uint8_t* z,
                             double* obj) {
    (void)obj;
    return lrqo_solve_exact_ex(V, n, r, K, 0, z, nullptr);
}

}  // extern "C"
