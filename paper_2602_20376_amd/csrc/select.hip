// Top-T selection: each block sorts one chunk of 2048 packed keys in LDS
// (bitonic, descending) and keeps its first T; passes repeat over the
// survivors until one block remains.
#include "lrqo_device.h"
#include "lrqo_runtime.h"
#include "select.h"

namespace lrqo {

namespace {

constexpr int kBlock = 256;
constexpr int kChunk = 2048;

// Keys come from f (index = position) or from a previous pass.  Padding keys
// are 0, below every real key (a real key's index is < 2^32-1, so its low
// word is nonzero).
__global__ __launch_bounds__(kBlock) void k_topk(const float* __restrict__ f,
                                                 const unsigned long long* __restrict__ keys_in,
                                                 uint32_t count, int T,
                                                 unsigned long long* __restrict__ keys_out) {
    __shared__ unsigned long long sk[kChunk];
    const uint32_t base = blockIdx.x * (uint32_t)kChunk;
    for (int e = threadIdx.x; e < kChunk; e += kBlock) {
        const uint32_t g = base + e;
        unsigned long long key = 0;
        if (g < count) key = f ? pack_key(f[g], g) : keys_in[g];
        sk[e] = key;
    }
    __syncthreads();
    for (int k = 2; k <= kChunk; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int e = threadIdx.x; e < kChunk; e += kBlock) {
                const int x = e ^ j;
                if (x > e) {
                    const unsigned long long a = sk[e], b = sk[x];
                    const bool desc = (e & k) == 0;
                    if (desc ? (a < b) : (a > b)) {
                        sk[e] = b;
                        sk[x] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int e = threadIdx.x; e < T; e += kBlock) keys_out[(size_t)blockIdx.x * T + e] = sk[e];
}

}  // namespace

size_t topk_buffer_keys(uint32_t count, int T) {
    return ((size_t)count + kChunk - 1) / kChunk * (size_t)T;
}

lrqo_status topk_select(const float* f, uint32_t count, int T, unsigned long long* buf_a,
                        unsigned long long* buf_b, hipStream_t st,
                        const unsigned long long** out) {
    const unsigned long long* keys = nullptr;
    uint32_t n = count;
    int ping = 0;
    bool from_f = true;
    for (;;) {
        const uint32_t blocks = (n + kChunk - 1) / kChunk;
        unsigned long long* dst = ping ? buf_b : buf_a;
        hipLaunchKernelGGL(k_topk, dim3(blocks), dim3(kBlock), 0, st, from_f ? f : nullptr, keys, n,
                           T, dst);
        LRQO_HIP(hipGetLastError());
        keys = dst;
        n = blocks * (uint32_t)T;
        ping ^= 1;
        from_f = false;
        if (blocks == 1) break;
    }
    *out = keys;
    return LRQO_OK;
}

}  // namespace lrqo
