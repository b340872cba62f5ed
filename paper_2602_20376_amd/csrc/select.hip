// Top-T selection of packed keys with one 64-key list per wavefront: lane l
// holds the l-th largest key seen so far.  Each wave streams 64-key tiles,
// sorts a tile across its lanes (bitonic network over lane shuffles) and
// merges it into the running list (half-cleaner against the reversed tile,
// then a bitonic merge); tiles with no key above the running 64th are
// skipped; input already sorted in lists of 64 (the slice sum's per-wave
// lists, or a previous pass's block lists when T = 64) is merged without the
// sort.  The four lists of a block are merged the same way, the block writes
// its best T, and passes repeat over the survivors until one block remains.
#include "lrqo_device.h"
#include "lrqo_runtime.h"
#include "select.h"

namespace lrqo {

namespace {

constexpr int kWaves = 4;
constexpr int kBlock = 64 * kWaves;
constexpr int kChunk = 2048;  // keys per block, kChunk / kWaves per wave

// Keys come from f (index = position) or from a previous pass.  Padding keys
// are 0, below every real key (a real key's index is < 2^32-1, so its low
// word is nonzero).
// distinct = 1: one key per objective value (the lowest index), for inputs
// where many candidates share a bit-identical score.
// floor_f (may be null; read on the device): scores strictly below *floor_f
// are dropped (their keys count as padding) when *floor_f >= 0.
__global__ __launch_bounds__(kBlock) void k_topk(const float* __restrict__ f,
                                                 const unsigned long long* __restrict__ keys_in,
                                                 uint32_t count, int T, int sorted, int distinct,
                                                 const float* __restrict__ floor_f,
                                                 unsigned long long* __restrict__ keys_out) {
    __shared__ unsigned long long top[kWaves][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t base = blockIdx.x * (uint32_t)kChunk + (uint32_t)w * (kChunk / kWaves);
    // non-negative floats order as their bits; a key with score x is at
    // least bits(x) << 32
    unsigned long long lo = 0;
    if (floor_f) {
        const float fl = *floor_f;
        if (fl >= 0.0f) lo = (unsigned long long)__float_as_uint(fl) << 32;
    }
    unsigned long long run = 0;
    for (int t = 0; t < kChunk / kWaves; t += 64) {
        const uint32_t g = base + (uint32_t)(t + lane);
        unsigned long long key = 0;
        if (g < count) key = f ? pack_key(f[g], g) : keys_in[g];
        key = key < lo ? 0ull : key;
        const unsigned long long floor64 = __shfl(run, 63, 64);
        if (__ballot(key > floor64) == 0) continue;  // uniform across the wave
        const unsigned long long tile = sorted ? key : wave_sort_desc(key, lane);
        run = distinct ? wave_top_union_distinct(run, tile, lane) : wave_top_union(run, tile, lane);
    }
    top[w][lane] = run;
    __syncthreads();
    if (w != 0) return;
    for (int v = 1; v < kWaves; ++v)
        run = distinct ? wave_top_union_distinct(run, top[v][lane], lane) : wave_top_union(run, top[v][lane], lane);
    if (lane < T) keys_out[(size_t)blockIdx.x * T + lane] = run;
}

// Per group of kChunk scores (k_topk's grouping): the key of its largest
// score.
__global__ __launch_bounds__(kBlock) void k_block_max(const float* __restrict__ f, uint32_t count,
                                                      unsigned long long* __restrict__ out) {
    __shared__ unsigned long long wm[kWaves];
    const uint32_t base = blockIdx.x * (uint32_t)kChunk;
    unsigned long long m = 0;
    for (int e = threadIdx.x; e < kChunk; e += kBlock) {
        const uint32_t g = base + (uint32_t)e;
        if (g < count) m = key_max(m, pack_key(f[g], g));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = key_max(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kWaves; ++w) m = key_max(m, wm[w]);
        out[blockIdx.x] = m;
    }
}

// *floor_out = the larger of *floor_in (when given) and the value of the
// T-th key of a distinct top-T list (-1 when the list holds fewer than T).
__global__ void k_floor_from(const unsigned long long* __restrict__ top, int T, const float* __restrict__ floor_in,
                             float* __restrict__ floor_out) {
    if (threadIdx.x != 0) return;
    float v = top[T - 1] != 0ull ? key_value(top[T - 1]) : -1.0f;
    if (floor_in) v = fmaxf(v, *floor_in);
    *floor_out = v;
}

}  // namespace

size_t topk_buffer_keys(uint32_t count, int T) {
    return ((size_t)count + kChunk - 1) / kChunk * (size_t)T;
}

namespace {

lrqo_status topk_passes(const float* f, const unsigned long long* keys, bool sorted, uint32_t count, int T,
                        bool distinct, const float* floor_f, unsigned long long* buf_a, unsigned long long* buf_b,
                        hipStream_t st, const unsigned long long** out) {
    uint32_t n = count;
    int ping = 0;
    bool from_f = f != nullptr;
    for (;;) {
        const uint32_t blocks = (n + kChunk - 1) / kChunk;
        unsigned long long* dst = ping ? buf_b : buf_a;
        hipLaunchKernelGGL(k_topk, dim3(blocks), dim3(kBlock), 0, st, from_f ? f : nullptr, keys, n,
                           T, sorted ? 1 : 0, distinct ? 1 : 0, from_f ? floor_f : nullptr, dst);
        LRQO_HIP(hipGetLastError());
        keys = dst;
        n = blocks * (uint32_t)T;
        ping ^= 1;
        from_f = false;
        sorted = T == 64;       // a block writes its list sorted, 64 apart
        if (blocks == 1) break;
    }
    *out = keys;
    return LRQO_OK;
}

}  // namespace

lrqo_status topk_select(const float* f, uint32_t count, int T, unsigned long long* buf_a,
                        unsigned long long* buf_b, hipStream_t st,
                        const unsigned long long** out, bool distinct, const float* floor_f) {
    return topk_passes(f, nullptr, false, count, T, distinct, floor_f, buf_a, buf_b, st, out);
}

lrqo_status topk_select_lists(const unsigned long long* lists, uint32_t count, int T,
                              unsigned long long* buf_a, unsigned long long* buf_b, hipStream_t st,
                              const unsigned long long** out) {
    return topk_passes(nullptr, lists, true, count, T, false, nullptr, buf_a, buf_b, st, out);
}

lrqo_status topk_block_floor(const float* f, uint32_t count, int T, const float* floor_in, float* floor_out,
                             unsigned long long* buf_a, unsigned long long* buf_b, hipStream_t st) {
    const uint32_t groups = (count + kChunk - 1) / kChunk;
    if (T < 1 || T > 64 || groups < (uint32_t)T) return LRQO_EINVAL;
    hipLaunchKernelGGL(k_block_max, dim3(groups), dim3(kBlock), 0, st, f, count, buf_b);
    LRQO_HIP(hipGetLastError());
    const unsigned long long* top = nullptr;
    LRQO_TRY(topk_passes(nullptr, buf_b, false, groups, T, true, nullptr, buf_a, buf_b, st, &top));
    hipLaunchKernelGGL(k_floor_from, dim3(1), dim3(64), 0, st, top, T, floor_in, floor_out);
    LRQO_HIP(hipGetLastError());
    return LRQO_OK;
}

}  // namespace lrqo
