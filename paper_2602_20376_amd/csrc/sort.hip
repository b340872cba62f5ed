// Stable LSD radix sort of (uint64 or uint32 key, uint32 value) pairs,
// 8-bit digits.
//
// Per pass (one 8-bit digit):
//   k_digit_hist     per tile of 2048 pairs: digit counts -> hist[digit][tile]
//   k_scan_rows      one wave per digit: exclusive prefix along the row, and
//                    the row's total
//   k_digit_scatter  per tile: the digits' first output slots (exclusive
//                    scan of the row totals, done by every block, plus the
//                    row prefix); four waves take consecutive quarters; each
//                    wave counts its digits, the waves' counts are offset
//                    in wave order, then every wave walks its quarter in
//                    64-pair steps: lanes holding the same digit are found
//                    with eight ballots, a lane's slot is the digit's running
//                    offset plus the number of such lanes below it, and the
//                    lowest of them advances the offset.  Slots therefore
//                    follow input order within a digit: the pass is stable.
//                    The pairs are first placed in a digit-ordered LDS copy
//                    of the tile and written out from it, so that each
//                    digit's run is written to consecutive addresses.
#include <algorithm>

#include "lrqo_device.h"
#include "lrqo_runtime.h"
#include "sort.h"

namespace lrqo {

namespace {

constexpr int kWaves = 4;
constexpr int kBlock = kWaves * kWave;   // 256
constexpr int kSteps = 8;                // 64-pair steps per wave
constexpr int kTile = kWaves * kSteps * kWave;  // 2048 pairs per block
constexpr int kBins = 256;
static_assert(kBlock == kBins, "one thread per digit bin");

template <typename Key>
__device__ __forceinline__ int digit_of(Key key, int shift) {
    return (int)((key >> shift) & 0xFFu);
}

template <typename Key>
__global__ __launch_bounds__(kBlock) void k_digit_hist(const Key* __restrict__ keys,
                                                       int64_t n, int shift, uint32_t* __restrict__ hist,
                                                       int64_t tiles) {
    __shared__ uint32_t h[kBins];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = blockIdx.x * (int64_t)kTile;
    for (int e = threadIdx.x; e < kTile; e += kBlock) {
        const int64_t idx = base + e;
        if (idx < n) atomicAdd(&h[digit_of(keys[idx], shift)], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * tiles + blockIdx.x] = h[threadIdx.x];
}

// Wave d turns row d of hist (one count per tile) into its exclusive prefix
// along the row and writes the row's total to rowtot[d]: chunks of 64 x 8
// entries, lane l holding 8 consecutive ones; prefix = carry + the wave's
// exclusive scan of the lanes' sums (shuffles) + the lane's running sum.
constexpr int kScanWaves = 4;

__global__ __launch_bounds__(kScanWaves * kWave) void k_scan_rows(uint32_t* __restrict__ hist, int64_t tiles,
                                                                  uint32_t* __restrict__ rowtot) {
    const int lane = threadIdx.x & (kWave - 1);
    const int d = blockIdx.x * kScanWaves + threadIdx.x / kWave;
    uint32_t* row = hist + (int64_t)d * tiles;
    uint32_t carry = 0u;
    for (int64_t c0 = 0; c0 < tiles; c0 += 8 * kWave) {
        uint32_t v[8], sum = 0u;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t idx = c0 + lane * 8 + u;
            v[u] = idx < tiles ? row[idx] : 0u;
            sum += v[u];
        }
        uint32_t incl = sum;
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const uint32_t y = __shfl_up(incl, off, kWave);
            if (lane >= off) incl += y;
        }
        uint32_t run = carry + incl - sum;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t idx = c0 + lane * 8 + u;
            if (idx < tiles) row[idx] = run;
            run += v[u];
        }
        carry += __shfl(incl, kWave - 1, kWave);
    }
    if (lane == 0) rowtot[d] = carry;
}

// Exclusive prefix over the block of one value per thread (256 threads):
// inclusive scan across each wave by shuffles, then the lower waves' sums.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t* wsum) {
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    uint32_t incl = x;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const uint32_t y = __shfl_up(incl, off, kWave);
        if (lane >= off) incl += y;
    }
    if (lane == kWave - 1) wsum[w] = incl;
    __syncthreads();
    uint32_t ex = incl - x;
    for (int v = 0; v < w; ++v) ex += wsum[v];
    __syncthreads();
    return ex;
}

template <typename Key>
__global__ __launch_bounds__(kBlock) void k_digit_scatter(const Key* __restrict__ keys_in,
                                                          const uint32_t* __restrict__ vals_in,
                                                          Key* __restrict__ keys_out,
                                                          uint32_t* __restrict__ vals_out, int64_t n,
                                                          int shift, const uint32_t* __restrict__ offs,
                                                          int64_t tiles, const uint32_t* __restrict__ rowtot) {
    __shared__ uint32_t cnt[kWaves][kBins];
    __shared__ uint32_t base[kWaves][kBins];
    __shared__ uint32_t wsum[kWaves];
    __shared__ uint32_t lstart[kBins], gbase[kBins];
    __shared__ Key lkeys[kTile];
    __shared__ uint32_t lvals[kTile];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    for (int v = 0; v < kWaves; ++v) cnt[v][threadIdx.x] = 0;
    // first slot of digit threadIdx.x: exclusive scan of the row totals
    const uint32_t dbase = block_excl_scan(rowtot[threadIdx.x], wsum);
    const int64_t tile0 = blockIdx.x * (int64_t)kTile;
    const int64_t chunk = tile0 + (int64_t)w * (kSteps * kWave);
    for (int t = 0; t < kSteps; ++t) {
        const int64_t idx = chunk + t * kWave + lane;
        if (idx < n) atomicAdd(&cnt[w][digit_of(keys_in[idx], shift)], 1u);
    }
    __syncthreads();
    uint32_t tile_count = 0;
    {
        const uint32_t g0 = dbase + offs[(int64_t)threadIdx.x * tiles + blockIdx.x];
        gbase[threadIdx.x] = g0;
        uint32_t run = g0;
        for (int v = 0; v < kWaves; ++v) {
            base[v][threadIdx.x] = run;
            run += cnt[v][threadIdx.x];
        }
        tile_count = run - g0;
    }
    // where each digit's pairs start in the tile's digit-ordered LDS copy
    lstart[threadIdx.x] = block_excl_scan(tile_count, wsum);
    __syncthreads();
    // rank every pair (its global slot), and place it at the same offset in
    // the LDS copy: lanes holding the same digit are found with eight
    // ballots, a lane's slot is the digit's running offset plus the number of
    // such lanes below it, and the lowest of them advances the offset
    const unsigned long long below = (1ull << lane) - 1ull;
    for (int t = 0; t < kSteps; ++t) {
        const int64_t idx = chunk + t * kWave + lane;
        const bool valid = idx < n;
        const Key key = valid ? keys_in[idx] : Key(0);
        const uint32_t val = !valid ? 0u : vals_in ? vals_in[idx] : (uint32_t)idx;
        const int d = digit_of(key, shift);
        unsigned long long match = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1;
            const unsigned long long m = __ballot(bit);
            match &= bit ? m : ~m;
        }
        const uint32_t lower = (uint32_t)__popcll(match & below);
        const uint32_t slot = base[w][d] + lower;   // every lane reads before the update below
        if (valid) {
            const uint32_t local = lstart[d] + (slot - gbase[d]);
            lkeys[local] = key;
            lvals[local] = val;
        }
        if (valid && lower == 0) base[w][d] += (uint32_t)__popcll(match);
        __builtin_amdgcn_wave_barrier();  // the next step's reads stay after this update
    }
    __syncthreads();
    // write out in the LDS order: runs of one digit go to consecutive slots
    const int count = (int)min((int64_t)kTile, n - tile0);
    for (int j = threadIdx.x; j < count; j += kBlock) {
        const Key key = lkeys[j];
        const int d = digit_of(key, shift);
        const uint32_t g = gbase[d] + ((uint32_t)j - lstart[d]);
        keys_out[g] = key;
        vals_out[g] = lvals[j];
    }
}

}  // namespace

size_t radix_hist_entries(int64_t n) {
    return (size_t)kBins * (size_t)((n + kTile - 1) / kTile) + kBins;
}

namespace {

template <typename Key>
void sort_passes(const Key* keys, Key* keys_a, uint32_t* vals_a, Key* keys_b, uint32_t* vals_b, uint32_t* hist,
                 int64_t n, unsigned digit_mask, hipStream_t st, const Key** out_keys, const uint32_t** out_vals) {
    constexpr int kDigits = (int)sizeof(Key);
    const int64_t tiles = (n + kTile - 1) / kTile;
    // one pass at least, so that the positions are written out even when
    // every digit is the same in all keys (that pass keeps the order)
    digit_mask &= (1u << kDigits) - 1u;
    if (!digit_mask) digit_mask = 1u;
    const Key* kin = keys;
    const uint32_t* vin = nullptr;   // first pass: the values are the positions
    Key* kout = keys_a;
    uint32_t* vout = vals_a;
    Key* knext = keys_b;
    uint32_t* vnext = vals_b;
    uint32_t* rowtot = hist + (size_t)kBins * tiles;
    for (int d = 0; d < kDigits; ++d) {
        if (!((digit_mask >> d) & 1u)) continue;
        const int shift = 8 * d;
        hipLaunchKernelGGL(k_digit_hist<Key>, dim3((unsigned)tiles), dim3(kBlock), 0, st, kin, n, shift, hist,
                           tiles);
        hipLaunchKernelGGL(k_scan_rows, dim3(kBins / kScanWaves), dim3(kScanWaves * kWave), 0, st, hist, tiles,
                           rowtot);
        hipLaunchKernelGGL(k_digit_scatter<Key>, dim3((unsigned)tiles), dim3(kBlock), 0, st, kin, vin, kout, vout,
                           n, shift, hist, tiles, rowtot);
        kin = kout;
        vin = vout;
        std::swap(kout, knext);
        std::swap(vout, vnext);
    }
    *out_keys = kin;
    *out_vals = vin;
}

}  // namespace

lrqo_status radix_sort_pairs(const unsigned long long* keys, unsigned long long* keys_a, uint32_t* vals_a,
                             unsigned long long* keys_b, uint32_t* vals_b, uint32_t* hist, int64_t n,
                             unsigned digit_mask, hipStream_t st, SortedPairs* out) {
    sort_passes(keys, keys_a, vals_a, keys_b, vals_b, hist, n, digit_mask, st, &out->keys, &out->vals);
    LRQO_HIP(hipGetLastError());
    return LRQO_OK;
}

lrqo_status radix_sort_pairs32(const uint32_t* keys, uint32_t* keys_a, uint32_t* vals_a, uint32_t* keys_b,
                               uint32_t* vals_b, uint32_t* hist, int64_t n, unsigned digit_mask, hipStream_t st,
                               SortedPairs32* out) {
    sort_passes(keys, keys_a, vals_a, keys_b, vals_b, hist, n, digit_mask, st, &out->keys, &out->vals);
    LRQO_HIP(hipGetLastError());
    return LRQO_OK;
}

}  // namespace lrqo
